// k_ragged.hip -- ragged batches: host-side plans and persistent kernels.
//
// A ragged batch holds pairs of uneven limb counts.  The plan sorts the pairs by
// work (largest first) once on the host, splits them by multiplication form and
// uploads the lists.  Each form runs as one persistent launch sized to the
// resident wave count; wave k takes items k, k + W, k + 2W, ... of the sorted
// list, so every wave gets a similar mix of large and small pairs without any
// shared counter (same-address atomics serialise at about 10-30 ns each on this
// part, which would cost more than the products of a 2^16-pair batch).  Mad items
// of at most 32 product limbs whose shorter operands have the same length are
// coupled by the plan and run two to a wave, one per half, before the other items.
// The launches hold no state between calls, so they can be captured in a HIP graph
// and replayed.
#include "bn_mul_dev.h"

#include <algorithm>

namespace {

constexpr int RAGGED_LDS_U64 = SmallMfma<2>::LDS_U64;

// Couples of small mad items (mul_item_mad_pair), wave k taking couples k, k + W, ...
__device__ __forceinline__ void run_pairs(const RItem *__restrict__ pairs, u32 npaired, u64 *__restrict__ r,
                                          const u64 *__restrict__ a, const u64 *__restrict__ b) {
    const u32 W = gridDim.x * 4;
    for (u32 c = blockIdx.x * 4 + (u32)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6); 2 * c < npaired; c += W)
        mul_item_mad_pair(pairs[2 * c], pairs[2 * c + 1], a, b, r);
}

__global__ __launch_bounds__(256) void k_mul_ragged_mad(const RItem *__restrict__ items, u32 nitems,
                                                        u64 *__restrict__ r, const u64 *__restrict__ a,
                                                        const u64 *__restrict__ b, const RItem *__restrict__ pairs,
                                                        u32 npaired) {
    run_pairs(pairs, npaired, r, a, b);
    const u32 W = gridDim.x * 4;
    // wave-uniform item index: descriptors, sizes and loop bounds stay scalar
    u32 it = blockIdx.x * 4 + (u32)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (it >= nitems) return;
    RItem next = items[it];
    for (; it < nitems; it += W) {
        const RItem m = next;
        if (it + W < nitems) next = items[it + W];  // the next descriptor loads during this product
        const u64 *pa = a + m.a_off;
        const u64 *pb = b + m.b_off;
        u64 *pr = r + m.r_off;
        const u32 P = m.na + m.nb;
        if (P <= 64)
            mul_item_mad<1>(pa, m.na, pb, m.nb, pr);
        else if (P <= 128)
            mul_item_mad<2>(pa, m.na, pb, m.nb, pr);
        else
            mul_item_mad<4>(pa, m.na, pb, m.nb, pr);
    }
}

// Bounded to at least six waves per SIMD, the compiler keeps the accumulators in
// ordinary registers (63 in all, no spills) instead of 64 + 32 accumulation registers,
// and the kernel runs at eight waves per SIMD instead of five: C4's MFMA form 73 -> 68 us.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_mul_ragged_mfma(const RItem *__restrict__ items, u32 nitems,
                                                         u64 *__restrict__ r, const u64 *__restrict__ a,
                                                         const u64 *__restrict__ b) {
    __shared__ u64 lds[4 * RAGGED_LDS_U64];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const u32 W = gridDim.x * 4;
    for (u32 it = blockIdx.x * 4 + w; it < nitems; it += W) {
        const RItem m = items[it];
        if (m.na + m.nb <= 128)
            mul_item_mfma_small<1>(a + m.a_off, m.na, b + m.b_off, m.nb, r + m.r_off, lds + w * RAGGED_LDS_U64);
        else
            mul_item_mfma_small<2>(a + m.a_off, m.na, b + m.b_off, m.nb, r + m.r_off, lds + w * RAGGED_LDS_U64);
        wave_sync();
    }
}

// Both forms in one persistent launch (a batch with mad and MFMA items): the item's
// form picks the path, wave-uniformly.  One launch instead of two back to back lets
// the waves that finish their share of one form go on with the other, so the two
// tails overlap.  The mad path takes products of at most 128 limbs (the plan gives
// automatic items of 129-256 limbs the MFMA form): without the four-step mad path the
// kernel fits 64 registers and runs at eight waves per SIMD without spills (with it:
// six waves and 80 bytes per lane spilled; C4 7% slower).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_mul_ragged_mixed(const RItem *__restrict__ items, u32 nitems,
                                                          u64 *__restrict__ r, const u64 *__restrict__ a,
                                                          const u64 *__restrict__ b, const RItem *__restrict__ pairs,
                                                          u32 npaired) {
    __shared__ u64 lds[4 * RAGGED_LDS_U64];
    run_pairs(pairs, npaired, r, a, b);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const u32 W = gridDim.x * 4;
    for (u32 it = blockIdx.x * 4 + w; it < nitems; it += W) {
        const RItem m = items[it];
        const u64 *pa = a + m.a_off;
        const u64 *pb = b + m.b_off;
        u64 *pr = r + m.r_off;
        const u32 P = m.na + m.nb;
        if (m.form == BN_MUL_MFMA || P > 128) {  // (the plan leaves no mad item above 128 limbs here)
            if (P <= 128)  // one column block: half the digit conversion and carry pass
                mul_item_mfma_small<1>(pa, m.na, pb, m.nb, pr, lds + w * RAGGED_LDS_U64);
            else
                mul_item_mfma_small<2>(pa, m.na, pb, m.nb, pr, lds + w * RAGGED_LDS_U64);
            wave_sync();
        } else if (P <= 64) {
            mul_item_mad<1>(pa, m.na, pb, m.nb, pr);
        } else {
            mul_item_mad<2>(pa, m.na, pb, m.nb, pr);
        }
    }
}

// Ragged add: one wave per pair, walking the pair in rows of 128 limbs (lane l
// holds limbs 2l, 2l+1 of a row); the carry crosses rows through the wave-uniform
// carry-out of the row's ballot scan.
template <bool SUB>
__global__ __launch_bounds__(256) void k_add_ragged(const RItem *__restrict__ items, u32 nitems,
                                                    u64 *__restrict__ r, const u64 *__restrict__ a,
                                                    const u64 *__restrict__ b, u64 *__restrict__ carry) {
    const int lane = threadIdx.x & 63;
    const u32 W = gridDim.x * 4;
    for (u32 it = blockIdx.x * 4 + (u32)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6); it < nitems; it += W) {
        const RItem m = items[it];
        const u64 n = m.na;
        const u64 *pa = a + m.a_off, *pb = b + m.b_off;
        u64 *pr = r + m.r_off;
        u64 c = 0;
        for (u64 base = 0; base < n; base += 128) {
            const u64 i0 = base + 2 * (u64)lane, i1 = i0 + 1;
            const bool v0 = i0 < n, v1 = i1 < n;
            const u64 x0 = v0 ? pa[i0] : 0, y0 = v0 ? pb[i0] : 0;
            const u64 x1 = v1 ? pa[i1] : 0, y1 = v1 ? pb[i1] : 0;
            const u64 s0 = SUB ? x0 - y0 : x0 + y0;
            const u64 s1 = SUB ? x1 - y1 : x1 + y1;
            const bool g0 = v0 && (SUB ? x0 < y0 : s0 < x0);
            const bool g1 = v1 && (SUB ? x1 < y1 : s1 < x1);
            const bool p0 = v0 && (SUB ? s0 == 0 : s0 == ~0ull);
            const bool p1 = v1 && (SUB ? s1 == 0 : s1 == ~0ull);
            const u64 Gm = __ballot(g1 || (p1 && g0));
            const u64 Pm = __ballot(p0 && p1);
            const u64 X = (Gm << 1) | c;
            const u64 T = X + Pm;
            const u64 C = T ^ Pm;
            const bool ci0 = (C >> lane) & 1ull;
            const bool co0 = g0 || (p0 && ci0);
            const bool co1 = g1 || (p1 && co0);
            if (v0) pr[i0] = SUB ? s0 - (u64)ci0 : s0 + (u64)ci0;
            if (v1) pr[i1] = SUB ? s1 - (u64)co0 : s1 + (u64)co0;
            if (carry && v0 && i0 == n - 1) carry[m.index] = co0;
            if (carry && v1 && i1 == n - 1) carry[m.index] = co1;
            c = (Gm >> 63) | ((Pm >> 63) & (C >> 63));
        }
        if (carry && n == 0 && lane == 0) carry[m.index] = 0;
    }
}

// Persistent grid: exactly as many 4-wave workgroups as stay resident at once (the
// runtime's occupancy for the kernel: registers and LDS decide it), but no more than
// the items need.  A grid larger than the resident set would run its last
// workgroups after the first ones finish, doubling the time of a balanced batch.
template <auto KERNEL>
u32 persistent_blocks(const bn_ctx *ctx, u32 nitems) {
    static const int per_cu = [] {  // one query per kernel (every device here is gfx950)
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, KERNEL, 256, 0) != hipSuccess || v < 1) v = 1;
        return v;
    }();
    const u32 want = (u32)std::max(1, ctx->num_cu) * (u32)per_cu;
    const u32 need = (nitems + 3) / 4;
    return std::max<u32>(1, std::min(want, need));
}

// a range of n limbs at limb offset off stays below 2^60 limbs (2^63 bytes), so the
// kernels' byte addresses cannot wrap
bool span_ok(u64 off, u64 n) { return off <= (1ull << 60) - n; }

bn_status upload_plan(bn_ctx *ctx, bn_plan *pl, std::vector<RItem> &small) {
    pl->nsmall = (u32)small.size();
    if (hipSetDevice(ctx->device) != hipSuccess) return BN_EHIP;
    if (!small.empty()) {
        if (hipMalloc(&pl->d_items, small.size() * sizeof(RItem)) != hipSuccess) return BN_ENOMEM;
        if (hipMemcpy(pl->d_items, small.data(), small.size() * sizeof(RItem), hipMemcpyHostToDevice) != hipSuccess)
            return BN_EHIP;
    }
    return BN_OK;
}

}  // namespace

bn_status plan_mul_ragged(bn_ctx *ctx, const bn_pair *pairs, size_t npairs, int form, bn_plan **out) {
    if (npairs > 0xffffffffull) return BN_ERANGE;
    bn_plan *pl = new bn_plan();
    pl->op = 0;
    pl->device = ctx->device;
    pl->npairs = npairs;
    std::vector<RItem> small;
    small.reserve(npairs);
    for (size_t i = 0; i < npairs; ++i) {
        const bn_pair &p = pairs[i];
        if (p.na == 0 || p.nb == 0 || p.na > (1u << 20) || p.nb > (1u << 20) || !span_ok(p.a_off, p.na) ||
            !span_ok(p.b_off, p.nb) || !span_ok(p.r_off, (u64)p.na + p.nb)) {
            delete pl;
            return BN_ERANGE;
        }
        RItem it{p.a_off, p.b_off, p.r_off, p.na, p.nb, 0, (u32)i};
        it.form = (u32)mul_pick_form(ctx, p.na, p.nb, form);
        // automatic one-wave items of 129-256 limbs take the MFMA form: the kernel that
        // runs both forms in one launch has no mad path for them (see k_mul_ragged_mixed)
        if (form == BN_MUL_AUTO && (u64)p.na + p.nb > 128 && (u64)p.na + p.nb <= 256) it.form = BN_MUL_MFMA;
        (it.form == BN_MUL_MFMA ? pl->nmfma : pl->nmad)++;
        pl->work += (u64)p.na * p.nb;
        if ((u64)p.na + p.nb <= 256) {
            small.push_back(it);
        } else {
            pl->large.push_back(it);
            pl->ws.work = std::max(pl->ws.work, mul_workspace_bytes(ctx, it.na, it.nb, 1, (int)it.form));
            pl->ws.status = std::max(pl->ws.status, mul_status_bytes(ctx, it.na, it.nb, 1, (int)it.form));
        }
    }
    // mad items first, then MFMA items; each group by work, largest first
    std::stable_sort(small.begin(), small.end(), [](const RItem &x, const RItem &y) {
        if (x.form != y.form) return x.form == BN_MUL_MAD;
        return (u64)x.na * x.nb > (u64)y.na * y.nb;
    });
    // Mad items of at most 32 product limbs go two to a wave when their shorter operands
    // have the same length (the couple then runs the same digit steps): couples by
    // shorter length, largest first; an item left without a partner stays single.
    std::vector<RItem> couples;
    if (ctx->tune.ragged_pair) {
        std::vector<RItem> rest;
        rest.reserve(small.size());
        std::vector<RItem> cand;
        for (const RItem &x : small) {
            if (x.form == BN_MUL_MAD && (u64)x.na + x.nb <= 32) cand.push_back(x);
            else rest.push_back(x);
        }
        std::stable_sort(cand.begin(), cand.end(),
                         [](const RItem &x, const RItem &y) { return std::min(x.na, x.nb) > std::min(y.na, y.nb); });
        for (size_t i = 0; i < cand.size();) {
            if (i + 1 < cand.size() && std::min(cand[i].na, cand[i].nb) == std::min(cand[i + 1].na, cand[i + 1].nb)) {
                couples.push_back(cand[i]);
                couples.push_back(cand[i + 1]);
                i += 2;
            } else {
                rest.push_back(cand[i]);
                i += 1;
            }
        }
        if (!couples.empty()) {
            small.swap(rest);
            std::stable_sort(small.begin(), small.end(), [](const RItem &x, const RItem &y) {
                if (x.form != y.form) return x.form == BN_MUL_MAD;
                return (u64)x.na * x.nb > (u64)y.na * y.nb;
            });
        }
    }
    pl->nsmall_mad = (u32)std::count_if(small.begin(), small.end(), [](const RItem &x) { return x.form == BN_MUL_MAD; });
    pl->npaired = (u32)couples.size();
    if (!couples.empty()) {
        if (hipSetDevice(ctx->device) != hipSuccess) {
            bn_plan_destroy(pl);
            return BN_EHIP;
        }
        if (hipMalloc(&pl->d_pairs, couples.size() * sizeof(RItem)) != hipSuccess) {
            bn_plan_destroy(pl);
            return BN_ENOMEM;
        }
        if (hipMemcpy(pl->d_pairs, couples.data(), couples.size() * sizeof(RItem), hipMemcpyHostToDevice) != hipSuccess) {
            bn_plan_destroy(pl);
            return BN_EHIP;
        }
    }
    bn_status st = upload_plan(ctx, pl, small);
    if (st != BN_OK) {
        bn_plan_destroy(pl);
        return st;
    }
    *out = pl;
    return BN_OK;
}

bn_status plan_add_ragged(bn_ctx *ctx, const bn_pair *pairs, size_t npairs, bn_plan **out) {
    if (npairs > 0xffffffffull) return BN_ERANGE;
    bn_plan *pl = new bn_plan();
    pl->op = 1;
    pl->device = ctx->device;
    pl->npairs = npairs;
    std::vector<RItem> items;
    items.reserve(npairs);
    for (size_t i = 0; i < npairs; ++i) {
        const bn_pair &p = pairs[i];
        if ((u64)p.na > BN_MAX_LIMBS || !span_ok(p.a_off, p.na) || !span_ok(p.b_off, p.na) || !span_ok(p.r_off, p.na)) {
            delete pl;
            return BN_ERANGE;
        }
        items.push_back(RItem{p.a_off, p.b_off, p.r_off, p.na, p.na, 0, (u32)i});
        pl->work += p.na;
    }
    std::stable_sort(items.begin(), items.end(), [](const RItem &x, const RItem &y) { return x.na > y.na; });
    bn_status st = upload_plan(ctx, pl, items);
    if (st != BN_OK) {
        bn_plan_destroy(pl);
        return st;
    }
    *out = pl;
    return BN_OK;
}

bn_status launch_mul_ragged(bn_ctx *ctx, const bn_plan *pl, u64 *r, const u64 *a, const u64 *b, hipStream_t s) {
    const u32 nmad = pl->nsmall_mad, nmfma = pl->nsmall - pl->nsmall_mad;
    // work units for the grid size: a couple of paired items counts once
    const u32 units = pl->nsmall + pl->npaired / 2;
    if (nmfma && (nmad || pl->npaired)) {
        hipLaunchKernelGGL(k_mul_ragged_mixed, dim3(persistent_blocks<k_mul_ragged_mixed>(ctx, units)), dim3(256), 0,
                           s, pl->d_items, pl->nsmall, r, a, b, pl->d_pairs, pl->npaired);
        bn_status st = bn_launch_status();
        if (st != BN_OK) return st;
    } else if (nmad || pl->npaired) {
        hipLaunchKernelGGL(k_mul_ragged_mad, dim3(persistent_blocks<k_mul_ragged_mad>(ctx, units)), dim3(256), 0, s, pl->d_items, nmad,
                           r, a, b, pl->d_pairs, pl->npaired);
        bn_status st = bn_launch_status();
        if (st != BN_OK) return st;
    } else if (nmfma) {
        hipLaunchKernelGGL(k_mul_ragged_mfma, dim3(persistent_blocks<k_mul_ragged_mfma>(ctx, nmfma)), dim3(256), 0, s,
                           pl->d_items + nmad, nmfma, r, a, b);
        bn_status st = bn_launch_status();
        if (st != BN_OK) return st;
    }
    for (const RItem &it : pl->large) {
        bn_status st = launch_mul_batch(ctx, r + it.r_off, a + it.a_off, b + it.b_off, it.na, it.nb, 1, (int)it.form, s);
        if (st != BN_OK) return st;
    }
    return BN_OK;
}

bn_status launch_add_ragged(bn_ctx *ctx, const bn_plan *pl, u64 *r, const u64 *a, const u64 *b, u64 *carry,
                            hipStream_t s) {
    if (!pl->nsmall) return BN_OK;
    hipLaunchKernelGGL(k_add_ragged<false>, dim3(persistent_blocks<k_add_ragged<false>>(ctx, pl->nsmall)), dim3(256), 0, s,
                       pl->d_items, pl->nsmall, r, a, b, carry);
    return bn_launch_status();
}
