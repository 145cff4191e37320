// k_karatsuba.hip -- Karatsuba levels above the batched schoolbook kernels.
//
// One level (App. A, Alg. 4, the paper's libraries' step above the base case): with
// X = 2^(64 k) and A = A_H X + A_L, B = B_H X + B_L (k = ceil(m / 2) limbs; when m is
// odd the high halves have k - 1 limbs and are zero-extended to k, the padding of the
// shorter operand that the proof of Theorem 2 uses),
//     P1 = A_H B_H,  P0 = A_L B_L,  PD = |A_H - A_L| |B_H - B_L|,
//     P2 = s_x s_y PD with s_x, s_y the signs of A_H - A_L and B_H - B_L,
//     A B = P1 X^2 + (P1 + P0 - P2) X + P0.
// The top level may take operands of different lengths na, nb: both are zero-extended
// to m = max(na, nb) on the fly (the split reads them with their own strides), and the
// product keeps exactly na + nb limbs.
// The GPU form is breadth-first: every level turns a batch of N products of m limbs
// into one batch of 3N products of k limbs (the split), the bottom batch goes to the
// schoolbook kernels in one launch, and the levels are combined bottom-up.  Batches
// are stored by kind: children [0, N) are the (A_L, B_L) halves, [N, 2N) the
// (A_H, B_H) halves and [2N, 3N) the absolute differences, so every add/sub of the
// split and of the combine is a uniform batch over contiguous arrays.  The split is one
// pass that copies the halves and finds, piece by piece, the highest limb where they
// differ, then one subtraction scan (both operands' differences in one launch) that
// takes lo - hi or hi - lo per pair from those keys.  The combine is one carry scan
// that forms every limb of P0 + P1 X^2 + (P0 + P1 - P2) X from the child products
// itself (the scan's EXT_COMB variant, same biased terms).
#include "bn_internal.h"

#include <algorithm>
#include <vector>

namespace {

// Operands of a split: operand q of a side is x + stride q, its limbs past `len` read
// as zero (len <= stride; at the top level len and stride are the caller's na or nb,
// below it both are the level's m).
struct SplitSrc {
    const u64 *x;
    u64 len, stride;
};
__device__ __forceinline__ u64 src_limb(const SplitSrc &s, u64 q, u64 i) {
    return i < s.len ? s.x[s.stride * q + i] : 0ull;
}

// The children lo = x[q][0, k) and hi = x[q][k, 2k) of the N operands of a and of b
// (copies, to d_x and d_x + N k), and the signs neg_x[q] = [hi < lo] in two steps with a
// fixed amount of work whatever the data (equal halves, as in all-ones or zero
// operands, leave nothing to stop early on): one workgroup per piece of SIGN_PIECE
// limbs of an operand copies them and writes key = (i + 1) * 2 + [hi_i < lo_i] for the
// highest limb i where the halves differ (0: no difference); the split scan then takes
// the largest key of an operand's pieces as its sign.
constexpr u64 SIGN_PIECE = 2048;  // 256 threads x 8 limbs

__global__ __launch_bounds__(256) void k_split_halves(SplitSrc a, SplitSrc b, u64 N, u64 k, u64 npieces,
                                                      u64 *__restrict__ da, u64 *__restrict__ db,
                                                      u64 *__restrict__ keys) {
    __shared__ u64 sh[4];
    const u64 seg = blockIdx.x / npieces, piece = blockIdx.x - seg * npieces;
    const bool is_b = seg >= N;
    const SplitSrc &x = is_b ? b : a;
    u64 *d = is_b ? db : da;
    const u64 q = is_b ? seg - N : seg;
    const u64 base = piece * SIGN_PIECE;
    u64 lo[8], hi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const u64 i = base + 256 * u + threadIdx.x;
        lo[u] = i < k ? src_limb(x, q, i) : 0;
        hi[u] = i < k ? src_limb(x, q, k + i) : 0;
    }
    u64 key = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const u64 i = base + 256 * u + threadIdx.x;
        if (i < k) {
            d[q * k + i] = lo[u];
            d[N * k + q * k + i] = hi[u];
        }
        if (hi[u] != lo[u]) key = std::max(key, ((i + 1) << 1) | (hi[u] < lo[u] ? 1u : 0u));
    }
    for (int off = 32; off > 0; off >>= 1) key = std::max(key, (u64)__shfl_xor(key, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) keys[blockIdx.x] = std::max(std::max(sh[0], sh[1]), std::max(sh[2], sh[3]));
}

// Workspace layout of a run (u64 offsets).
struct KLevel {
    u64 N, m;        // products and operand limbs at this level (m_0 = max(na, nb), m_(l+1) = ceil(m_l / 2))
    u64 out;         // result limbs per product: 2m, na + nb at the top
    u64 A, B, R;     // operands (N x m each) and products (N x 2m) of this level (level >= 1)
    u64 negA, negB;  // signs of A_H - A_L and B_H - B_L of this level's split (N each, negB = negA + N)
};
struct KPlan {
    std::vector<KLevel> lv;  // 0 .. levels
    u64 keys;                // split: per-piece sign keys (2 N_l pieces_l, largest level)
    u64 total;               // u64 words
};

KPlan karatsuba_plan(u64 na, u64 nb, u64 npairs, int levels) {
    KPlan p{};
    u64 off = 0;
    auto take = [&](u64 words) {
        const u64 o = off;
        off += (words + 31) & ~31ull;  // 256-byte alignment
        return o;
    };
    p.lv.resize(levels + 1);
    u64 N = npairs, m = std::max(na, nb), maxkeys = 0;
    for (int l = 0; l <= levels; ++l) {
        KLevel &L = p.lv[l];
        L.N = N;
        L.m = m;
        L.out = l == 0 ? na + nb : 2 * m;
        if (l > 0) {
            L.A = take(N * m);
            L.B = take(N * m);
            L.R = take(N * 2 * m);
        }
        const u64 k = (m + 1) / 2;
        if (l < levels) {
            L.negA = take(2 * N);
            L.negB = L.negA + N;
            maxkeys = std::max(maxkeys, 2 * N * ((k + SIGN_PIECE - 1) / SIGN_PIECE));
        }
        N *= 3;
        m = k;
    }
    p.keys = take(maxkeys);
    p.total = off;
    return p;
}

}  // namespace

size_t karatsuba_workspace_bytes(u64 na, u64 nb, u64 npairs, int levels) {
    return (size_t)karatsuba_plan(na, nb, npairs, levels).total * sizeof(u64);
}

// Every buffer a run touches: its own arrays, the bottom batch's multiplication
// workspace, and status words for the largest of its scans (splits: N_l pairs of k
// limbs; combines: N_l pairs of out_l; the bottom batch's own scans).
WsNeed karatsuba_need(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs, int levels, int form) {
    WsNeed w;
    if (npairs == 0 || na == 0 || nb == 0 || levels < 0) return w;
    if (levels == 0) {
        w.work = mul_workspace_bytes(ctx, na, nb, npairs, form);
        w.status = mul_status_bytes(ctx, na, nb, npairs, form);
        return w;
    }
    const KPlan p = karatsuba_plan(na, nb, npairs, levels);
    w.kwork = (size_t)p.total * sizeof(u64);
    for (int l = 0; l < levels; ++l) {
        const u64 N = p.lv[l].N, k = (p.lv[l].m + 1) / 2, out = p.lv[l].out;
        w.status = std::max({w.status, flat_scan_ext_status_bytes(k, 2 * N * k), flat_scan_ext_status_bytes(k, N * k),
                             flat_scan_ext_status_bytes(out, N * out)});
    }
    const KLevel &Bt = p.lv[levels];
    w.work = mul_workspace_bytes(ctx, Bt.m, Bt.m, Bt.N, form);
    w.status = std::max(w.status, mul_status_bytes(ctx, Bt.m, Bt.m, Bt.N, form));
    return w;
}

bn_status launch_mul_karatsuba(bn_ctx *ctx, u64 *r, const u64 *a, u64 na, const u64 *b, u64 nb, u64 npairs,
                               int levels, int form, hipStream_t s) {
    if (npairs == 0) return BN_OK;
    if (levels == 0 || na == 0 || nb == 0) return launch_mul_batch(ctx, r, a, b, na, nb, npairs, form, s);
    const KPlan p = karatsuba_plan(na, nb, npairs, levels);
    bn_status st = bn_ensure(ctx, ctx->kwork, p.total * sizeof(u64), s);
    if (st != BN_OK) return st;
    u64 *w = static_cast<u64 *>(ctx->kwork.ptr);
    // ---- split, top-down ----
    for (int l = 0; l < levels; ++l) {
        const KLevel &P = p.lv[l], &C = p.lv[l + 1];
        const u64 N = P.N, k = C.m;
        const SplitSrc pa = l == 0 ? SplitSrc{a, na, na} : SplitSrc{w + P.A, P.m, P.m};
        const SplitSrc pb = l == 0 ? SplitSrc{b, nb, nb} : SplitSrc{w + P.B, P.m, P.m};
        u64 *ca = w + C.A, *cb = w + C.B;  // [lows | highs | |differences|], N x k each
        const u64 Nk = N * k;
        const u64 npieces = (k + SIGN_PIECE - 1) / SIGN_PIECE;
        if (2 * N * npieces > 0x7fffffffull) return BN_ERANGE;
        hipLaunchKernelGGL(k_split_halves, dim3((u32)(2 * N * npieces)), dim3(256), 0, s, pa, pb, N, k, npieces, ca, cb,
                           w + p.keys);
        if ((st = bn_launch_status()) != BN_OK) return st;
        // |hi - lo| into the children [2N, 3N) of both sides: one two-part subtraction that
        // takes lo - hi for the pairs whose keys say hi < lo, and records those signs
        // (negA, then negB) for the combine
        ScanPart2 bside;
        bside.r = cb + 2 * Nk;
        bside.a = cb + Nk;
        bside.b = cb;
        bside.npairs = N;
        ScanSwap sw;
        sw.keys = w + p.keys;
        sw.npieces = npieces;
        sw.neg = w + P.negA;
        if ((st = launch_flat_scan_mem(ctx, true, ca + 2 * Nk, ca + Nk, ca, k, N, nullptr, false, 0, nullptr, s, nullptr,
                                       -1, nullptr, &bside, &sw)) != BN_OK)
            return st;
    }
    // ---- the bottom batch on the schoolbook kernels ----
    const KLevel &Bt = p.lv[levels];
    if ((st = launch_mul_batch(ctx, w + Bt.R, w + Bt.A, w + Bt.B, Bt.m, Bt.m, Bt.N, form, s)) != BN_OK) return st;
    // ---- combine, bottom-up ----
    for (int l = levels - 1; l >= 0; --l) {
        const KLevel &P = p.lv[l], &C = p.lv[l + 1];
        const u64 N = P.N, k = C.m, twok = 2 * k;
        const u64 *P0 = w + C.R, *P1 = P0 + N * twok, *PD = P1 + N * twok;
        u64 *out = l == 0 ? r : w + P.R;
        // out = P0 + P1 X^2 + (P1 + P0 - P2) X, its terms formed inside one carry scan
        // (modulo X^out: the product fits out limbs, so no carry leaves the top)
        ScanComb cm;
        cm.P0 = P0;
        cm.P1 = P1;
        cm.PD = PD;
        cm.negA = w + P.negA;
        cm.negB = w + P.negB;
        cm.k = k;
        if ((st = launch_flat_scan_comb(ctx, out, cm, P.out, N, s)) != BN_OK) return st;
    }
    return BN_OK;
}
