// k_karatsuba.hip -- Karatsuba levels above the batched schoolbook kernels.
//
// One level (App. A, Alg. 4, the paper's libraries' step above the base case): with
// X = 2^(64 k) and A = A_H X + A_L, B = B_H X + B_L (k = m / 2 limbs),
//     P1 = A_H B_H,  P0 = A_L B_L,  PD = |A_H - A_L| |B_H - B_L|,
//     P2 = s_x s_y PD with s_x, s_y the signs of A_H - A_L and B_H - B_L,
//     A B = P1 X^2 + (P1 + P0 - P2) X + P0.
// The GPU form is breadth-first: every level turns a batch of N products of m limbs
// into one batch of 3N products of k limbs (the split), the bottom batch goes to the
// schoolbook kernels in one launch, and the levels are combined bottom-up.  Batches
// are stored by kind: children [0, N) are the (A_L, B_L) halves, [N, 2N) the
// (A_H, B_H) halves and [2N, 3N) the absolute differences, so every add/sub of the
// split and of the combine is a uniform batch over contiguous arrays and runs on the
// flat scan kernel; the few copies in between are plain streaming kernels.
#include "bn_internal.h"

#include <algorithm>
#include <vector>

namespace {

// For both operands x in {a, b}: lo_x[q] = x[q][0, k), hi_x[q] = x[q][k, 2k), the two
// halves of N operands of 2k limbs (the halves go to dst_x and dst_x + N k).
__global__ void k_split_halves(const u64 *__restrict__ a, const u64 *__restrict__ b, u64 N, u64 k,
                               u64 *__restrict__ da, u64 *__restrict__ db) {
    const u64 total = N * k;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 q = idx / k, i = idx - q * k;
        da[idx] = a[2 * k * q + i];
        da[total + idx] = a[2 * k * q + k + i];
        db[idx] = b[2 * k * q + i];
        db[total + idx] = b[2 * k * q + k + i];
    }
}

// For both operands: dst_x[q] = neg_x[q] ? neg-difference : pos-difference, i.e.
// |hi - lo| from hi - lo and lo - hi (k limbs each), neg_x[q] the borrow of hi - lo.
__global__ void k_select_abs(u64 *__restrict__ dst_a, u64 *__restrict__ dst_b, const u64 *__restrict__ pos,
                             const u64 *__restrict__ negd, const u64 *__restrict__ neg_a,
                             const u64 *__restrict__ neg_b, u64 N, u64 k) {
    const u64 total = N * k;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 q = idx / k;
        dst_a[idx] = neg_a[q] ? negd[idx] : pos[idx];
        dst_b[idx] = neg_b[q] ? negd[total + idx] : pos[total + idx];
    }
}

// Operands of the final addition of a level, per product q (4k limbs each):
//   out[q] = P0 + P1 X^2              (the two halves side by side),
//   Y[q]   = (P1 + P0 - P2) X         (2k limbs and a top limb at k .. 3k).
// With S = P0 + P1 (carry cS), the middle term is S - PD (borrow bM) when s_x s_y > 0
// and S + PD (carry cP) otherwise; it is never negative (it equals A_H B_L + A_L B_H).
__global__ void k_assemble(u64 *__restrict__ out, u64 *__restrict__ Y, const u64 *__restrict__ P0,
                           const u64 *__restrict__ P1, const u64 *__restrict__ Tplus, const u64 *__restrict__ Tminus,
                           const u64 *__restrict__ cS, const u64 *__restrict__ cP, const u64 *__restrict__ bM,
                           const u64 *__restrict__ negA, const u64 *__restrict__ negB, u64 N, u64 k) {
    const u64 total = N * 4 * k;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 q = idx / (4 * k), i = idx - q * 4 * k;
        out[idx] = i < 2 * k ? P0[2 * k * q + i] : P1[2 * k * q + i - 2 * k];
        const bool same = negA[q] == negB[q];  // s_x s_y > 0: P2 = +PD
        u64 y = 0;
        if (i >= k && i < 3 * k)
            y = same ? Tminus[2 * k * q + i - k] : Tplus[2 * k * q + i - k];
        else if (i == 3 * k)
            y = same ? cS[q] - bM[q] : cS[q] + cP[q];
        Y[idx] = y;
    }
}

u32 stream_blocks(u64 total) { return (u32)std::max<u64>(1, std::min<u64>((total + 255) / 256, 65536)); }

// Workspace layout of a run (u64 offsets).
struct KLevel {
    u64 N, m;        // products and operand limbs at this level
    u64 A, B, R;     // operands (N x m each) and products (N x 2m) of this level (level >= 1)
    u64 negA, negB;  // borrows of A_H - A_L and B_H - B_L of this level's split (N each)
};
struct KPlan {
    std::vector<KLevel> lv;  // 0 .. levels
    u64 d1, d2;              // hi - lo and lo - hi of a then b (2 N_l k each, largest level)
    u64 S, Tp, Tm, Y;        // combine temporaries (largest level)
    u64 cS, cP, bM;          // combine carries (largest level)
    u64 total;               // u64 words
};

KPlan karatsuba_plan(u64 n, u64 npairs, int levels) {
    KPlan p{};
    u64 off = 0;
    auto take = [&](u64 words) {
        const u64 o = off;
        off += (words + 31) & ~31ull;  // 256-byte alignment
        return o;
    };
    p.lv.resize(levels + 1);
    u64 N = npairs, m = n, maxNk = 0, maxN = 0;
    for (int l = 0; l <= levels; ++l) {
        KLevel &L = p.lv[l];
        L.N = N;
        L.m = m;
        if (l > 0) {
            L.A = take(N * m);
            L.B = take(N * m);
            L.R = take(N * 2 * m);
        }
        if (l < levels) {
            L.negA = take(N);
            L.negB = take(N);
            maxNk = std::max(maxNk, N * (m / 2));
            maxN = std::max(maxN, N);
        }
        N *= 3;
        m /= 2;
    }
    p.d1 = take(2 * maxNk);  // hi - lo of a, then of b
    p.d2 = take(2 * maxNk);  // lo - hi of a, then of b
    p.S = take(2 * maxNk);
    p.Tp = take(2 * maxNk);
    p.Tm = take(2 * maxNk);
    p.Y = take(4 * maxNk);
    p.cS = take(maxN);
    p.cP = take(maxN);
    p.bM = take(maxN);
    p.total = off;
    return p;
}

}  // namespace

size_t karatsuba_workspace_bytes(u64 n, u64 npairs, int levels) {
    return (size_t)karatsuba_plan(n, npairs, levels).total * sizeof(u64);
}

bn_status launch_mul_karatsuba(bn_ctx *ctx, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs, int levels,
                               int form, hipStream_t s) {
    if (npairs == 0 || n == 0) return BN_OK;
    if (levels == 0) return launch_mul_batch(ctx, r, a, b, n, n, npairs, form, s);
    const KPlan p = karatsuba_plan(n, npairs, levels);
    bn_status st = bn_ensure(ctx, ctx->kwork, p.total * sizeof(u64), s);
    if (st != BN_OK) return st;
    u64 *w = static_cast<u64 *>(ctx->kwork.ptr);
    // ---- split, top-down ----
    for (int l = 0; l < levels; ++l) {
        const KLevel &P = p.lv[l], &C = p.lv[l + 1];
        const u64 N = P.N, k = P.m / 2;
        const u64 *pa = l == 0 ? a : w + P.A;
        const u64 *pb = l == 0 ? b : w + P.B;
        u64 *ca = w + C.A, *cb = w + C.B;  // [lows | highs | |differences|], N x k each
        const u64 Nk = N * k;
        hipLaunchKernelGGL(k_split_halves, dim3(stream_blocks(Nk)), dim3(256), 0, s, pa, pb, N, k, ca, cb);
        if ((st = bn_launch_status()) != BN_OK) return st;
        for (int side = 0; side < 2; ++side) {
            u64 *dst = side ? cb : ca;
            // high - low with its borrow (the sign), and low - high
            if ((st = launch_flat_scan(ctx, true, w + p.d1 + side * Nk, dst + Nk, dst, k, N,
                                       w + (side ? P.negB : P.negA), s)) != BN_OK)
                return st;
            if ((st = launch_flat_scan(ctx, true, w + p.d2 + side * Nk, dst, dst + Nk, k, N, nullptr, s)) != BN_OK)
                return st;
        }
        hipLaunchKernelGGL(k_select_abs, dim3(stream_blocks(Nk)), dim3(256), 0, s, ca + 2 * Nk, cb + 2 * Nk, w + p.d1,
                           w + p.d2, w + P.negA, w + P.negB, N, k);
        if ((st = bn_launch_status()) != BN_OK) return st;
    }
    // ---- the bottom batch on the schoolbook kernels ----
    const KLevel &Bt = p.lv[levels];
    if ((st = launch_mul_batch(ctx, w + Bt.R, w + Bt.A, w + Bt.B, Bt.m, Bt.m, Bt.N, form, s)) != BN_OK) return st;
    // ---- combine, bottom-up ----
    for (int l = levels - 1; l >= 0; --l) {
        const KLevel &P = p.lv[l], &C = p.lv[l + 1];
        const u64 N = P.N, k = P.m / 2, twok = 2 * k;
        const u64 *P0 = w + C.R, *P1 = P0 + N * twok, *PD = P1 + N * twok;
        u64 *out = l == 0 ? r : w + P.R;
        if ((st = launch_flat_scan(ctx, false, w + p.S, P0, P1, twok, N, w + p.cS, s)) != BN_OK) return st;
        if ((st = launch_flat_scan(ctx, false, w + p.Tp, w + p.S, PD, twok, N, w + p.cP, s)) != BN_OK) return st;
        if ((st = launch_flat_scan(ctx, true, w + p.Tm, w + p.S, PD, twok, N, w + p.bM, s)) != BN_OK) return st;
        hipLaunchKernelGGL(k_assemble, dim3(stream_blocks(N * 4 * k)), dim3(256), 0, s, out, w + p.Y, P0, P1,
                           w + p.Tp, w + p.Tm, w + p.cS, w + p.cP, w + p.bM, w + P.negA, w + P.negB, N, k);
        if ((st = bn_launch_status()) != BN_OK) return st;
        // out = P0 + P1 X^2 + (P1 + P0 - P2) X; the product fits 4k limbs, so no carry out
        if ((st = launch_flat_scan(ctx, false, out, out, w + p.Y, 4 * k, N, nullptr, s)) != BN_OK) return st;
    }
    return BN_OK;
}
