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
// split and of the combine is a uniform batch over contiguous arrays.  Both are a
// streaming pass and one carry scan: the signs of A_H - A_L and B_H - B_L come first
// (the highest limb where the halves differ, found piece by piece),
// then every limb of |A_H - A_L| and of P0 + P1 X^2 + (P0 + P1 - P2) X is a signed
// sum of a few limbs, stored biased as a low word and a small high word, and one
// flat carry scan adds the two.
#include "bn_internal.h"

#include <algorithm>
#include <vector>

namespace {

typedef unsigned __int128 u128;

// neg_x[q] = [hi < lo] for the halves lo = x[q][0, k), hi = x[q][k, 2k) of the N
// operands of a and of b, in two steps with a fixed amount of work whatever the data
// (equal halves, as in all-ones or zero operands, leave nothing to stop early on):
// one workgroup per piece of SIGN_PIECE limbs of an operand finds the highest limb i
// where the halves differ and writes key = (i + 1) * 2 + [hi_i < lo_i] (0: no
// difference); then the largest key of an operand's pieces gives its sign.
constexpr u64 SIGN_PIECE = 2048;  // 256 threads x 8 limbs

__global__ __launch_bounds__(256) void k_split_sign_pieces(const u64 *__restrict__ a, const u64 *__restrict__ b,
                                                           u64 N, u64 k, u64 npieces, u64 *__restrict__ keys) {
    __shared__ u64 sh[4];
    const u64 seg = blockIdx.x / npieces, piece = blockIdx.x - seg * npieces;
    const bool is_b = seg >= N;
    const u64 *x = (is_b ? b : a) + 2 * k * (is_b ? seg - N : seg);
    const u64 base = piece * SIGN_PIECE;
    u64 lo[8], hi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const u64 i = base + 256 * u + threadIdx.x;
        lo[u] = i < k ? x[i] : 0;
        hi[u] = i < k ? x[k + i] : 0;
    }
    u64 key = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const u64 i = base + 256 * u + threadIdx.x;
        if (hi[u] != lo[u]) key = std::max(key, ((i + 1) << 1) | (hi[u] < lo[u] ? 1u : 0u));
    }
    for (int off = 32; off > 0; off >>= 1) key = std::max(key, (u64)__shfl_xor(key, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) keys[blockIdx.x] = std::max(std::max(sh[0], sh[1]), std::max(sh[2], sh[3]));
}

__global__ void k_split_sign_reduce(const u64 *__restrict__ keys, u64 N, u64 npieces, u64 *__restrict__ negA,
                                    u64 *__restrict__ negB) {
    const u64 seg = blockIdx.x * (u64)blockDim.x + threadIdx.x;
    if (seg >= 2 * N) return;
    u64 m = 0;
    for (u64 p = 0; p < npieces; ++p) m = std::max(m, keys[seg * npieces + p]);
    if (seg < N) negA[seg] = m & 1;
    else negB[seg - N] = m & 1;
}

// For both operands: the children lo and hi (copies, to dst_x and dst_x + N k) and the
// terms of |hi - lo| = s (hi - lo), s = -1 when neg_x[q]: at limb i the value
// s (hi_i - lo_i) + 2^64 - [i > 0] lies in [0, 2^65); its low word goes to L_x, its
// high word (0 or 1) to H_x one limb up.  The offsets add up to X^k (zero modulo X^k),
// so L_x + H_x is |hi - lo|.
__global__ void k_split_terms(const u64 *__restrict__ a, const u64 *__restrict__ b, u64 N, u64 k,
                              u64 *__restrict__ da, u64 *__restrict__ db, const u64 *__restrict__ negA,
                              const u64 *__restrict__ negB, u64 *__restrict__ L, u64 *__restrict__ H) {
    const u64 total = N * k;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 q = idx / k, i = idx - q * k;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const u64 *x = (side ? b : a) + 2 * k * q;
            u64 *d = side ? db : da;
            const u64 lo = x[i], hi = x[k + i];
            d[idx] = lo;
            d[total + idx] = hi;
            const bool neg = (side ? negB : negA)[q] != 0;
            const u128 v = (u128)(neg ? lo : hi) - (neg ? hi : lo) + ((u128)1 << 64) - (i > 0 ? 1u : 0u);
            u64 *l = L + side * total, *h = H + side * total;
            l[idx] = (u64)v;
            if (i + 1 < k) h[idx + 1] = (u64)(v >> 64);
            if (i == 0) h[idx] = 0;
        }
    }
}

// The terms of a level's result, per product q (4k limbs): at limb i,
//     v_i = [i < 2k] P0_i + [i >= 2k] P1_(i-2k) + [k <= i < 3k] (P0_t + P1_t -+ PD_t),  t = i - k,
// with -PD when the two differences have the same sign (P2 = +PD) and +PD otherwise.
// v_i lies in (-2^64, 2^66); stored as v_i + 2^64 - [i > 0] (in [0, 2^67)): the low
// word to L, the high word to H one limb up (H_0 = 0).  The offsets add up to
// sum_i (X - [i > 0]) X^i = X^(4k), zero modulo X^(4k), and the product fits 4k limbs,
// so L + H (one carry scan, single-bit carries: H <= 4) is the product.
__global__ void k_combine_terms(u64 *__restrict__ L, u64 *__restrict__ H, const u64 *__restrict__ P0,
                                const u64 *__restrict__ P1, const u64 *__restrict__ PD, const u64 *__restrict__ negA,
                                const u64 *__restrict__ negB, u64 N, u64 k) {
    const u64 four = 4 * k, total = N * four;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 q = idx / four, i = idx - q * four;
        const u64 *p0 = P0 + 2 * k * q, *p1 = P1 + 2 * k * q;
        u128 v = (u128)(i < 2 * k ? p0[i] : p1[i - 2 * k]) + ((u128)1 << 64) - (i > 0 ? 1u : 0u);
        if (i >= k && i < 3 * k) {
            const u64 t = i - k;
            const u64 d = PD[2 * k * q + t];
            v += (u128)p0[t] + p1[t];
            v = negA[q] == negB[q] ? v - d : v + d;
        }
        L[idx] = (u64)v;
        if (i + 1 < four) H[idx + 1] = (u64)(v >> 64);
        if (i == 0) H[idx] = 0;
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
    u64 d1, d2;              // split terms: low words, shifted high words (a then b, N_l k each)
    u64 L, H;                // combine terms: low words and shifted high words (4 N_l k each)
    u64 keys;                // split: per-piece sign keys (2 N_l pieces_l, largest level)
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
    u64 N = npairs, m = n, maxNk = 0, maxkeys = 0;
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
            maxkeys = std::max(maxkeys, 2 * N * ((m / 2 + SIGN_PIECE - 1) / SIGN_PIECE));
        }
        N *= 3;
        m /= 2;
    }
    p.d1 = take(2 * maxNk);  // hi - lo of a, then of b
    p.d2 = take(2 * maxNk);  // lo - hi of a, then of b
    p.L = take(4 * maxNk);
    p.H = take(4 * maxNk);
    p.keys = take(maxkeys);
    p.total = off;
    return p;
}

}  // namespace

size_t karatsuba_workspace_bytes(u64 n, u64 npairs, int levels) {
    return (size_t)karatsuba_plan(n, npairs, levels).total * sizeof(u64);
}

// Every buffer a run touches: its own arrays, the bottom batch's multiplication
// workspace, and status words for the largest of its scans (splits: N_l pairs of k
// limbs; combines: N_l pairs of 4 k; the bottom batch's own scans).
WsNeed karatsuba_need(const bn_ctx *ctx, u64 n, u64 npairs, int levels, int form) {
    WsNeed w;
    if (npairs == 0 || n == 0 || levels < 0) return w;
    if (levels == 0) {
        w.work = mul_workspace_bytes(ctx, n, n, npairs, form);
        w.status = mul_status_bytes(ctx, n, n, npairs, form);
        return w;
    }
    const KPlan p = karatsuba_plan(n, npairs, levels);
    w.kwork = (size_t)p.total * sizeof(u64);
    for (int l = 0; l < levels; ++l) {
        const u64 N = p.lv[l].N, k = p.lv[l].m / 2;
        w.status = std::max({w.status, flat_scan_status_bytes(ctx, k, N * k), flat_scan_status_bytes(ctx, 4 * k, N * 4 * k)});
    }
    const KLevel &Bt = p.lv[levels];
    w.work = mul_workspace_bytes(ctx, Bt.m, Bt.m, Bt.N, form);
    w.status = std::max(w.status, mul_status_bytes(ctx, Bt.m, Bt.m, Bt.N, form));
    return w;
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
        const u64 npieces = (k + SIGN_PIECE - 1) / SIGN_PIECE;
        if (2 * N * npieces > 0x7fffffffull) return BN_ERANGE;
        hipLaunchKernelGGL(k_split_sign_pieces, dim3((u32)(2 * N * npieces)), dim3(256), 0, s, pa, pb, N, k, npieces,
                           w + p.keys);
        if ((st = bn_launch_status()) != BN_OK) return st;
        hipLaunchKernelGGL(k_split_sign_reduce, dim3((u32)((2 * N + 255) / 256)), dim3(256), 0, s, w + p.keys, N,
                           npieces, w + P.negA, w + P.negB);
        if ((st = bn_launch_status()) != BN_OK) return st;
        hipLaunchKernelGGL(k_split_terms, dim3(stream_blocks(Nk)), dim3(256), 0, s, pa, pb, N, k, ca, cb, w + P.negA,
                           w + P.negB, w + p.d1, w + p.d2);
        if ((st = bn_launch_status()) != BN_OK) return st;
        for (int side = 0; side < 2; ++side)  // |hi - lo| = L + H, the children [2N, 3N)
            if ((st = launch_flat_scan(ctx, false, (side ? cb : ca) + 2 * Nk, w + p.d1 + side * Nk, w + p.d2 + side * Nk,
                                       k, N, nullptr, s)) != BN_OK)
                return st;
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
        hipLaunchKernelGGL(k_combine_terms, dim3(stream_blocks(N * 4 * k)), dim3(256), 0, s, w + p.L, w + p.H, P0, P1,
                           PD, w + P.negA, w + P.negB, N, k);
        if ((st = bn_launch_status()) != BN_OK) return st;
        // out = P0 + P1 X^2 + (P1 + P0 - P2) X = L + H; the product fits 4k limbs, so no carry out
        if ((st = launch_flat_scan(ctx, false, out, w + p.L, w + p.H, 4 * k, N, nullptr, s)) != BN_OK) return st;
    }
    return BN_OK;
}
