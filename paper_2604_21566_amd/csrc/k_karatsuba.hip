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

// neg_x[q] = [hi < lo] for the halves lo = x[q][0, k), hi = x[q][k, 2k) of the N
// operands of a and of b, in two steps with a fixed amount of work whatever the data
// (equal halves, as in all-ones or zero operands, leave nothing to stop early on):
// one workgroup per piece of SIGN_PIECE limbs of an operand finds the highest limb i
// where the halves differ and writes key = (i + 1) * 2 + [hi_i < lo_i] (0: no
// difference); then the largest key of an operand's pieces gives its sign.
constexpr u64 SIGN_PIECE = 2048;  // 256 threads x 8 limbs

__global__ __launch_bounds__(256) void k_split_sign_pieces(SplitSrc a, SplitSrc b, u64 N, u64 k, u64 npieces,
                                                           u64 *__restrict__ keys) {
    __shared__ u64 sh[4];
    const u64 seg = blockIdx.x / npieces, piece = blockIdx.x - seg * npieces;
    const bool is_b = seg >= N;
    const SplitSrc &x = is_b ? b : a;
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
__global__ void k_split_terms(SplitSrc a, SplitSrc b, u64 N, u64 k, u64 *__restrict__ da, u64 *__restrict__ db,
                              const u64 *__restrict__ negA, const u64 *__restrict__ negB, u64 *__restrict__ L,
                              u64 *__restrict__ H) {
    const u64 total = N * k;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 q = idx / k, i = idx - q * k;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const SplitSrc &x = side ? b : a;
            u64 *d = side ? db : da;
            const u64 lo = src_limb(x, q, i), hi = src_limb(x, q, k + i);
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

// The terms of a level's result, per product q (`out` limbs, out <= 4k): at limb i,
//     v_i = [i < 2k] P0_i + [i >= 2k] P1_(i-2k) + [k <= i < 3k] (P0_t + P1_t -+ PD_t),  t = i - k,
// with -PD when the two differences have the same sign (P2 = +PD) and +PD otherwise.
// v_i lies in (-2^64, 2^66); stored as v_i + 2^64 - [i > 0] (in [0, 2^67)): the low
// word to L, the high word to H one limb up (H_0 = 0).  The offsets add up to
// sum_{i < out} (X - [i > 0]) X^i = X^out, zero modulo X^out, the terms of limbs at or
// above `out` are multiples of X^out, and the product fits `out` limbs (2m at a level
// of m-limb operands, na + nb at the top), so L + H modulo X^out (one carry scan,
// single-bit carries: H <= 4) is the product.
__global__ void k_combine_terms(u64 *__restrict__ L, u64 *__restrict__ H, const u64 *__restrict__ P0,
                                const u64 *__restrict__ P1, const u64 *__restrict__ PD, const u64 *__restrict__ negA,
                                const u64 *__restrict__ negB, u64 N, u64 k, u64 out) {
    const u64 total = N * out;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 q = idx / out, i = idx - q * out;
        const u64 *p0 = P0 + 2 * k * q, *p1 = P1 + 2 * k * q;
        u128 v = (u128)(i < 2 * k ? p0[i] : p1[i - 2 * k]) + ((u128)1 << 64) - (i > 0 ? 1u : 0u);
        if (i >= k && i < 3 * k) {
            const u64 t = i - k;
            const u64 d = PD[2 * k * q + t];
            v += (u128)p0[t] + p1[t];
            v = negA[q] == negB[q] ? v - d : v + d;
        }
        L[idx] = (u64)v;
        if (i + 1 < out) H[idx + 1] = (u64)(v >> 64);
        if (i == 0) H[idx] = 0;
    }
}

u32 stream_blocks(u64 total) { return (u32)std::max<u64>(1, std::min<u64>((total + 255) / 256, 65536)); }

// Workspace layout of a run (u64 offsets).
struct KLevel {
    u64 N, m;        // products and operand limbs at this level (m_0 = max(na, nb), m_(l+1) = ceil(m_l / 2))
    u64 out;         // result limbs per product: 2m, na + nb at the top
    u64 A, B, R;     // operands (N x m each) and products (N x 2m) of this level (level >= 1)
    u64 negA, negB;  // borrows of A_H - A_L and B_H - B_L of this level's split (N each)
};
struct KPlan {
    std::vector<KLevel> lv;  // 0 .. levels
    u64 d1, d2;              // split terms: low words, shifted high words (a then b, N_l k each)
    u64 L, H;                // combine terms: low words and shifted high words (N_l out_l each)
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
    u64 N = npairs, m = std::max(na, nb), maxNk = 0, maxout = 0, maxkeys = 0;
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
            L.negA = take(N);
            L.negB = take(N);
            maxNk = std::max(maxNk, N * k);
            maxout = std::max(maxout, N * L.out);
            maxkeys = std::max(maxkeys, 2 * N * ((k + SIGN_PIECE - 1) / SIGN_PIECE));
        }
        N *= 3;
        m = k;
    }
    p.d1 = take(2 * maxNk);  // hi - lo of a, then of b
    p.d2 = take(2 * maxNk);  // lo - hi of a, then of b
    p.L = take(maxout);
    p.H = take(maxout);
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
        w.status = std::max({w.status, flat_scan_status_bytes(ctx, k, N * k), flat_scan_status_bytes(ctx, out, N * out)});
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
        const u64 N = P.N, k = C.m, twok = 2 * k;
        const u64 *P0 = w + C.R, *P1 = P0 + N * twok, *PD = P1 + N * twok;
        u64 *out = l == 0 ? r : w + P.R;
        hipLaunchKernelGGL(k_combine_terms, dim3(stream_blocks(N * P.out)), dim3(256), 0, s, w + p.L, w + p.H, P0, P1,
                           PD, w + P.negA, w + P.negB, N, k, P.out);
        if ((st = bn_launch_status()) != BN_OK) return st;
        // out = P0 + P1 X^2 + (P1 + P0 - P2) X = L + H modulo X^out; the product fits
        // out limbs, so no carry leaves the top
        if ((st = launch_flat_scan(ctx, false, out, w + p.L, w + p.H, P.out, N, nullptr, s)) != BN_OK) return st;
    }
    return BN_OK;
}
