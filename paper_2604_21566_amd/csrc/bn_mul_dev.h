// bn_mul_dev.h -- device building blocks of the two multiplication forms.
//
// Both forms follow DoT multiplication (Sec. 3.2, Algorithm 2, "vertical and
// crosswise"): every cross product A_i * B_j is independent and lands in output
// column i + j (Theorem 2); the column sums are formed first and the carries are
// resolved once at the end.  What differs from the paper is the digit size and the
// unit that forms the products:
//   * mad form  : 32-bit digits, v_mad_u64_u32 with a carry-out into a 96-bit
//                 column accumulator (the paper's IFMA lo/hi products become one
//                 32x32->64 multiply-add per digit pair);
//   * MFMA form : 8-bit digits (the paper splits 64-bit limbs to fit its
//                 multiplier; here the digits are balanced signed bytes of the
//                 operand, one more than its byte count), the digit convolution
//                 written as a block-Toeplitz matrix product on
//                 v_mfma_i32_32x32x32_i8 with int32 accumulation.
// The deferred carry pass (Algorithm 2, phase 5) is: fold each limb's column sums
// into V_j = lo_j + 2^64 hi_j, then r = sum_j lo_j X^j + sum_j hi_j X^(j+1), i.e.
// one big-integer addition whose carries are single bits (g/p scan).  Signed limb
// values are stored biased, V_j + K 2^64 - [j > 0] K, offsets that sum to K X^P.
#pragma once

#include "bn_internal.h"

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned __int128 u128;

#define BN_DPP_WAVE_SHR1 0x138

// lo:hi (96-bit) += x * y, using the carry-out of v_mad_u64_u32.  x is wave-uniform
// and stays in an SGPR (one scalar source per VOP3 instruction).
__device__ __forceinline__ void mac96(u64 &lo, u32 &hi, u32 x, u32 y) {
    u64 cc;
    asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
        "v_addc_co_u32 %2, %1, 0, %2, %1"
        : "+v"(lo), "=&s"(cc), "+v"(hi)
        : "s"(x), "v"(y));
}

// Value of a wave-uniform step's operand held in lane k of v (k uniform).
__device__ __forceinline__ u32 lane_value(u32 v, u32 k) { return (u32)__builtin_amdgcn_readlane((int)v, (int)k); }

// Wave-local LDS ordering point (all waves of a workgroup run independently).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Deferred carry pass inside one wave.  Lane l owns limbs j = l*L + k (k < L) with
// values V_j = lo[k] + 2^64 hi[k] (hi small).  Writes r[j] for j < P.  The sum of all
// V_j X^j is the product, which fits P limbs, so the final carry is zero.
template <int L>
__device__ __forceinline__ void wave_normalise_store(const u64 (&lo)[L], const u64 (&hi)[L], u32 P, u64 *r) {
    const int lane = threadIdx.x & 63;
    u64 prev = __shfl_up(hi[L - 1], 1);
    if (lane == 0) prev = 0;
    u64 x[L];
    bool g[L], p[L];
    bool G = false, PP = true;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const u32 j = (u32)lane * L + k;
        const u64 h = (k == 0) ? prev : hi[k - 1];
        x[k] = lo[k] + h;
        const bool v = j < P;
        g[k] = v && (x[k] < h);
        p[k] = v && (x[k] == ~0ull);
        G = g[k] || (p[k] && G);
        PP = PP && p[k];
    }
    const u64 Gm = __ballot(G), Pm = __ballot(PP);
    const u64 C = ((Gm << 1) + Pm) ^ Pm;
    bool c = (C >> lane) & 1ull;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const u32 j = (u32)lane * L + k;
        if (j < P) r[j] = x[k] + (u64)c;
        c = g[k] || (p[k] && c);
    }
}

// ------------------------------------------------------------------ mad form ----
// One wave computes one product of P = na + nb <= 64 L limbs.  Lane l owns the
// 32-bit columns t = 2 L l + q (q < 2L).  All lanes step through the 32-bit digits
// x of a together: alpha_x is wave-uniform; column t needs beta_{t-x}.  The beta
// window of a lane slides down by one digit per step, so the new bottom element is
// the neighbouring lane's top element: one DPP wave_shr:1 per step (lane 0 receives
// beta at a negative index, i.e. 0).
template <int L>
__device__ void mul_item_mad(const u64 *__restrict__ a, u32 na, const u64 *__restrict__ b, u32 nb,
                             u64 *__restrict__ r) {
    static_assert(L > 0 && (L & (L - 1)) == 0 && L <= 16, "2 L steps per group must divide the 64 of a load");
    // the step loop runs over the digits of a: make a the shorter operand (a*b = b*a)
    if (na > nb) {
        const u64 *t = a;
        a = b;
        b = t;
        const u32 tn = na;
        na = nb;
        nb = tn;
    }
    constexpr int Q = 2 * L;
    const int lane = threadIdx.x & 63;
    const u32 *a32 = reinterpret_cast<const u32 *>(a);
    const u32 *b32 = reinterpret_cast<const u32 *>(b);
    const u32 nx = 2 * na, ny = 2 * nb;
    const u32 t0 = (u32)lane * Q;
    u32 R[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const u32 y = t0 + q;
        R[q] = y < ny ? b32[y] : 0u;
    }
    u64 lo[Q];
    u32 hi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        lo[q] = 0;
        hi[q] = 0;
    }
    // The digits of a are the same for every lane: scalar loads, 2 Q per group of steps
    // (a group past nx reads no memory beyond the operand; its missing digits are 0 and
    // their steps only cost time).
    {
        for (u32 s0 = 0; s0 < nx; s0 += 2 * Q) {
            u32 ad[2 * Q];
#pragma unroll
            for (int s = 0; s < 2 * Q; ++s) ad[s] = s0 + s < nx ? a32[s0 + s] : 0u;
#pragma unroll
            for (int s = 0; s < 2 * Q; ++s) {
                const u32 al = ad[s];
#pragma unroll
                for (int q = 0; q < Q; ++q) mac96(lo[q], hi[q], al, R[(q - s + 2 * Q) % Q]);
                const int k = (Q - 1 - s + 2 * Q) % Q;
                R[k] = (u32)__builtin_amdgcn_update_dpp(0, (int)R[k], BN_DPP_WAVE_SHR1, 0xf, 0xf, true);
            }
        }
    }
    u64 vlo[L], vhi[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const u128 v = (u128)lo[2 * k] + ((u128)hi[2 * k] << 64) + ((u128)lo[2 * k + 1] << 32) +
                       ((u128)hi[2 * k + 1] << 96);
        vlo[k] = (u64)v;
        vhi[k] = (u64)(v >> 64);
    }
    wave_normalise_store<L>(vlo, vhi, na + nb, r);
}

// mac96 with the digit x in a vector register (it differs between the two halves of
// the wave in mul_item_mad_pair).
__device__ __forceinline__ void mac96v(u64 &lo, u32 &hi, u32 x, u32 y) {
    u64 cc;
    asm("v_mad_u64_u32 %0, %1, %3, %4, %0\n\t"
        "v_addc_co_u32 %2, %1, 0, %2, %1"
        : "+v"(lo), "=&s"(cc), "+v"(hi)
        : "v"(x), "v"(y));
}

// Two products of at most 32 limbs each on one wave: lanes 0-31 compute item 0 as
// mul_item_mad<1> would on 32 lanes (lane l owns 32-bit columns 2l, 2l + 1), lanes
// 32-63 item 1.  The shorter operands of the two items must have the same length, so
// both halves run the same digit steps; the digits of each half's shorter operand come
// from vector loads of half-uniform addresses.  Lane 32 starts item 1's window: the
// wave-wide shift would hand it lane 31's element, so it takes 0 instead.  The carry
// pass runs as two 32-lane scans (each half's masks on their own).
__device__ void mul_item_mad_pair(const RItem &m0, const RItem &m1, const u64 *__restrict__ a,
                                  const u64 *__restrict__ b, u64 *__restrict__ r) {
    const int lane = threadIdx.x & 63;
    const bool h = lane >= 32;
    const u32 hl = (u32)lane & 31u;
    // each item's shorter operand is x (its digits are the steps), the other y
    const bool sw0 = m0.na > m0.nb, sw1 = m1.na > m1.nb;
    const u64 *x0 = sw0 ? b + m0.b_off : a + m0.a_off, *y0 = sw0 ? a + m0.a_off : b + m0.b_off;
    const u64 *x1 = sw1 ? b + m1.b_off : a + m1.a_off, *y1 = sw1 ? a + m1.a_off : b + m1.b_off;
    const u32 nx = 2 * (sw0 ? m0.nb : m0.na);  // digits of x, the same for both items
    const u32 ny = h ? 2 * (sw1 ? m1.na : m1.nb) : 2 * (sw0 ? m0.na : m0.nb);
    const u32 *x32 = reinterpret_cast<const u32 *>(h ? x1 : x0);
    const u32 *y32 = reinterpret_cast<const u32 *>(h ? y1 : y0);
    const u32 t0 = 2 * hl;
    u32 R[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) R[q] = t0 + q < ny ? y32[t0 + q] : 0u;
    u64 lo[2] = {0, 0};
    u32 hi[2] = {0, 0};
    for (u32 s0 = 0; s0 < nx; s0 += 4) {
        u32 ad[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) ad[s] = s0 + s < nx ? x32[s0 + s] : 0u;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int q = 0; q < 2; ++q) mac96v(lo[q], hi[q], ad[s], R[(q - s + 4) % 2]);
            const int k = (1 - s + 4) % 2;
            const u32 sh = (u32)__builtin_amdgcn_update_dpp(0, (int)R[k], BN_DPP_WAVE_SHR1, 0xf, 0xf, true);
            R[k] = lane == 32 ? 0u : sh;
        }
    }
    // limb hl of this half's product: V = lo0 + 2^32 lo1 + 2^64 hi0 + 2^96 hi1
    const u128 v = (u128)lo[0] + ((u128)hi[0] << 64) + ((u128)lo[1] << 32) + ((u128)hi[1] << 96);
    const u64 vlo = (u64)v, vhi = (u64)(v >> 64);
    const u32 P = h ? m1.na + m1.nb : m0.na + m0.nb;
    u64 prev = __shfl_up(vhi, 1);
    if (hl == 0) prev = 0;
    const u64 x = vlo + prev;
    const bool valid = hl < P;
    const u64 Gm = __ballot(valid && x < prev), Pm = __ballot(valid && x == ~0ull);
    const u32 G0 = (u32)Gm, P0 = (u32)Pm, G1 = (u32)(Gm >> 32), P1 = (u32)(Pm >> 32);
    const u32 C0 = ((G0 << 1) + P0) ^ P0, C1 = ((G1 << 1) + P1) ^ P1;
    const u64 c = ((h ? C1 : C0) >> hl) & 1u;
    if (valid) r[(h ? m1.r_off : m0.r_off) + hl] = x + c;
}

// ----------------------------------------------------------------- MFMA form ----
// Digit convolution as block-Toeplitz products.  With 8-bit digits a_i, b_j and
// output digit columns t = 32 W + rr (rr < 32):
//     C[32 W + rr] = sum_d sum_k T_d[rr][k] * A_d[k][W]
//     T_d[rr][k]   = b[32 (d-1) + rr + 1 + k]          (Toeplitz in rr - k)
//     A_d[k][W]    = a[32 (W-d) + 31 - k]              (32-digit chunk W-d, reversed)
// so one v_mfma_i32_32x32x32_i8 per (d, block of 32 W) forms 32x32 column sums.
// The instruction multiplies signed int8, so both operands enter as balanced signed
// digits in [-128, 127] (one more digit than the operand has bytes; see
// wave_balanced_digits): the digits sum to the operand exactly, so every column sum
// is the true signed column sum of the product and needs no correction.  A digit
// product lies in [-16256, 16384]; one-wave products (at most 8 * 512 + 1 digit pairs
// per column) keep exact int32 sums, and the large kernel's int32 bound is stated
// where its epilogue decodes the sums (k_mul.hip).
//
// Operand registers: lane (x = lane & 31, h = lane >> 5) supplies bytes k = 16 h .. 16 h + 15
// of row x of T_d (A-operand) and of column x of A_d (B-operand).  Both operands
// use the same (h, byte) -> k assignment, so the contraction pairs the right bytes
// whatever order the hardware uses inside the K dimension.

// T_d row fragment from a byte array staged in LDS (as 32-bit words).  `off` is the
// byte offset of the row's first digit, 32 (d-1) + rr + 1 + 16 h relative to the
// staging base; reads 5 aligned words and funnel-shifts them.
__device__ __forceinline__ v4i toeplitz_frag(const u32 *__restrict__ lds_words, u32 off) {
    const u32 q = off >> 2, s = off & 3u;
    const u32 w0 = lds_words[q], w1 = lds_words[q + 1], w2 = lds_words[q + 2], w3 = lds_words[q + 3],
              w4 = lds_words[q + 4];
    v4i t;
    t.x = (int)__builtin_amdgcn_alignbyte(w1, w0, s);
    t.y = (int)__builtin_amdgcn_alignbyte(w2, w1, s);
    t.z = (int)__builtin_amdgcn_alignbyte(w3, w2, s);
    t.w = (int)__builtin_amdgcn_alignbyte(w4, w3, s);
    return t;
}

// The same fragment in two halves, so that the LDS reads of the next step can be
// issued before the current step's MFMAs: load the five words, combine later.
struct TWords {
    u32 w0, w1, w2, w3, w4;
};
__device__ __forceinline__ TWords toeplitz_words(const u32 *__restrict__ lds_words, u32 off) {
    const u32 q = off >> 2;
    return TWords{lds_words[q], lds_words[q + 1], lds_words[q + 2], lds_words[q + 3], lds_words[q + 4]};
}
template <class P>
__device__ __forceinline__ TWords tw_at(P lds_words, int q) {
    return TWords{lds_words[q], lds_words[q + 1], lds_words[q + 2], lds_words[q + 3], lds_words[q + 4]};
}
__device__ __forceinline__ v4i toeplitz_combine(const TWords &t, u32 s) {
    v4i f;
    f.x = (int)__builtin_amdgcn_alignbyte(t.w1, t.w0, s);
    f.y = (int)__builtin_amdgcn_alignbyte(t.w2, t.w1, s);
    f.z = (int)__builtin_amdgcn_alignbyte(t.w3, t.w2, s);
    f.w = (int)__builtin_amdgcn_alignbyte(t.w4, t.w3, s);
    return f;
}

// Accumulator element (reg g of lane l) -> (row rr, column x) of the 32x32 tile.
__device__ __forceinline__ u32 acc_row(int g, int lane) { return (u32)((g & 3) + 4 * (lane >> 5) + 8 * (g >> 2)); }


// ------------------------------------------------- small products, MFMA form ----
constexpr u64 BN_XOR80 = 0x8080808080808080ull;

// Balanced signed digits of one operand by one wave: digits d_i in [-128, 127] with
// sum d_i 256^i = the operand, one extra digit for the carry out of the top.  Adding
// 128 to every byte with full carries gives bytes b_i + 128 + c_i (mod 256) and
// carries c_{i+1} = [b_i + c_i >= 128] -- the recurrence of the balanced conversion --
// so the two's-complement bytes of the digits are the bytes of
// (x + 0x8080...80) xor 0x8080...80 over n + 1 limbs (limb n holds the top carry as
// its digit 0; limbs above it come out zero).  Lane l returns limbs LPL l .. LPL l +
// LPL - 1 of that over 64 LPL limbs (n < 64 LPL): one addition of a constant, carries
// resolved with a ballot scan as in wave_normalise_store.
template <int LPL>
__device__ __forceinline__ void wave_balanced_digits(const u64 *__restrict__ limbs, u32 n, u64 (&out)[LPL]) {
    const int lane = threadIdx.x & 63;
    u64 s[LPL];
    bool g[LPL], p[LPL];
    bool G = false, PP = true;
#pragma unroll
    for (int k = 0; k < LPL; ++k) {
        const u32 m = LPL * lane + k;
        const u64 v = m < n ? limbs[m] : 0ull;
        s[k] = v + BN_XOR80;
        g[k] = s[k] < v;
        p[k] = s[k] == ~0ull;
        G = g[k] || (p[k] && G);
        PP = PP && p[k];
    }
    const u64 Gm = __ballot(G), Pm = __ballot(PP);
    const u64 C = ((Gm << 1) + Pm) ^ Pm;
    bool c = (C >> lane) & 1ull;
#pragma unroll
    for (int k = 0; k < LPL; ++k) {
        out[k] = (s[k] + (u64)c) ^ BN_XOR80;
        c = g[k] || (p[k] && c);
    }
}

// One row of 256 limbs of the deferred carry pass: lane l owns limbs base + 4l + k
// with values lo[k] + 2^64 hi[k] (hi >= 0, small); `carry` and `prev_hi` (the high
// word of the limb below the row) come in from the row below and go out to the row
// above.  Writes the limbs below P.
__device__ __forceinline__ void wave_normalise_row(const u64 (&lo)[4], const u64 (&hi)[4], u32 base, u32 P, u64 *r,
                                                   u64 &carry, u64 &prev_hi) {
    const int lane = threadIdx.x & 63;
    u64 prev = __shfl_up(hi[3], 1);
    if (lane == 0) prev = prev_hi;
    u64 x[4];
    bool g[4], p[4];
    bool G = false, PP = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const u64 h = (k == 0) ? prev : hi[k - 1];
        x[k] = lo[k] + h;
        g[k] = x[k] < h;
        p[k] = x[k] == ~0ull;
        G = g[k] || (p[k] && G);
        PP = PP && p[k];
    }
    const u64 Gm = __ballot(G), Pm = __ballot(PP);
    const u64 C = (((Gm << 1) | carry) + Pm) ^ Pm;
    bool c = (C >> lane) & 1ull;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const u32 j = base + 4 * (u32)lane + k;
        if (j < P) r[j] = x[k] + (u64)c;
        c = g[k] || (p[k] && c);
    }
    carry = (Gm >> 63) | ((Pm >> 63) & (C >> 63));
    prev_hi = (u64)(u32)__builtin_amdgcn_readlane((int)(u32)hi[3], 63) |
              ((u64)(u32)__builtin_amdgcn_readlane((int)(u32)(hi[3] >> 32), 63) << 32);
}

// Shapes of the one-wave MFMA product with NB column blocks of 128 output limbs
// (products of up to 128 NB limbs; NB = 1, 2 or 4).
template <int NB>
struct SmallMfma {
    static constexpr int LPL = 2 * NB;       // limbs per lane in the digit conversion
    // b digits: 4 zero limbs, nb + 1 <= 64 NB + 1 limbs and the read-ahead; the size
    // also places the a digits (measured: 152 words for NB = 2 made the a reads 8%
    // slower than 272)
    static constexpr int BZ = 128 * NB + 16;
    static constexpr int AR = 64 * LPL;      // a digits, chunk-reversed (na + 1 <= 128 NB limbs)
    static constexpr int LDS_U64 = BZ + AR;  // per wave
};

// One product of P = na + nb <= 128 NB limbs on the MFMA form, one wave.
// lds: SmallMfma<NB>::LDS_U64 words private to the wave.
//
// The digits are balanced (wave_balanced_digits), so every MFMA column sum is the
// exact signed column sum C_t of the product, sum_t C_t 256^t = a b, and no
// correction is needed: limb j's value is V_j = sum_{u<8} C_{8j+u} 2^(8u).  For the
// carry pass every V_j (j < P) gets K 2^64 added and every V_j (0 < j < P) K
// subtracted: that adds K X^P in total, which vanishes modulo X^P, and keeps every
// high word non-negative (|V_j| < 2^86, K = 2^40), so the unsigned carry pass returns
// a b mod X^P = a b.  Column sums are exact int32: at most 8 * 512 + 1 products of
// absolute value at most 2^14.
template <int NB>
__device__ __forceinline__ void mul_item_mfma_small(const u64 *__restrict__ a, u32 na, const u64 *__restrict__ b,
                                                    u32 nb, u64 *__restrict__ r, u64 *lds) {
    using S = SmallMfma<NB>;
    // the Toeplitz steps run over the digits of b: make b the shorter operand
    if (nb > na) {
        const u64 *t = a;
        a = b;
        b = t;
        const u32 tn = na;
        na = nb;
        nb = tn;
    }
    // the lane index through an opaque move: keeps a caller's item loop from hoisting
    // the many lane-dependent values of the epilogue out of the loop (which would hold
    // them in registers across items and cut the occupancy)
    int lane;
    asm volatile("v_and_b32 %0, 63, %1" : "=v"(lane) : "v"((int)threadIdx.x));
    const u32 x = lane & 31, h = lane >> 5;
    const u32 P = na + nb;
    const u32 ndb = 8 * nb + 1;        // digits of b, with the carry digit
    const u32 nca = (na + 1 + 3) / 4;  // 32-digit chunks of a (with the carry digit)
    u64 *bz = lds;                     // [0,4) zero pad, [4, 4+nb+1) b digits, then zeros
    u64 *aR = lds + S::BZ;             // a digits, chunk-reversed, 4*nca limbs
    {
        u64 db[S::LPL], da[S::LPL];
        wave_balanced_digits<S::LPL>(b, nb, db);
        wave_balanced_digits<S::LPL>(a, na, da);
#pragma unroll
        for (int k = 0; k < S::LPL; ++k) {
            const u32 m = S::LPL * lane + k;
            if (4 + m < (u32)S::BZ) bz[4 + m] = db[k];
            if (m < 4 * nca) aR[4 * nca - 1 - m] = __builtin_bswap64(da[k]);
        }
        // zero pad, from the opaque lane index (lane >> 6 is 0): a literal zero here was
        // kept in registers across the caller's item loop and spilled
        if (lane < 4) bz[lane] = (u64)((u32)lane >> 6);
    }
    wave_sync();

    const u32 dmax = (ndb + 30) / 32;
    const u32 nblk = (P + 127) / 128;  // column blocks that hold output limbs
    const u32 *bz32 = reinterpret_cast<const u32 *>(bz);
    v16i acc[NB];
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) acc[blk] = v16i{0};
    for (u32 d = 0; d <= dmax; ++d) {
        const v4i T = toeplitz_frag(bz32, 32 * d + x + 1 + 16 * h);
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) {
            if (blk == 0 || (u32)blk < nblk) {  // block 0 always holds output limbs
                const int c = 32 * blk + (int)x - (int)d;
                v4i A = {0, 0, 0, 0};
                if (c >= 0 && c < (int)nca) A = *reinterpret_cast<const v4i *>(aR + 4 * nca - 4 * (c + 1) + 2 * h);
                acc[blk] = __builtin_amdgcn_mfma_i32_32x32x32_i8(T, A, acc[blk], 0, 0, 0);
            }
        }
    }

    // Limb j = 4 W + m holds digit columns t = 32 W + 8 m + u (u < 8); lane (x, h) has
    // u = 4h .. 4h+3 of limbs 4 (32 blk + x) + m.  Each lane folds its four columns of
    // every limb (signed, below 2^52 in magnitude), then partners (lane xor 32) swap
    // halves so that lane l ends up owning limbs 256 s + 4 l + m of blocks 2 s + h;
    // the carry pass then runs over rows of 256 limbs.  With one block (NB = 1) both
    // partners end up with the block's limbs; lanes 32-63 hold them as limbs 128-255,
    // above every limb of the product (P <= 128): the row's stores skip them and their
    // carries only move further up.
    constexpr i64 K = (i64)1 << 40;
    u64 carry = 0, prev_hi = 0;
#pragma unroll
    for (int sr = 0; sr < (NB + 1) / 2; ++sr) {
        u64 vlo[4], vhi[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            i64 part[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int blk = 2 * sr + e < NB ? 2 * sr + e : 0;
                i64 w = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) w += (i64)acc[blk][4 * m + i] * ((i64)1 << (8 * i));
                part[e] = w;
            }
            const i64 own = h ? part[1] : part[0];
            const i64 rcv = __shfl_xor(h ? part[0] : part[1], 32);
            // digits 0..3 weigh 2^0, digits 4..7 weigh 2^32
            const i64 lo4 = h ? rcv : own, hi4 = h ? own : rcv;
            const u32 j = 256 * sr + 4 * (u32)lane + m;
            const __int128 v = (__int128)lo4 + ((__int128)hi4 << 32) + ((__int128)K << 64) - (j > 0 ? K : 0);
            vlo[m] = (u64)v;
            vhi[m] = (u64)((unsigned __int128)v >> 64);
        }
        wave_normalise_row(vlo, vhi, 256 * sr, P, r, carry, prev_hi);
    }
}
