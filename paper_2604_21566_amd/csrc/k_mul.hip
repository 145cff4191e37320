// k_mul.hip -- multiplication kernels and the uniform-batch dispatcher.
//
// Small products (na + nb <= 512 limbs on the MFMA form, <= 1024 on the mad form): one
// wave per pair does everything -- column products, fold, and the in-wave carry pass
// -- with no workspace.
// Large products, mad form: work items (output-column block x slice of the
// contraction range, so every item has about the same work) add their 96-bit column
// sums into a workspace with 64-bit atomics, and a fold kernel turns the column sums
// into per-limb (lo, hi) pairs.  MFMA form: the operands are converted to balanced
// signed digits by one carry scan each; a workgroup owns a band of output columns
// and runs their whole contraction range (unsplit: exact int32 sums decoded in the
// epilogue, which writes the per-limb values itself, no atomics) or one slice of it
// (split: per-slice int32 partials, added by a fold kernel).  Either way the deferred
// carry pass is the add kernel itself: r = LO + (HI shifted up one limb).
#include "bn_mul_dev.h"

#include <algorithm>

namespace {

constexpr u64 XOR80 = 0x8080808080808080ull;
constexpr u64 MUL_BIAS = 1ull << 62;  // K of the biased signed limb values
constexpr u64 SMALL_MAX_P = 1024;       // one-wave mad products: up to 16 limbs of output per lane
constexpr u64 SMALL_MFMA_MAX_P = 512;   // one-wave MFMA products: up to four 128-limb column blocks

// Products that run on one wave each (no workspace).
bool mul_one_wave(u64 P, int form) { return P <= (form == BN_MUL_MFMA ? SMALL_MFMA_MAX_P : SMALL_MAX_P); }

// -------------------------------------------------------------- small kernels ----

// Uniform batch of small products: wave w of block blk handles pair 4*blk + w.  The
// MFMA form is bounded to eight (one or two column blocks) or four (four blocks) waves
// per SIMD: the compiler then keeps the accumulators in ordinary registers (53 / 80 in
// all, no spills) instead of splitting off accumulation registers, one to two more
// waves than without the bound (192- and 256-limb products 17-20% faster).
template <int FORM, int L>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(FORM == BN_MUL_MFMA ? (L <= 2 ? 8 : 4) : 1, 8))) void k_mul_small(u64 *__restrict__ r, const u64 *__restrict__ a,
                                                   const u64 *__restrict__ b, u32 na, u32 nb, u64 npairs) {
    __shared__ u64 lds[FORM == BN_MUL_MFMA ? 4 * SmallMfma<L>::LDS_U64 : 1];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const u64 p = (u64)blockIdx.x * 4 + w;
    if (p >= npairs) return;
    const u64 *pa = a + p * na;
    const u64 *pb = b + p * nb;
    u64 *pr = r + p * (u64)(na + nb);
    if (FORM == BN_MUL_MFMA)
        mul_item_mfma_small<L>(pa, na, pb, nb, pr, lds + w * SmallMfma<L>::LDS_U64);
    else
        mul_item_mad<L>(pa, na, pb, nb, pr);
}

// ----------------------------------------------------------- large: mad form ----
// Work item (one wave): 32-bit output columns [T0, T0 + 64 Q) x digits x of a in one
// slice of XC.  Column sums are 96-bit (lo 64 + hi 32) and are added into the
// workspace with two 64-bit atomics (the returned old low word tells whether the
// low add wrapped).
template <int Q>
__global__ __launch_bounds__(256) void k_mul_large_mad(const u64 *__restrict__ a, const u64 *__restrict__ b, u64 na,
                                                       u64 nb, u64 nxc, u64 nitems, u32 XC, u64 *__restrict__ colLo,
                                                       u64 *__restrict__ colHi) {
    const int lane = threadIdx.x & 63;
    const u64 item = (u64)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= nitems) return;
    const u64 pair = blockIdx.y;
    const u64 cb = item / nxc, xc = item % nxc;
    const u32 *a32 = reinterpret_cast<const u32 *>(a + pair * na);
    const u32 *b32 = reinterpret_cast<const u32 *>(b + pair * nb);
    const i64 nx = 2 * (i64)na, ny = 2 * (i64)nb;
    const i64 T0 = (i64)cb * 64 * Q;
    const i64 xs = std::max<i64>((i64)xc * XC, T0 + 1 - ny);
    const i64 xe = std::min<i64>(std::min<i64>(((i64)xc + 1) * XC, T0 + 64 * Q), nx);
    if (xs >= xe) return;
    const i64 tl = T0 + (i64)Q * lane;

    u32 R[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const i64 y = tl + q - xs;
        R[q] = (y >= 0 && y < ny) ? b32[y] : 0u;
    }
    u64 lo[Q];
    u32 hi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        lo[q] = 0;
        hi[q] = 0;
    }
    // 64 digits of a and the 64 lane-0 fill values of beta per coalesced load; each
    // step broadcasts its pair with readlane.  Steps past xe use a zero digit.
    for (i64 xb = xs; xb < xe; xb += 64) {
        const u32 areg = (xb + lane < xe) ? a32[xb + lane] : 0u;
        const i64 yf = T0 - xb - 1 - lane;  // fill for step xb + lane
        const u32 freg = (yf >= 0 && yf < ny) ? b32[yf] : 0u;
        for (u32 s0 = 0; s0 < 64 && xb + s0 < xe; s0 += Q) {
#pragma unroll
            for (int s = 0; s < Q; ++s) {
                const u32 al = lane_value(areg, s0 + s);
#pragma unroll
                for (int q = 0; q < Q; ++q) mac96(lo[q], hi[q], al, R[(q - s + Q) % Q]);
                const u32 fill = lane_value(freg, s0 + s);
                const int k = (Q - 1 - s + Q) % Q;
                R[k] = (u32)__builtin_amdgcn_update_dpp((int)fill, (int)R[k], BN_DPP_WAVE_SHR1, 0xf, 0xf, false);
            }
        }
    }
    const u64 ncol = 2 * (na + nb);
    u64 *cl = colLo + pair * ncol;
    u64 *ch = colHi + pair * ncol;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const u64 t = (u64)tl + q;
        if (t < ncol && (lo[q] | hi[q])) {
            const u64 old = __hip_atomic_fetch_add(cl + t, lo[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const u64 add = (u64)hi[q] + ((old + lo[q]) < old ? 1u : 0u);
            if (add) __hip_atomic_fetch_add(ch + t, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Column sums (32-bit columns) -> per-limb lo and shifted hi.
__global__ void k_fold_mad(const u64 *__restrict__ colLo, const u64 *__restrict__ colHi, u64 P, u64 total,
                           u64 *__restrict__ LO, u64 *__restrict__ HS) {
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 p = idx / P, j = idx - p * P;
        const u64 base = p * 2 * P + 2 * j;
        const u128 K0 = (u128)colLo[base] + ((u128)colHi[base] << 64);
        const u128 K1 = (u128)colLo[base + 1] + ((u128)colHi[base + 1] << 64);
        const u128 V = K0 + (K1 << 32);
        LO[idx] = (u64)V;
        if (j + 1 < P) HS[idx + 1] = (u64)(V >> 64);
        if (j == 0) HS[idx] = 0;
    }
}

// ---------------------------------------------------------- large: MFMA form ----
// Operands enter as balanced signed digits: the flat scan adds 0x80...80 to every
// operand of the batch (one pass over a, one over b, each limb read and written once),
// and digit i is byte i of the sum xor 0x80, read as int8 in [-128, 127]; the scan's
// carry out of a pair is that operand's extra top digit (index 8 n, value 0 or 1).  The
// digits sum to the operand exactly (the same conversion as the one-wave kernel), so
// every MFMA column sum is the true signed column sum and needs no correction.

// k-th group in decreasing-work order when work over groups [0, n) is symmetric and
// unimodal about the centre (true for the columns of a product): centre first, then
// alternately outwards.
__device__ __forceinline__ u32 middle_out(u32 k, u32 n) {
    if (n & 1) {
        const u32 c = (n - 1) / 2;
        if (k == 0) return c;
        return (k & 1) ? c - (k + 1) / 2 : c + k / 2;
    }
    const u32 m = n / 2 - 1;
    return (k & 1) ? m + (k + 1) / 2 : m - k / 2;
}

template <class T>
using lds_cptr = const __attribute__((address_space(3))) T *;  // read-only pointer into LDS

constexpr int AZ_SLOT_U64 = 10;  // one 64-digit chunk per 80-byte LDS slot: ds_read_b128 without bank conflicts


// Large products on the MFMA form.  Output digit columns are grouped 64 R at a time
// (t = 64 R W + r, r < 64 R; R = 1 or 2), the Toeplitz step consumes 64 digits of b:
//     C[64 R W + r] = sum_d sum_k T_d[r][k] A_d[k][W],
//     T_d[r][k] = b'[64 (d-1) + r + 1 + k],   A_d[k][W] = a'[64 (R W - d) + 63 - k].
// A W-block (32 W = 256 R output limbs, 64 R rows = 2 R 32-row M-blocks) takes 4 R
// 32x32x32 MFMAs per step.  The 2 R + 1 distinct Toeplitz fragments of a step (rows +
// K-slice offsets 0, 32, ..., 64 R) are shared by the wave's NW blocks, and all but
// two of them are the next step's first ones: every step reads two new Toeplitz
// fragments and two a fragments per block, whatever R, so R = 2 feeds twice the
// MFMAs from the same LDS reads.  A workgroup (4 waves, 4 NW blocks) covers the whole
// contraction range of its blocks (or, SPLIT, one slice of it when there are too
// few workgroups to fill the device), staging D steps of b digits and the matching
// window of a chunks (byte-reversed) in LDS per round: no atomics and no
// workspace zeroing in the unsplit case.  Accumulation is int32.  Unsplit launches
// are used while a column holds at most 131586 digit products: its register holds
// the true signed sum M modulo 2^32 and M lies in [-16256 cnt, 16384 cnt], narrower
// than 2^32, so the epilogue decodes it exactly, folds the 64 R columns of each W
// into 8 R signed limb values and writes them biased (see the epilogue) as lo and
// shifted hi.  Split launches keep every slice
// at most 2046 steps when columns are longer (2046 * 64 * 2^14 < 2^31, exact) and
// write the slice sums to per-slice int32 arrays that a fold kernel adds.
// Workgroups are ordered by decreasing work.
// Instruction order of one step of the large MFMA kernel: the LDS reads of the next
// step go out first, then half of the MFMAs, then the VALU work (byte shifts of the
// fragments just read, addresses) between the other half (the scheduler would
// otherwise issue each read just before its use and wait for it).
template <int NW, int R>
__device__ __forceinline__ void mfma_step_order() {
    constexpr int MFMA = 0x008, VALU = 0x002, DSR = 0x100;
    constexpr int N = 4 * R * NW;  // MFMAs per step
    __builtin_amdgcn_sched_group_barrier(DSR, 5 + 2 * NW, 0);
    __builtin_amdgcn_sched_group_barrier(MFMA, N / 2, 0);
#pragma unroll
    for (int k = 0; k < N / 2; ++k) {
        __builtin_amdgcn_sched_group_barrier(VALU, N >= 8 ? 3 : 6, 0);
        __builtin_amdgcn_sched_group_barrier(MFMA, 1, 0);
    }
}

// One step: acc[i][m] += T(32 m) A0[i] + T(32 m + 32) A1[i] for the 2 R M-blocks m,
// with F[q] = T(32 q), q = 0 .. 2 R.  The first MFMA of every accumulator goes out
// before the second one of any, so that independent MFMAs separate each pair.
template <int NW, int R>
__device__ __forceinline__ void mfma_step(v16i (&acc)[NW][2 * R], const v4i (&F)[2 * R + 1], const v4i (&A0)[NW],
                                          const v4i (&A1)[NW]) {
#pragma unroll
    for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int m = 0; m < 2 * R; ++m) acc[i][m] = __builtin_amdgcn_mfma_i32_32x32x32_i8(F[m], A0[i], acc[i][m], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int m = 0; m < 2 * R; ++m)
            acc[i][m] = __builtin_amdgcn_mfma_i32_32x32x32_i8(F[m + 1], A1[i], acc[i][m], 0, 0, 0);
}

// Registers capped at 168, so that three workgroups share a CU (three waves per SIMD)
// when the staging window is at most 234 steps (224 by default); a few values of the
// set-up and the epilogue spill, nothing in the step loop.  The third wave pays at
// mid sizes (4096 limbs: 224 steps 2% faster than 256); on 16384-limb products the
// capped code is fastest with 256 steps at two workgroups per CU.
template <int NW, int R, bool SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_mul_large_mfma(
    const u64 *__restrict__ a, const u64 *__restrict__ b, u64 na, u64 nb, u64 npairs, const u64 *__restrict__ tops,
    u32 D, u32 ngroups, u32 nslices, u64 *__restrict__ LO, u64 *__restrict__ HS, int *__restrict__ part) {
    extern __shared__ u64 lds[];
    u64 *bz = lds;                         // 8 (D + 2 + R) words of signed b digits
    u64 *az = lds + 8 * ((u64)D + 2 + R);  // (128 NW R + D) chunk slots of reversed signed a digits
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar branches below
    const u32 x = lane & 31, h = lane >> 5;
    // block -> (slice, group, pair); groups in decreasing-work order
    const u64 slice = SPLIT ? blockIdx.x % nslices : 0;
    const u64 bq = SPLIT ? blockIdx.x / nslices : blockIdx.x;
    const u64 pair = bq % npairs;
    const u32 g = middle_out((u32)(bq / npairs), ngroups);
    const i64 P = (i64)(na + nb);
    // a and b (the converted operands) have 8 n + 1 digits each, the last one the top
    // carry, stored in tops[pair] (a) and tops[npairs + pair] (b)
    const i64 nca = (8 * (i64)na + 64) / 64;  // 64-digit chunks of a
    // steps d in [dmin, dmax] reach b digits: rows r < 64 R of step d read digits from
    // 64 (d - 1) + 1 up to 64 d + 64 R - 1
    const i64 dmin = 1 - R, dmax = (8 * (i64)nb + 63) / 64;
    const i64 nWb = (P + 256 * R - 1) / (256 * R);
    const i64 wb0 = (i64)g * 4 * NW;
    const i64 W0g = 32 * wb0, Wend = W0g + 128 * NW - 1;
    const u64 *pa = a + pair * na, *pb = b + pair * nb;
    const u64 top_a = tops[pair], top_b = tops[npairs + pair];

    // a chunk c = R W - d meets column group W at step d
    i64 wlo = INT64_MAX, whi = INT64_MIN;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const i64 wb = wb0 + (i64)wave * NW + i;
        if (wb < nWb) {
            const i64 blo = std::max<i64>(dmin, R * 32 * wb - nca + 1);
            const i64 bhi = std::min<i64>(dmax, R * (32 * wb + 31));
            if (blo <= bhi) {
                wlo = std::min(wlo, blo);
                whi = std::max(whi, bhi);
            }
        }
    }
    const i64 lastb = std::min<i64>(wb0 + 4 * NW, nWb) - 1;
    i64 ulo = std::max<i64>(dmin, R * W0g - nca + 1);
    i64 uhi = std::min<i64>(dmax, R * (32 * lastb + 31));
    const i64 ulo_all = ulo, uhi_all = uhi;
    if (SPLIT) {
        // this workgroup's slice of the contraction range: an even number of steps, at
        // most 2046 (exact int32 sums)
        const i64 sl = (((dmax - dmin + (i64)nslices) / (i64)nslices) + 1) & ~(i64)1;
        ulo = std::max<i64>(ulo, dmin + (i64)slice * sl);
        uhi = std::min<i64>(uhi, dmin + (i64)slice * sl + sl - 1);
    }
    // Steps run in pairs.  A step outside every block's own range adds zero (its a
    // chunks or b digits are zero-padded), so an odd range grows by one such step at
    // an end where the workgroup's blocks end; a slice boundary in the middle of the
    // blocks' ranges stays put (slices of even length then meet there).
    if (ulo <= uhi && ((uhi - ulo) & 1) == 0) {
        if (uhi == uhi_all) ++uhi;
        else if (ulo == ulo_all) --ulo;
    }

    v16i acc[NW][2 * R];
#pragma unroll
    for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int m = 0; m < 2 * R; ++m) acc[i][m] = v16i{0};
    const u32 *bz32 = reinterpret_cast<const u32 *>(bz);
    const u32 nbz = 8 * (D + 2 + R);

    for (i64 d0 = ulo; d0 <= uhi; d0 += D) {
        const i64 d1 = std::min<i64>(d0 + D - 1, uhi);
        const i64 cbase = R * W0g - d1;
        const i64 nslots = R * Wend - d0 - cbase + 1;
        __syncthreads();
        // Staging, SG elements per thread at a time: unconditional loads from clamped
        // indices first (no branch between a load and its use, so one wait per group),
        // then the bytes turned into signed digits (xor 0x80), the limb past the operand
        // replaced by the top digit and the others out of range by zero.
        constexpr int SG = 8;
        for (u32 k0 = threadIdx.x; k0 < nbz; k0 += 256 * SG) {
            u64 v[SG];
#pragma unroll
            for (int j = 0; j < SG; ++j) {
                const i64 m = 8 * (d0 - 1) + (i64)(k0 + 256 * j);
                v[j] = pb[std::min<i64>(std::max<i64>(m, 0), (i64)nb - 1)];
            }
#pragma unroll
            for (int j = 0; j < SG; ++j) {
                const u32 k = k0 + 256 * j;
                const i64 m = 8 * (d0 - 1) + (i64)k;
                if (k < nbz) bz[k] = (m >= 0 && m < (i64)nb) ? (v[j] ^ XOR80) : (m == (i64)nb ? top_b : 0ull);
            }
        }
        for (u32 k0 = threadIdx.x; k0 < 8 * nslots; k0 += 256 * SG) {
            u64 v[SG];
#pragma unroll
            for (int j = 0; j < SG; ++j) {
                const u32 k = k0 + 256 * j;
                const i64 m = 8 * (cbase + (i64)(k >> 3)) + 7 - (i64)(k & 7);
                v[j] = pa[std::min<i64>(std::max<i64>(m, 0), (i64)na - 1)];
            }
#pragma unroll
            for (int j = 0; j < SG; ++j) {
                const u32 k = k0 + 256 * j;
                const i64 m = 8 * (cbase + (i64)(k >> 3)) + 7 - (i64)(k & 7);
                if (k < 8 * nslots)
                    az[AZ_SLOT_U64 * (k >> 3) + (k & 7)] =
                        (m >= 0 && m < (i64)na) ? __builtin_bswap64(v[j] ^ XOR80)
                                                : (m == (i64)na ? __builtin_bswap64(top_a) : 0ull);
            }
        }
        __syncthreads();
        i64 dlo = std::max(d0, wlo), dhi = std::min(d1, whi);
        if (dlo <= dhi) {
            // an even step count: grow by a step past the wave's blocks, inside the round
            if (((dhi - dlo) & 1) == 0) {
                if (dhi < d1) ++dhi;
                else if (dlo > d0) --dlo;
            }
            // Two steps per trip with two register sets (X, Y): while one step's MFMAs
            // run, the LDS reads of the next step land in the other set, a whole step
            // ahead of their use.  The byte shift is the same for every fragment of a
            // lane.  Fragment T(d, 32 q) is 8 q words after T(d, 0), and T(d + 1, 32 q)
            // = T(d, 32 q + 64): step d + 1 needs two new fragments, T(d, 64 R + 32) and
            // T(d, 64 R + 64).
            const u32 sh = (x + 1) & 3u;
            const u32 lane_off = x + 1 + 16 * h;
            // Running LDS pointers: pT = fragment T(d, 0) in bz (a step moves it by 16
            // words), pA[i] = block i's a chunk slot at step d + 2 in az (a step moves
            // it back one slot; the trip's reads sit at non-negative offsets from it).
            // The reads for step d + 2 in the last trip may lie one step past dhi: still
            // inside the staged arrays (b digits up to step d1 + 1 + R are staged; slot
            // -1 is the end of bz), unused.
            lds_cptr<u32> pT = (lds_cptr<u32>)bz32 + (lane_off >> 2) + 16 * (int)(dlo - d0);
            lds_cptr<u64> pA[NW];
#pragma unroll
            for (int i = 0; i < NW; ++i)
                pA[i] = (lds_cptr<u64>)az +
                        AZ_SLOT_U64 * (int)(R * (32 * (wb0 + (i64)wave * NW + i) + (i64)x) - cbase - dlo - 2) + 2 * (int)h;
            v4i F[2 * R + 1], G[2 * R + 1];
            v4i AX0[NW], AX1[NW], AY0[NW], AY1[NW];
            // prologue: step dlo's fragments into F, its a fragments into AX
            // (volatile: keeps the compiler from merging these reads with the loop's
            // reads of the same registers into one read at the top of the loop)
#pragma unroll
            for (int q = 0; q <= 2 * R; ++q) F[q] = toeplitz_combine(tw_at(pT, 8 * q), sh);
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                AX0[i] = *(const volatile __attribute__((address_space(3))) v4i *)(pA[i] + 2 * AZ_SLOT_U64);
                AX1[i] = *(const volatile __attribute__((address_space(3))) v4i *)(pA[i] + 2 * AZ_SLOT_U64 + 4);
            }
            // Every block of the wave runs every step of the wave's range: outside a
            // block's own range its a chunks are zero-padded in LDS, so those MFMAs add
            // zero.  No branches around MFMAs (the compiler would copy the
            // accumulators).  One basic block per trip.
            for (i64 d = dlo; d <= dhi; d += 2) {
                // ---- step d on X; reads of step d + 1 into Y ----
                const TWords ty1 = tw_at(pT, 16 * R + 8);
                const TWords ty2 = tw_at(pT, 16 * R + 16);
#pragma unroll
                for (int i = 0; i < NW; ++i) {
                    AY0[i] = *(lds_cptr<v4i>)(pA[i] + AZ_SLOT_U64);
                    AY1[i] = *(lds_cptr<v4i>)(pA[i] + AZ_SLOT_U64 + 4);
                }
                mfma_step<NW, R>(acc, F, AX0, AX1);
#pragma unroll
                for (int q = 0; q + 2 <= 2 * R; ++q) G[q] = F[q + 2];
                G[2 * R - 1] = toeplitz_combine(ty1, sh);
                G[2 * R] = toeplitz_combine(ty2, sh);
                mfma_step_order<NW, R>();
                // ---- step d + 1 on Y; reads of step d + 2 into X ----
                const TWords tx1 = tw_at(pT, 16 * R + 24);
                const TWords tx2 = tw_at(pT, 16 * R + 32);
#pragma unroll
                for (int i = 0; i < NW; ++i) {
                    AX0[i] = *(lds_cptr<v4i>)(pA[i]);
                    AX1[i] = *(lds_cptr<v4i>)(pA[i] + 4);
                }
                mfma_step<NW, R>(acc, G, AY0, AY1);
#pragma unroll
                for (int q = 0; q + 2 <= 2 * R; ++q) F[q] = G[q + 2];
                F[2 * R - 1] = toeplitz_combine(tx1, sh);
                F[2 * R] = toeplitz_combine(tx2, sh);
                pT += 32;
#pragma unroll
                for (int i = 0; i < NW; ++i) pA[i] -= 2 * AZ_SLOT_U64;
                mfma_step_order<NW, R>();
            }
        }
    }

    if (SPLIT) {
        // this slice's column sums (exact int32) -> its own partial array, every column
        // of the workgroup's blocks written (zeros for an empty slice); a fold kernel
        // adds the slices
        int *pc = part + ((u64)slice * npairs + pair) * 8 * (u64)P;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const i64 wb = wb0 + (i64)wave * NW + i;
            if (wb >= nWb) continue;
#pragma unroll
            for (int mi = 0; mi < 2 * R; ++mi)
#pragma unroll
                for (int gg = 0; gg < 16; ++gg) {
                    const u64 t = 64 * R * ((u64)(32 * wb) + x) + 32 * mi + acc_row(gg, lane);
                    if (t < 8 * (u64)P) pc[t] = acc[i][mi][gg];
                }
        }
        return;
    }
    // ---- epilogue: exact column sums -> signed limb values -> lo / shifted hi ----
    // Lane (x, h) holds, for each of its blocks, columns t = 64 R W + 32 mi + 8 m + 4 h + ii
    // (W = 32 wb + x): limb jl = 4 mi + m of W's 8 R, digits u = 4 h + ii.  M-blocks
    // pair up (mi = 2 s, 2 s + 1): lane h keeps limb 8 s + 4 h + m and takes the other
    // half of its digits from the partner lane (lane xor 32).  A column sum lies in
    // [-16256 cnt, 16384 cnt] with cnt <= cmax digit pairs; the register holds it
    // modulo 2^32, and only the upper end can pass 2^31 (cmax <= 131586), so one
    // comparison with -16256 cmax recovers it.  The limb value V_j = sum_u C_(8j+u) 256^u
    // is signed, |V_j| < 2^90; it is stored as V_j + K 2^64 - [j > 0] K (K = 2^62, so
    // lo and hi are unsigned): the offsets telescope to K X^P, zero modulo X^P, so the
    // carry pass still gives the product.
    const i64 lowest = -16256 * (8 * (i64)std::min(na, nb) + 1);
    u64 *lo_out = LO + pair * (u64)P, *hs_out = HS + pair * (u64)P;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const i64 wb = wb0 + (i64)wave * NW + i;
        if (wb >= nWb) continue;
        const u64 W = (u64)(32 * wb) + x;
#pragma unroll
        for (int s = 0; s < R; ++s) {
            // the lane's four columns of limb (e, m): |sum| < 2^32 2^24 (4/3) < 2^57
            i64 w[2][4];
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    i64 ws = 0;
#pragma unroll
                    for (int ii = 0; ii < 4; ++ii) {
                        i64 c = (i64)acc[i][2 * s + e][4 * m + ii];
                        if (c < lowest) c += (i64)1 << 32;
                        ws += c * ((i64)1 << (8 * ii));
                    }
                    w[e][m] = ws;
                }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const i64 keep = h ? w[1][m] : w[0][m];
                const i64 got = (i64)__shfl_xor((u64)(h ? w[0][m] : w[1][m]), 32);
                const i64 lo4 = h ? got : keep, hi4 = h ? keep : got;  // digits 0..3, 4..7
                const u64 j = 8 * R * W + 8 * s + 4 * h + m;
                const u128 V = (u128)(__int128)lo4 + ((u128)(__int128)hi4 << 32) + ((u128)MUL_BIAS << 64) -
                               (j > 0 ? (u128)MUL_BIAS : (u128)0);
                if (j < (u64)P) {
                    lo_out[j] = (u64)V;
                    if (j + 1 < (u64)P) hs_out[j + 1] = (u64)(V >> 64);
                    if (j == 0) hs_out[0] = 0;
                }
            }
        }
    }
}

// Slice sums from the split MFMA kernel (each exact as int32) -> signed limb values
// -> biased lo / shifted hi, as the unsplit epilogue stores them.
__global__ void k_fold_mfma_cols(const int *__restrict__ part, u32 nslices, u64 P, u64 npairs, u64 *__restrict__ LO,
                                 u64 *__restrict__ HS) {
    const u64 total = P * npairs, sstride = npairs * 8 * P;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 j = idx % P;
        const int *pc = part + 8 * idx;
        i64 m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (u32 sl = 0; sl < nslices; ++sl)
#pragma unroll
            for (int u = 0; u < 8; ++u) m[u] += pc[sl * sstride + u];
        // |m| <= 2^14 (8 min(na, nb) + 1) < 2^39 for any operand that fits the device
        __int128 v = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) v += (__int128)m[u] * ((__int128)1 << (8 * u));
        const u128 V = (u128)v + ((u128)MUL_BIAS << 64) - (j > 0 ? (u128)MUL_BIAS : (u128)0);
        LO[idx] = (u64)V;
        if (j + 1 < P) HS[idx + 1] = (u64)(V >> 64);
        if (j == 0) HS[idx] = 0;
    }
}

// ---------------------------------------------------------------- workspace ----
struct LargeLayout {
    size_t colLo, colHi, part, ca, cb, tops, LO, HS, total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static LargeLayout large_layout(u64 na, u64 nb, u64 npairs, int form, u32 nslices) {
    const bool split = nslices > 1;
    LargeLayout L{};
    const u64 P = na + nb;
    size_t off = 0;
    if (form == BN_MUL_MAD) {
        L.colLo = off;
        off = align256(off + npairs * 2 * P * 8);
        L.colHi = off;
        off = align256(off + npairs * 2 * P * 8);
    } else {
        if (split) {
            L.part = off;
            off = align256(off + (size_t)nslices * npairs * 8 * P * 4);
        }
        L.ca = off;  // converted operands (balanced digits), same layout as a and b
        off = align256(off + npairs * na * 8);
        L.cb = off;
        off = align256(off + npairs * nb * 8);
        L.tops = off;  // their top digits: a's for every pair, then b's
        off = align256(off + npairs * 2 * 8);
    }
    L.LO = off;
    off = align256(off + npairs * P * 8);
    L.HS = off;
    off = align256(off + npairs * P * 8);
    L.total = off;
    return L;
}

}  // namespace

// Contraction slices for the large MFMA kernel: enough workgroups to fill the device
// (about four per CU), slices of at least 128 steps, and at most 2046 steps per slice
// when the int32 slice sums need it.
struct MfmaPlan {
    u64 ngroups;
    u32 nslices;
};
static MfmaPlan mfma_plan(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs) {
    const u64 P = na + nb;
    MfmaPlan mp{(P + 2047) / 2048, 1};  // a workgroup covers 2048 output limbs
    const u64 steps = (8 * nb + 63) / 64 + (u64)ctx->tune.mfma_rows;  // d from 1 - R to dmax
    const u64 blocks = mp.ngroups * npairs;
    const u64 target = (u64)std::max(1, ctx->num_cu) * 4;
    // digit products in a column: at most the shorter operand's digit count (8 n + 1
    // balanced digits)
    const u64 maxcnt = 8 * std::min(na, nb) + 1;
    u64 S = 1;
    if (blocks < target) S = std::max<u64>(1, std::min<u64>((target + blocks - 1) / blocks, (steps + 127) / 128));
    // a slice sum is added to the workspace as a plain int32: |sum| <= 2^14 cnt must stay
    // below 2^31, so slices longer than 2047 steps need cnt <= 131071 (slices are
    // rounded up to an even length: at most 2046 steps)
    if (S > 1 && maxcnt > 131071) S = std::max<u64>(S, (steps + 2045) / 2046);
    // an unsplit launch decodes its int32 sums exactly while cnt <= 131586
    if (S == 1 && maxcnt > 131586) S = std::max<u64>(2, (steps + 2045) / 2046);
    mp.nslices = (u32)S;
    return mp;
}

bool mul_small_range(u64 P) { return P <= SMALL_MAX_P; }

// Staging window of the large MFMA kernel: the tuned value, or by size: 224 steps
// (three workgroups per CU) unless the launch is unsplit with long contractions
// (shorter operand >= 10240 limbs), where the rounds of 256 steps at two workgroups
// per CU are faster (interleaved measurements: 2048 - 8192 limbs 224 faster by 2-7%,
// 12288 and 16384 limbs 256 faster by 2%, one split 16500-limb product 224 by 1%).
static u32 mfma_window(const bn_ctx *ctx, u64 na, u64 nb, u32 nslices) {
    if (ctx->tune.mfma_chunk) return (u32)ctx->tune.mfma_chunk;
    return (std::min(na, nb) >= 10240 && nslices == 1) ? 256u : 224u;
}

int mul_pick_form(const bn_ctx *ctx, u64 na, u64 nb, int form) {
    if (form != BN_MUL_AUTO) return form;
    // products of at most 1024 limbs (mad: one wave; MFMA: one wave up to 512 limbs)
    // and larger ones (column-workspace kernels) have a crossover each; products of at
    // most 64, 65-128, 129-256, 257-512 and 513-1024 limbs may have their own (the mad
    // form's lanes hold 1, 2, 4, 8 or 16 limbs there while its steps follow the shorter
    // operand; the MFMA form runs 1, 2 or 4 column blocks in one wave, then the
    // workspace kernels)
    const u64 P = na + nb;
    i64 x = mul_small_range(P) ? ctx->tune.mul_small_crossover_limbs : ctx->tune.mul_crossover_limbs;
    const i64 cls = P <= 64 ? ctx->tune.mul_crossover_p64 : P <= 128 ? ctx->tune.mul_crossover_p128
                  : P <= 256 ? ctx->tune.mul_crossover_p256 : P <= 512 ? ctx->tune.mul_crossover_p512
                  : mul_small_range(P) ? ctx->tune.mul_crossover_p1024 : -1;
    if (cls >= 0) x = cls;
    return (i64)std::min(na, nb) >= x ? BN_MUL_MFMA : BN_MUL_MAD;
}

size_t mul_workspace_bytes(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs, int form) {
    if (na == 0 || nb == 0 || npairs == 0) return 0;
    form = mul_pick_form(ctx, na, nb, form);
    if (mul_one_wave(na + nb, form)) return 0;
    return large_layout(na, nb, npairs, form, form == BN_MUL_MFMA ? mfma_plan(ctx, na, nb, npairs).nslices : 1u).total;
}

size_t mul_status_bytes(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs, int form) {
    if (na == 0 || nb == 0 || npairs == 0) return 0;
    form = mul_pick_form(ctx, na, nb, form);
    if (mul_one_wave(na + nb, form)) return 0;
    size_t bytes = flat_scan_status_bytes(ctx, na + nb, (na + nb) * npairs);  // the carry pass
    if (form == BN_MUL_MFMA)  // the operand conversions (one two-part launch for equal lengths)
        bytes = std::max({bytes, flat_scan_ext_status_bytes(na, na * npairs), flat_scan_ext_status_bytes(nb, nb * npairs),
                          na == nb ? flat_scan_ext_status_bytes(na, 2 * na * npairs) : (size_t)0});
    return bytes;
}

bn_status launch_mul_batch(bn_ctx *ctx, u64 *r, const u64 *a, const u64 *b, u64 na, u64 nb, u64 npairs, int form,
                           hipStream_t s) {
    if (npairs == 0) return BN_OK;
    const u64 P = na + nb;
    if (na == 0 || nb == 0) return launch_fill_u64(r, P * npairs, 0, s);
    form = mul_pick_form(ctx, na, nb, form);
    if (mul_one_wave(P, form)) {
        const u64 blocks = (npairs + 3) / 4;
        if (blocks > 0x7fffffffull) return BN_ERANGE;
        if (form == BN_MUL_MFMA && P <= 128)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MFMA, 1>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else if (form == BN_MUL_MFMA && P <= 256)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MFMA, 2>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else if (form == BN_MUL_MFMA)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MFMA, 4>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else if (P <= 64)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MAD, 1>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else if (P <= 128)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MAD, 2>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else if (P <= 256)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MAD, 4>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else if (P <= 512)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MAD, 8>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MAD, 16>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        return bn_launch_status();
    }
    const MfmaPlan mp = mfma_plan(ctx, na, nb, npairs);
    const bool split = form == BN_MUL_MFMA && mp.nslices > 1;
    const LargeLayout L = large_layout(na, nb, npairs, form, split ? mp.nslices : 1u);
    bn_status st = bn_ensure(ctx, ctx->work, L.total, s);
    if (st != BN_OK) return st;
    char *ws = static_cast<char *>(ctx->work.ptr);
    u64 *LO = reinterpret_cast<u64 *>(ws + L.LO);
    u64 *HS = reinterpret_cast<u64 *>(ws + L.HS);
    const u64 total = P * npairs;
    u64 fold_blocks = std::min<u64>((total + 255) / 256, 65536);
    if (form == BN_MUL_MAD) {
        u64 *colLo = reinterpret_cast<u64 *>(ws + L.colLo);
        u64 *colHi = reinterpret_cast<u64 *>(ws + L.colHi);
        if ((st = launch_fill_u64(colLo, (L.colHi - L.colLo) / 8 + npairs * 2 * P, 0, s)) != BN_OK) return st;
        constexpr int Q = 16;
        const u64 ncb = (2 * P + 64 * Q - 1) / (64 * Q);
        // digits of a per work item: the tuned slice, smaller when there are too few
        // items to give every SIMD several waves
        u32 XC = (u32)ctx->tune.mad_xchunk;
        const u64 want = (u64)std::max(1, ctx->num_cu) * 32;
        const u64 per_slice = ncb * npairs;
        if (per_slice * ((2 * na + XC - 1) / XC) < want) {
            const u64 nx_wanted = (want + per_slice - 1) / per_slice;
            XC = (u32)std::max<u64>(256, ((2 * na + nx_wanted - 1) / nx_wanted + 63) / 64 * 64);
        }
        const u64 nxc = (2 * na + XC - 1) / XC;
        const u64 nitems = ncb * nxc;
        const u64 blocks = (nitems + 3) / 4;
        if (blocks > 0x7fffffffull) return BN_ERANGE;
        for (u64 p0 = 0; p0 < npairs; p0 += 65535) {  // grid.y holds the pair
            const u64 np = std::min<u64>(65535, npairs - p0);
            hipLaunchKernelGGL((k_mul_large_mad<Q>), dim3((u32)blocks, (u32)np), dim3(256), 0, s, a + p0 * na,
                               b + p0 * nb, na, nb, nxc, nitems, XC, colLo + p0 * 2 * P, colHi + p0 * 2 * P);
            if ((st = bn_launch_status()) != BN_OK) return st;
        }
        hipLaunchKernelGGL(k_fold_mad, dim3((u32)fold_blocks), dim3(256), 0, s, colLo, colHi, P, total, LO, HS);
        if ((st = bn_launch_status()) != BN_OK) return st;
    } else {
        u64 *ca = reinterpret_cast<u64 *>(ws + L.ca);
        u64 *cb = reinterpret_cast<u64 *>(ws + L.cb);
        u64 *tops = reinterpret_cast<u64 *>(ws + L.tops);
        // balanced digits: every operand + 0x80...80, the carries out as top digits (both
        // operands in one two-part launch when their lengths agree)
        if (na == nb) {
            ScanPart2 bside;
            bside.r = cb;
            bside.a = b;
            bside.npairs = npairs;
            if ((st = launch_flat_scan_mem(ctx, false, ca, a, nullptr, na, npairs, nullptr, true, XOR80, tops, s,
                                           nullptr, -1, nullptr, &bside)) != BN_OK)
                return st;
        } else {
            if ((st = launch_flat_scan_ext(ctx, false, ca, a, nullptr, na, npairs, nullptr, true, XOR80, tops, s)) !=
                BN_OK)
                return st;
            if ((st = launch_flat_scan_ext(ctx, false, cb, b, nullptr, nb, npairs, nullptr, true, XOR80, tops + npairs,
                                           s)) != BN_OK)
                return st;
        }
        // (blocks per wave, Toeplitz row groups): both shapes cover 2048 output limbs
        // per workgroup and stage the same LDS window
        const int R = ctx->tune.mfma_rows;
        const int NW = 2 / R;
        const u32 D = mfma_window(ctx, na, nb, split ? mp.nslices : 1u);
        const u64 blocks = mp.ngroups * npairs * mp.nslices;
        if (blocks > 0x7fffffffull) return BN_ERANGE;
        const size_t lds = (size_t)64 * (D + 2 + R) + (size_t)80 * (128 * NW * R + D);
        int *part = split ? reinterpret_cast<int *>(ws + L.part) : nullptr;
        auto kern = R == 2 ? (split ? k_mul_large_mfma<1, 2, true> : k_mul_large_mfma<1, 2, false>)
                           : (split ? k_mul_large_mfma<2, 1, true> : k_mul_large_mfma<2, 1, false>);
        hipLaunchKernelGGL(kern, dim3((u32)blocks), dim3(256), lds, s, ca, cb, na, nb, npairs, tops, D,
                           (u32)mp.ngroups, split ? mp.nslices : 1u, LO, HS, part);
        if (split) {
            if ((st = bn_launch_status()) != BN_OK) return st;
            hipLaunchKernelGGL(k_fold_mfma_cols, dim3((u32)fold_blocks), dim3(256), 0, s, part, mp.nslices, P, npairs,
                               LO, HS);
        }
        if ((st = bn_launch_status()) != BN_OK) return st;
    }
    // deferred carry pass: r = LO + HS (1-bit carries), segments of P limbs
    return launch_flat_scan(ctx, false, r, LO, HS, P, npairs, nullptr, s);
}
