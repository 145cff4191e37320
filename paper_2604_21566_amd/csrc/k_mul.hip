// k_mul.hip -- multiplication kernels and the uniform-batch dispatcher.
//
// Small products (na + nb <= 256 limbs): one wave per pair does everything --
// column products, fold, and the in-wave carry pass -- with no workspace.
// Large products: a product kernel accumulates column sums into a workspace with
// atomics (work items = output-column block x slice of the contraction range, so
// every item has about the same work), a fold kernel turns column sums into
// per-limb (lo, hi) pairs, and the deferred carry pass is the add kernel itself:
// r = LO + (HI shifted up one limb).
#include "bn_mul_dev.h"

#include <algorithm>

namespace {

constexpr u64 XOR80 = 0x8080808080808080ull;

// -------------------------------------------------------------- small kernels ----

// Uniform batch of small products: wave w of block blk handles pair 4*blk + w.
template <int FORM, int L>
__global__ __launch_bounds__(256) void k_mul_small(u64 *__restrict__ r, const u64 *__restrict__ a,
                                                   const u64 *__restrict__ b, u32 na, u32 nb, u64 npairs) {
    __shared__ u64 lds[FORM == BN_MUL_MFMA ? 4 * SMALL_MFMA_LDS_U64 : 1];
    const int w = threadIdx.x >> 6;
    const u64 p = (u64)blockIdx.x * 4 + w;
    if (p >= npairs) return;
    const u64 *pa = a + p * na;
    const u64 *pb = b + p * nb;
    u64 *pr = r + p * (u64)(na + nb);
    if (FORM == BN_MUL_MFMA)
        mul_item_mfma_small(pa, na, pb, nb, pr, lds + w * SMALL_MFMA_LDS_U64);
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
    for (i64 xb = xs; xb < xe; xb += Q) {
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const i64 x = xb + s;
            const u32 al = x < xe ? a32[x] : 0u;
#pragma unroll
            for (int q = 0; q < Q; ++q) mac96(lo[q], hi[q], al, R[(q - s + Q) % Q]);
            const i64 yf = T0 - x - 1;
            const u32 fill = (yf >= 0 && yf < ny) ? b32[yf] : 0u;
            const int k = (Q - 1 - s + Q) % Q;
            R[k] = (u32)__builtin_amdgcn_update_dpp((int)fill, (int)R[k], BN_DPP_WAVE_SHR1, 0xf, 0xf, false);
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
constexpr int AR_PAD = 128;  // zero limbs on each side of the reversed digit array (32 chunks)

// Per pair: digit prefix tables of a and b, and the reversed signed digits of a with
// zero padding.  One workgroup per pair.
__device__ void block_prefix_digits(const u64 *__restrict__ limbs, u64 n, u32 *__restrict__ lp, u32 *sh) {
    const u32 tid = threadIdx.x, nt = blockDim.x;
    const u64 per = (n + nt - 1) / nt;
    const u64 lo = std::min<u64>(n, tid * per), hi = std::min<u64>(n, lo + per);
    u32 s = 0;
    for (u64 k = lo; k < hi; ++k) s += bytesum64(limbs[k]);
    sh[tid] = s;
    __syncthreads();
    if (tid == 0) {
        u32 run = 0;
        for (u32 i = 0; i < nt; ++i) {
            const u32 v = sh[i];
            sh[i] = run;
            run += v;
        }
    }
    __syncthreads();
    u32 run = sh[tid];
    for (u64 k = lo; k < hi; ++k) {
        lp[k] = run;
        run += bytesum64(limbs[k]);
    }
    if (hi == n && lo < hi) lp[n] = run;
    if (n == 0 && tid == 0) lp[0] = 0;
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_mfma_prep(const u64 *__restrict__ a, const u64 *__restrict__ b, u64 na,
                                                   u64 nb, u32 *__restrict__ lpa, u32 *__restrict__ lpb,
                                                   u64 *__restrict__ aR) {
    __shared__ u32 sh[256];
    const u64 p = blockIdx.x;
    const u64 *pa = a + p * na, *pb = b + p * nb;
    block_prefix_digits(pa, na, lpa + p * (na + 1), sh);
    block_prefix_digits(pb, nb, lpb + p * (nb + 1), sh);
    const u64 nca = (na + 3) / 4;
    const u64 len = 4 * nca + 2 * AR_PAD;
    u64 *dst = aR + p * len;
    for (u64 k = threadIdx.x; k < len; k += blockDim.x) {
        u64 v = 0;
        if (k >= (u64)AR_PAD && k < AR_PAD + 4 * nca) {
            const u64 m = 4 * nca - 1 - (k - AR_PAD);
            if (m < na) v = __builtin_bswap64(pa[m] ^ XOR80);
        }
        dst[k] = v;
    }
}

// Work item (one workgroup of 4 waves): W-blocks [4 NW g, 4 NW (g+1)) (each 32 output
// groups of 32 digit columns) x Toeplitz steps d in [k D, (k+1) D).  The b digits of
// the step range are staged once in LDS and shared by all waves; each wave builds
// the Toeplitz fragment once per step and uses it for its NW blocks.
template <int NW>
__global__ __launch_bounds__(256) void k_mul_large_mfma(const u64 *__restrict__ b, const u64 *__restrict__ aR, u64 na,
                                                        u64 nb, u64 nchunks, u32 D, u64 *__restrict__ col) {
    extern __shared__ u64 bz[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u32 x = lane & 31, h = lane >> 5;
    const u64 pair = blockIdx.y;
    const u64 g = blockIdx.x / nchunks, kc = blockIdx.x % nchunks;
    const i64 nca = (i64)((na + 3) / 4);
    const i64 ndb = 8 * (i64)nb;
    const i64 dmax = (ndb + 30) / 32;
    const i64 d0 = (i64)kc * D;
    const i64 d1 = std::min<i64>(d0 + D, dmax + 1);
    const i64 P = (i64)(na + nb);
    const i64 nWb = (8 * P + 1023) / 1024;  // W-blocks holding output columns
    const i64 wbFirst = (i64)g * 4 * NW;
    const i64 wbLast = std::min<i64>(wbFirst + 4 * NW, nWb) - 1;
    // union of useful steps over the group's blocks: d in [32 Wb - nca + 1, 32 Wb + 31]
    const i64 ulo = std::max<i64>(d0, 32 * wbFirst - nca + 1);
    const i64 uhi = std::min<i64>(d1 - 1, 32 * wbLast + 31);
    if (ulo > uhi) return;

    const u64 *pb = b + pair * nb;
    const u32 nst = 4 * (D + 3);
    for (u32 k = threadIdx.x; k < nst; k += blockDim.x) {
        const i64 m = 4 * (d0 - 1) + (i64)k;
        bz[k] = (m >= 0 && m < (i64)nb) ? (pb[m] ^ XOR80) : 0ull;
    }
    __syncthreads();

    const u64 *ar = aR + pair * (4 * (u64)nca + 2 * AR_PAD) + AR_PAD;
    const u32 *bz32 = reinterpret_cast<const u32 *>(bz);
    v16i acc[NW];
    i64 blo[NW], bhi[NW];
    i64 wlo = INT64_MAX, whi = INT64_MIN;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        acc[i] = v16i{0};
        const i64 wb = wbFirst + (i64)wave * NW + i;
        blo[i] = std::max<i64>(d0, 32 * wb - nca + 1);
        bhi[i] = (wb < nWb) ? std::min<i64>(d1 - 1, 32 * wb + 31) : INT64_MIN;
        if (blo[i] <= bhi[i]) {
            wlo = std::min(wlo, blo[i]);
            whi = std::max(whi, bhi[i]);
        }
    }
    for (i64 d = wlo; d <= whi; ++d) {
        const v4i T = toeplitz_frag(bz32, (u32)(32 * (d - d0)) + x + 1 + 16 * h);
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            if (d >= blo[i] && d <= bhi[i]) {
                const i64 wb = wbFirst + (i64)wave * NW + i;
                const i64 c = 32 * wb + (i64)x - d;  // in [-31, nca + 30]
                const v4i A = *reinterpret_cast<const v4i *>(ar + 4 * nca - 4 * (c + 1) + 2 * h);
                acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(T, A, acc[i], 0, 0, 0);
            }
        }
    }
    u64 *pc = col + pair * 8 * (u64)P;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        if (blo[i] > bhi[i]) continue;
        const i64 wb = wbFirst + (i64)wave * NW + i;
#pragma unroll
        for (int gg = 0; gg < 16; ++gg) {
            const u64 t = 32ull * (u64)(32 * wb + x) + acc_row(gg, lane);
            const int v = acc[i][gg];
            if (t < 8ull * (u64)P && v != 0)
                __hip_atomic_fetch_add(pc + t, (u64)(i64)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Signed-digit column sums (8-bit columns) -> exact unsigned sums -> per-limb lo/shifted hi.
__global__ void k_fold_mfma(const u64 *__restrict__ col, const u64 *__restrict__ a, const u64 *__restrict__ b,
                            const u32 *__restrict__ lpa, const u32 *__restrict__ lpb, u64 na, u64 nb, u64 total,
                            u64 *__restrict__ LO, u64 *__restrict__ HS) {
    const u64 P = na + nb;
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < total; idx += (u64)gridDim.x * blockDim.x) {
        const u64 p = idx / P, j = idx - p * P;
        const u64 *pa = a + p * na, *pb = b + p * nb;
        const u32 *la = lpa + p * (na + 1), *lb = lpb + p * (nb + 1);
        const u64 *pc = col + p * 8 * P;
        u128 V = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const u64 t = 8 * j + u;
            const i64 cf = column_fix((i64)pc[t], t, 8 * na, 8 * nb, pa, la, pb, lb);
            V += (u128)(u64)cf << (8 * u);
        }
        LO[idx] = (u64)V;
        if (j + 1 < P) HS[idx + 1] = (u64)(V >> 64);
        if (j == 0) HS[idx] = 0;
    }
}

// ---------------------------------------------------------------- workspace ----
struct LargeLayout {
    size_t colLo, colHi, col64, lpa, lpb, aR, LO, HS, total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static LargeLayout large_layout(u64 na, u64 nb, u64 npairs, int form) {
    LargeLayout L{};
    const u64 P = na + nb;
    size_t off = 0;
    if (form == BN_MUL_MAD) {
        L.colLo = off;
        off = align256(off + npairs * 2 * P * 8);
        L.colHi = off;
        off = align256(off + npairs * 2 * P * 8);
    } else {
        L.col64 = off;
        off = align256(off + npairs * 8 * P * 8);
        L.lpa = off;
        off = align256(off + npairs * (na + 1) * 4);
        L.lpb = off;
        off = align256(off + npairs * (nb + 1) * 4);
        L.aR = off;
        off = align256(off + npairs * (4 * ((na + 3) / 4) + 2 * AR_PAD) * 8);
    }
    L.LO = off;
    off = align256(off + npairs * P * 8);
    L.HS = off;
    off = align256(off + npairs * P * 8);
    L.total = off;
    return L;
}

}  // namespace

int mul_pick_form(const bn_ctx *ctx, u64 na, u64 nb, int form) {
    if (form != BN_MUL_AUTO) return form;
    return (i64)std::min(na, nb) >= ctx->tune.mul_crossover_limbs ? BN_MUL_MFMA : BN_MUL_MAD;
}

size_t mul_workspace_bytes(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs, int form) {
    if (na == 0 || nb == 0 || npairs == 0) return 0;
    form = mul_pick_form(ctx, na, nb, form);
    if (na + nb <= 256) return 0;
    return large_layout(na, nb, npairs, form).total;
}

bn_status launch_mul_batch(bn_ctx *ctx, u64 *r, const u64 *a, const u64 *b, u64 na, u64 nb, u64 npairs, int form,
                           hipStream_t s) {
    if (npairs == 0) return BN_OK;
    const u64 P = na + nb;
    if (na == 0 || nb == 0) return launch_fill_u64(r, P * npairs, 0, s);
    form = mul_pick_form(ctx, na, nb, form);
    if (P <= 256) {
        const u64 blocks = (npairs + 3) / 4;
        if (blocks > 0x7fffffffull) return BN_ERANGE;
        if (form == BN_MUL_MFMA)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MFMA, 4>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else if (P <= 64)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MAD, 1>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else if (P <= 128)
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MAD, 2>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        else
            hipLaunchKernelGGL((k_mul_small<BN_MUL_MAD, 4>), dim3((u32)blocks), dim3(256), 0, s, r, a, b, (u32)na,
                               (u32)nb, npairs);
        return bn_launch_status();
    }
    if (npairs > 65535) return BN_ERANGE;  // grid.y
    const LargeLayout L = large_layout(na, nb, npairs, form);
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
        constexpr int Q = 8;
        const u64 ncb = (2 * P + 64 * Q - 1) / (64 * Q);
        const u32 XC = (u32)ctx->tune.mad_xchunk;
        const u64 nxc = (2 * na + XC - 1) / XC;
        const u64 nitems = ncb * nxc;
        const u64 blocks = (nitems + 3) / 4;
        if (blocks > 0x7fffffffull) return BN_ERANGE;
        hipLaunchKernelGGL((k_mul_large_mad<Q>), dim3((u32)blocks, (u32)npairs), dim3(256), 0, s, a, b, na, nb, nxc,
                           nitems, XC, colLo, colHi);
        if ((st = bn_launch_status()) != BN_OK) return st;
        hipLaunchKernelGGL(k_fold_mad, dim3((u32)fold_blocks), dim3(256), 0, s, colLo, colHi, P, total, LO, HS);
        if ((st = bn_launch_status()) != BN_OK) return st;
    } else {
        u64 *col = reinterpret_cast<u64 *>(ws + L.col64);
        u32 *lpa = reinterpret_cast<u32 *>(ws + L.lpa);
        u32 *lpb = reinterpret_cast<u32 *>(ws + L.lpb);
        u64 *aR = reinterpret_cast<u64 *>(ws + L.aR);
        if ((st = launch_fill_u64(col, npairs * 8 * P, 0, s)) != BN_OK) return st;
        hipLaunchKernelGGL(k_mfma_prep, dim3((u32)npairs), dim3(256), 0, s, a, b, na, nb, lpa, lpb, aR);
        if ((st = bn_launch_status()) != BN_OK) return st;
        constexpr int NW = 2;
        const u32 D = (u32)ctx->tune.mfma_chunk;
        const u64 dmax = (8 * nb + 30) / 32;
        const u64 nchunks = (dmax + 1 + D - 1) / D;
        const u64 nWb = (8 * P + 1023) / 1024;
        const u64 ngroups = (nWb + 4 * NW - 1) / (4 * NW);
        const u64 blocks = ngroups * nchunks;
        if (blocks > 0x7fffffffull) return BN_ERANGE;
        const size_t lds = (size_t)4 * (D + 3) * 8;
        hipLaunchKernelGGL((k_mul_large_mfma<NW>), dim3((u32)blocks, (u32)npairs), dim3(256), lds, s, b, aR, na, nb,
                           nchunks, D, col);
        if ((st = bn_launch_status()) != BN_OK) return st;
        hipLaunchKernelGGL(k_fold_mfma, dim3((u32)fold_blocks), dim3(256), 0, s, col, a, b, lpa, lpb, na, nb, total,
                           LO, HS);
        if ((st = bn_launch_status()) != BN_OK) return st;
    }
    // deferred carry pass: r = LO + HS (1-bit carries), segments of P limbs
    return launch_flat_scan(ctx, false, r, LO, HS, P, npairs, nullptr, s);
}
