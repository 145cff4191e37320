// k_addsub.hip -- flat segmented add/sub as one generate/propagate prefix scan.
//
// DoT (Sec. 3.1, Algorithm 1) separates the limb-parallel work (phase 1: raw limb
// sums; phase 2: carry detection via Lemma 1) from carry resolution (phases 3-4).
// On CDNA4 the resolution is restated as a prefix scan over (generate, propagate)
// flags with three levels:
//   * inside a wave: one __ballot per flag gives 64-bit masks G and P, and the
//     Kogge-Stone style integer addition that phase 4 applies to its w-bit masks
//     resolves all 64 lanes at once: C = (((G << 1) | cin) + P) xor P is the
//     carry-into-lane mask (valid because a limb never both generates and
//     propagates);
//   * across the waves of a workgroup: their (g, p) aggregates through LDS;
//   * across workgroups: decoupled look-back over per-tile status words, in place
//     of Algorithm 1's sequential chunk-to-chunk carry (c_out of one chunk is the
//     c_in of the next).
// A batch of independent pairs is one flat array cut into segments of n limbs: a
// segment start kills propagation into its first limb and masks its carry-in, so
// the same kernel serves batched pairs, one huge pair and the normalise step of
// multiplication.
//
// Tile layout: a workgroup of WAVES waves owns WAVES*ROWS*128 consecutive limbs;
// wave w owns ROWS consecutive 128-limb rows; in a row, lane l holds limbs
// 2l and 2l+1 (one 16-byte load per operand), so every load instruction of a wave
// reads one contiguous 1 KiB block.
#include "bn_internal.h"

#include <algorithm>

namespace {

// Native 2 x 64-bit vector for the streaming loads and stores (the non-temporal
// builtins take native vector types only).
typedef unsigned long long u64v2 __attribute__((ext_vector_type(2)));

constexpr u64 ST_A = 1;   // tile aggregate ready, tile propagates its carry-in (carry-out unknown)
constexpr u64 ST_I0 = 2;  // tile carry-out known: 0
constexpr u64 ST_I1 = 3;  // tile carry-out known: 1

__device__ __forceinline__ u64 ld_relaxed(const u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(u64 *p, u64 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Raw limb result and its generate / propagate flags (phases 1-2).
//   add: s = x + y mod 2^64, generate = [s < x] (Lemma 1), propagate = [s == 2^64 - 1]
//   sub: s = x - y mod 2^64, generate = [x < y],            propagate = [s == 0]
// In both cases generate and propagate are never both set.
template <bool SUB>
__device__ __forceinline__ void limb_gp(u64 x, u64 y, u64 &s, bool &g, bool &p) {
    if (SUB) {
        s = x - y;
        g = x < y;
        p = (s == 0);
    } else {
        s = x + y;
        g = s < x;
        p = (s == ~0ull);
    }
}

// Carry resolution of one 64-lane row from its generate mask G, propagate mask P
// and the carry into lane 0.  Returns the carry-into-lane mask; cout receives the
// carry out of lane 63.
__device__ __forceinline__ u64 row_resolve(u64 G, u64 P, u64 cin, u64 &cout) {
    const u64 X = (G << 1) | cin;
    const u64 T = X + P;
    const u64 C = T ^ P;
    cout = (G >> 63) | ((P >> 63) & (C >> 63));
    return C;
}

__device__ __forceinline__ void divmod_u64(u64 x, u64 n, int nshift, u64 &q, u64 &r) {
    if (nshift >= 0) {
        q = x >> nshift;
        r = x & (n - 1);
    } else if (((x | n) >> 32) == 0) {
        const u32 qq = (u32)x / (u32)n;
        q = qq;
        r = (u32)x - qq * (u32)n;
    } else {
        q = x / n;
        r = x - q * n;
    }
}

struct ScanGeom {
    u64 N;         // total limbs
    u64 n;         // segment (pair) length
    int nshift;    // log2(n) if n is a power of two, else -1
    u64 TL;        // limbs per tile
    u64 epoch;     // chained launches: this launch's epoch, or 0 to read it from the control block
    const u64 *cin;  // EXT_CIN: per-segment carry (borrow) into the segment's first limb (bit 0)
    u64 nseg;        // segments (pairs)
    u64 bval;        // EXT_BCONST: the value of every limb of b
    u32 no_self_help;  // 1 when r overlaps a or b: a waiting tile never reads another tile's operands
    u64 nbz;           // EXT_BZX: limbs of b per pair (b's pair stride); b reads as 0 past them
    u32 defer;         // chained launches: no tile waits for another's look-back (see k_flat_scan, phase 3)
    uint8_t *codes;    // deferred launches: one byte per tile (1: its carry-in repair is left to the fill pass)
    ScanComb comb;     // EXT_COMB: the terms of a Karatsuba combine
    ScanSwap swap;     // EXT_SWAP: per-pair operand order and its record
    u64 N1;            // two-part launches: limbs of the first part (a whole number of tiles), else 0
    u64 *r2;           // ... and the second part's arrays (b2 null when b is unused)
    const u64 *a2, *b2;
};

// Kernel variants beyond the plain a +- b: a per-segment carry-in, b given as one limb
// value repeated (b = 0: the carry-in alone propagates through a; b = 0x80...80: the
// balanced-digit conversion of a product's operands), and b shorter than a in every
// pair (its own pair stride nbz, zero-extended to the segment length: the unequal
// lengths of the proof of Theorem 2).
constexpr int EXT_CIN = 1, EXT_BCONST = 2, EXT_BZX = 4;
// EXT_COMB: the sum is a Karatsuba level's result formed from its three child products
// (a and b unused): product q (segment of n = out limbs) is
//     P0 + P1 X^(2k) + (P0 + P1 -+ PD) X^k,
// with -PD when the two halves' differences had the same sign.  Its limb i term
//     v_i = [i < 2k] P0_i + [i >= 2k] P1_(i-2k) + [k <= i < 3k] (P0_t + P1_t -+ PD_t),  t = i - k,
// lies in (-2^64, 2^66) and is taken as v_i + 2^64 - [i > 0] in [0, 2^67) (the offsets
// add up to X^out, zero modulo X^out, and the product fits out limbs): the scan adds
// its low word and the high word of the limb below, whose sum has single-bit carries.
constexpr int EXT_COMB = 8;
// EXT_SWAP (subtraction): pair q computes b - a when its sign says so (ScanSwap).
constexpr int EXT_SWAP = 16;

// Sign of pair q of an EXT_SWAP launch: bit 0 of the largest of its keys.
__device__ __forceinline__ bool swap_sign(const ScanSwap &S, u64 q) {
    u64 m = 0;
    for (u64 p = 0; p < S.npieces; ++p) m = m > S.keys[q * S.npieces + p] ? m : S.keys[q * S.npieces + p];
    return (m & 1u) != 0;
}

// v_i + 2^64 - [i > 0] of product q (EXT_COMB).
__device__ __forceinline__ unsigned __int128 comb_term(const ScanComb &C, u64 q, u64 i) {
    typedef unsigned __int128 u128;
    const u64 k = C.k, base = 2 * k * q;
    u128 v = (u128)(i < 2 * k ? C.P0[base + i] : C.P1[base + i - 2 * k]) + ((u128)1 << 64) - (i > 0 ? 1u : 0u);
    if (i >= k && i < 3 * k) {
        const u64 t = i - k;
        v += (u128)C.P0[base + t] + C.P1[base + t];
        const u64 d = C.PD[base + t];
        v = C.negA[q] == C.negB[q] ? v - d : v + d;
    }
    return v;
}

// Limb of b that meets limb idx = q n + pos of a.
template <int EXT>
__device__ __forceinline__ u64 b_limb(const u64 *__restrict__ b, const ScanGeom &G, u64 idx, u64 q, u64 pos) {
    if constexpr ((EXT & EXT_BCONST) != 0) return G.bval;
    if constexpr ((EXT & EXT_BZX) != 0) return pos < G.nbz ? b[q * G.nbz + pos] : 0ull;
    return b[idx];
}

template <int EXT>
__device__ __forceinline__ bool seg_cin(const ScanGeom &G, u64 q) {
    if constexpr ((EXT & EXT_CIN) != 0) return q < G.nseg && (G.cin[q] & 1ull) != 0;
    return false;
}

// (generate, propagate) aggregate of tile u computed from the operands by one
// wave, 128 limbs per step.  Used when the tile has not published its status yet
// (self-help), so the waiting tile never depends on another workgroup making progress.
template <bool SUB, int EXT>
__device__ void tile_aggregate_from_data(const u64 *__restrict__ a, const u64 *__restrict__ b, const ScanGeom &G,
                                         u64 u, u32 &g_out, u32 &p_out) {
    const int lane = threadIdx.x & 63;
    const u64 lo = u * G.TL;
    const u64 hi = (lo + G.TL < G.N) ? lo + G.TL : G.N;
    u32 g = 0, p = 1;
    for (u64 base = lo; base < hi; base += 128) {
        const u64 i0 = base + 2 * (u64)lane;
        u64 q, pos;
        divmod_u64(i0, G.n, G.nshift, q, pos);
        bool g0 = false, p0 = false, g1 = false, p1 = false;
        u64 s;
        const bool wrap = pos + 1 == G.n;  // limb i0 + 1 starts the next segment
        if constexpr ((EXT & EXT_COMB) != 0) {
            // the terms of both limbs and of the limb below (see comb_term)
            unsigned __int128 v0 = 0, v1 = 0;
            u64 yb = 0;
            if (i0 < hi) {
                v0 = comb_term(G.comb, q, pos);
                if (pos > 0) yb = (u64)(comb_term(G.comb, q, pos - 1) >> 64);
                limb_gp<SUB>((u64)v0, yb, s, g0, p0);
            }
            if (i0 + 1 < hi) {
                v1 = comb_term(G.comb, wrap ? q + 1 : q, wrap ? 0 : pos + 1);
                limb_gp<SUB>((u64)v1, wrap ? 0ull : (u64)(v0 >> 64), s, g1, p1);
            }
        } else if constexpr ((EXT & EXT_SWAP) != 0) {
            if (i0 < hi) {
                const bool sw = swap_sign(G.swap, q);
                limb_gp<SUB>(sw ? b[i0] : a[i0], sw ? a[i0] : b[i0], s, g0, p0);
            }
            if (i0 + 1 < hi) {
                const bool sw = swap_sign(G.swap, wrap ? q + 1 : q);
                limb_gp<SUB>(sw ? b[i0 + 1] : a[i0 + 1], sw ? a[i0 + 1] : b[i0 + 1], s, g1, p1);
            }
        } else {
            if (i0 < hi) limb_gp<SUB>(a[i0], b_limb<EXT>(b, G, i0, q, pos), s, g0, p0);
            if (i0 + 1 < hi)
                limb_gp<SUB>(a[i0 + 1], b_limb<EXT>(b, G, i0 + 1, wrap ? q + 1 : q, wrap ? 0 : pos + 1), s, g1, p1);
        }
        // a segment's first limb takes the segment's carry-in, not its neighbour's carry
        g0 = g0 || (pos == 0 && p0 && seg_cin<EXT>(G, q));
        g1 = g1 || (pos + 1 == G.n && i0 + 1 < hi && p1 && seg_cin<EXT>(G, q + 1));
        p0 = p0 && pos != 0;
        p1 = p1 && pos + 1 != G.n;
        const u64 Gm = __ballot(g1 || (p1 && g0));
        const u64 Pm = __ballot(p0 && p1);
        u64 co;
        row_resolve(Gm, Pm, g, co);
        g = (u32)co;
        p &= (Pm == ~0ull) ? 1u : 0u;
    }
    g_out = g;
    p_out = p;
}

// Wave-wide decoupled look-back for the carry into tile t.  Lane l reads the
// status of the l-th nearest predecessor in the current window; the nearest one
// that is not an all-propagate aggregate decides: a known carry-out ends the walk;
// an unpublished tile is waited for up to `spin_limit` polls, after which the wave
// computes that tile's aggregate from the operands itself and walks on.  Tiles
// below index 0 count as "carry-out 0".  `dist` returns how many tiles back the
// deciding predecessor was.
//
// Deferred launches: the carry into tile t from its 64-tile window, or 2 (left to the
// fill pass) when every tile in the window propagates.  The nearest predecessor that
// does not propagate publishes its carry-out right after its own loads and never waits
// for anyone, so a wait for it is short; after `spin_limit` polls (it may not have
// been dispatched yet) the carry-in is left to the fill pass as well.
__device__ u32 lookback_defer(const u64 *status, u64 t, u64 epoch, u32 spin_limit) {
    const int lane = threadIdx.x & 63;
    const i64 idx = (i64)t - 1 - lane;
    for (u32 spins = 0;; ++spins) {
        u64 st = (epoch << 2) | ST_I0;  // below tile 0: carry-out 0
        if (idx >= 0) st = ld_relaxed(status + idx);
        const u32 state = ((st >> 2) == epoch) ? (u32)(st & 3) : 0u;
        const u64 notA = __ballot(state != ST_A);
        if (notA == 0) return 2u;
        const u32 sf = __shfl(state, __ffsll((unsigned long long)notA) - 1);
        if (sf >= ST_I0) return sf & 1u;
        if (spins >= spin_limit) return 2u;
        __builtin_amdgcn_s_sleep(1);
    }
}

// In place (r overlapping a or b) there is no self-help: the unpublished tile may
// publish and overwrite its operands with sums between our status read and our
// operand reads, so the wave only waits.  Every wait still ends: a tile publishes
// before it waits for anything, and the lowest unfinished tile is resident because
// workgroups of one XCD are dispatched in index order (the argument every decoupled
// look-back without self-help rests on).
template <bool SUB, int EXT>
__device__ u32 lookback(const u64 *status, u64 t, u64 epoch, u32 spin_limit, u64 *latch,
                        const u64 *__restrict__ a, const u64 *__restrict__ b, const ScanGeom &G, u64 &dist) {
    const int lane = threadIdx.x & 63;
    // fast probe: the nearest predecessor usually knows its carry-out already
    {
        u64 st = 0;
        if (lane == 0) st = ld_relaxed(status + t - 1);
        st = __shfl(st, 0);
        const u32 state = ((st >> 2) == epoch) ? (u32)(st & 3) : 0u;
        dist = 1;
        if (state >= ST_I0) return state & 1u;
    }
    i64 base = (i64)t - 1;
    u32 spins = 0;
    while (true) {
        const i64 idx = base - lane;
        u64 st = (epoch << 2) | ST_I0;
        if (idx >= 0) st = ld_relaxed(status + idx);
        const u32 state = ((st >> 2) == epoch) ? (u32)(st & 3) : 0u;
        const u64 notA = __ballot(state != ST_A);
        if (notA == 0) {
            base -= 64;
            continue;
        }
        const int first = __ffsll((unsigned long long)notA) - 1;
        const u32 sf = __shfl(state, first);
        dist = (u64)((i64)t - (base - first));  // base - first >= -1: "tile -1" is a carry-out 0
        if (sf != 0) return sf & 1u;
        if (G.no_self_help || ++spins <= spin_limit) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        // self-help: the tiles between `first` and t are all-propagate, so the carry
        // into t is the carry out of tile u
        const u64 u = (u64)(base - first);
        u32 gu, pu;
        tile_aggregate_from_data<SUB, EXT>(a, b, G, u, gu, pu);
        if (lane == 0) __hip_atomic_fetch_or(latch, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!pu) return gu;
        base = (i64)u - 1;
        spins = 0;
    }
}

template <bool SUB, int WAVES, int ROWS, bool VEC, bool CHAIN, int EXT = 0>
__global__ __launch_bounds__(WAVES * 64) void k_flat_scan(u64 *__restrict__ r, const u64 *__restrict__ a,
                                                          const u64 *__restrict__ b, ScanGeom G, u64 step_mod,
                                                          u64 step_div, u64 *__restrict__ carry,
                                                          ScanCtl *__restrict__ ctl, u64 *__restrict__ status,
                                                          u32 spin_limit, u32 dbg) {
    constexpr bool chain = CHAIN;
    __shared__ u32 sh_g[WAVES], sh_p[WAVES], sh_cin[WAVES], sh_cin_true[WAVES], sh_pt;

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    // Tile t is workgroup t.  chain == 0: every tile starts a segment (the tile
    // length is a multiple of the segment length), so no tile needs its
    // predecessor's carry and the look-back machinery is skipped.  chain == 1:
    // tiles publish status words tagged with the launch epoch and look back.  The
    // epoch comes with the launch, or (launches recorded into a graph, which replay
    // the same arguments) from the control block, which a one-thread kernel after
    // the launch moves on (a plain load: it only changes between launches).
    const u64 t = blockIdx.x;
    const u64 epoch = chain ? (G.epoch ? G.epoch : ctl->epoch) : 0;
    constexpr u64 TL = (u64)WAVES * ROWS * 128;
    const u64 N = G.N, n = G.n;
    const u64 idx0 = t * TL + (u64)w * ROWS * 128 + 2 * (u64)lane;
    // Two-part launches: the tiles past the first part take the second part's arrays
    // (limb idx of the launch is limb idx - N1 there).  The second part starts a
    // segment, so no look-back or self-help ever crosses from one part into the other.
    if (G.N1 != 0 && t * TL >= G.N1) {
        r = G.r2 - G.N1;
        a = G.a2 - G.N1;
        if (G.b2) b = G.b2 - G.N1;
    }

    // ---- phase 1: loads (all rows issued before any use) ----
    // A full tile (the common case) loads without per-row guards so that every
    // load of the wave is in flight at once; only the last tile checks bounds.
    // Operands are read once and results written once: non-temporal loads and
    // stores keep them from displacing other lines in the caches (measured +10%).
    const bool full = VEC && (t + 1) * TL <= N;
    u64 x0[ROWS], x1[ROWS], y0[ROWS], y1[ROWS];
    constexpr bool BC = (EXT & EXT_BCONST) != 0;
    if constexpr ((EXT & EXT_COMB) != 0) {
        // x = low word of the limb's term, y = high word of the term one limb down (0
        // at a segment start): from the lane below, lane 63 of the row below, or, for
        // the wave's first limb, computed here.  Every row's loads go out first
        // (predicated, no branch between a load and the next), then the arithmetic.
        const ScanComb &C = G.comb;
        const u64 k = C.k;
        u64 q, pos;
        divmod_u64(idx0, n, G.nshift, q, pos);
        u32 hprev = 0;  // high word of the term below the wave's first limb
        if (lane == 0 && pos > 0 && idx0 < N) hprev = (u32)(comb_term(C, q, pos - 1) >> 64);
        u64 lm[ROWS][2], l0[ROWS][2], l1[ROWS][2], ld[ROWS][2];  // main, P0_t, P1_t, PD_t
        bool mid[ROWS][2], same[ROWS][2], inb[ROWS][2], st[ROWS][2];
        // Even k, even segments and 16-byte aligned arrays: a lane's two limbs (an even
        // position and the next) share their segment, their array and their band, so each
        // array is one 16-byte load.
        const bool pairs = (k & 1) == 0 && (n & 1) == 0 &&
                           (((uintptr_t)C.P0 | (uintptr_t)C.P1 | (uintptr_t)C.PD) & 15u) == 0;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const u64 idx = idx0 + (u64)j * 128;
            if (pairs) {
                const u64 base = 2 * k * q;
                const bool in = idx < N;  // N is even: both limbs or neither
                const bool md = in && pos >= k && pos < 3 * k;
                const u64 t = md ? pos - k : 0;
                typedef unsigned long long v2 __attribute__((ext_vector_type(2)));
                const u64 *pm = pos < 2 * k ? C.P0 + base + pos : C.P1 + base + pos - 2 * k;
                const v2 vm = in ? *reinterpret_cast<const v2 *>(pm) : v2{0, 0};
                const v2 v0 = md ? *reinterpret_cast<const v2 *>(C.P0 + base + t) : v2{0, 0};
                const v2 v1 = md ? *reinterpret_cast<const v2 *>(C.P1 + base + t) : v2{0, 0};
                const v2 vd = md ? *reinterpret_cast<const v2 *>(C.PD + base + t) : v2{0, 0};
                const bool sm = in && C.negA[q] == C.negB[q];
                lm[j][0] = vm.x;
                lm[j][1] = vm.y;
                l0[j][0] = v0.x;
                l0[j][1] = v0.y;
                l1[j][0] = v1.x;
                l1[j][1] = v1.y;
                ld[j][0] = vd.x;
                ld[j][1] = vd.y;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    same[j][e] = sm;
                    mid[j][e] = md;
                    inb[j][e] = in;
                    st[j][e] = e == 0 && pos == 0;
                }
                pos += step_mod;
                q += step_div;
                if (pos >= n) {
                    pos -= n;
                    q += 1;
                }
                continue;
            }
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const bool wrap = e == 1 && pos + 1 == n;  // limb idx + 1 starts the next segment
                const u64 qq = wrap ? q + 1 : q, ii = e == 0 ? pos : (wrap ? 0 : pos + 1);
                const u64 base = 2 * k * qq;
                const bool in = idx + e < N;
                const bool md = in && ii >= k && ii < 3 * k;
                const u64 t = md ? ii - k : 0;
                const u64 *pm = ii < 2 * k ? C.P0 + base + ii : C.P1 + base + ii - 2 * k;
                lm[j][e] = in ? *pm : 0ull;
                l0[j][e] = md ? C.P0[base + t] : 0ull;
                l1[j][e] = md ? C.P1[base + t] : 0ull;
                ld[j][e] = md ? C.PD[base + t] : 0ull;
                same[j][e] = in && C.negA[qq] == C.negB[qq];
                mid[j][e] = md;
                inb[j][e] = in;
                st[j][e] = ii == 0;
            }
            pos += step_mod;
            q += step_div;
            if (pos >= n) {
                pos -= n;
                q += 1;
            }
        }
        u32 h1[ROWS];
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            unsigned __int128 v[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                unsigned __int128 w = (unsigned __int128)lm[j][e] + ((unsigned __int128)1 << 64) - (st[j][e] ? 0u : 1u);
                if (mid[j][e]) {
                    w += (unsigned __int128)l0[j][e] + l1[j][e];
                    w = same[j][e] ? w - ld[j][e] : w + ld[j][e];
                }
                v[e] = inb[j][e] ? w : 0;
            }
            x0[j] = (u64)v[0];
            x1[j] = (u64)v[1];
            y1[j] = st[j][1] ? 0ull : (u64)(v[0] >> 64);
            h1[j] = (u32)(v[1] >> 64);
        }
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const u32 below = (u32)__shfl_up((int)h1[j], 1);
            const u32 first = j == 0 ? hprev : (u32)__builtin_amdgcn_readlane((int)h1[j - 1], 63);
            y0[j] = st[j][0] ? 0ull : (u64)(lane == 0 ? first : below);
        }
    } else if constexpr ((EXT & EXT_BZX) != 0) {
        // b limbs by segment position (8-byte loads; consecutive lanes still read
        // consecutive limbs inside a pair)
        u64 q, pos;
        divmod_u64(idx0, n, G.nshift, q, pos);
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const u64 idx = idx0 + (u64)j * 128;
            if (full) {
                const u64v2 va = __builtin_nontemporal_load(reinterpret_cast<const u64v2 *>(a + idx));
                x0[j] = va.x;
                x1[j] = va.y;
            } else {
                x0[j] = idx < N ? a[idx] : 0;
                x1[j] = idx + 1 < N ? a[idx + 1] : 0;
            }
            const bool wrap = pos + 1 == n;
            y0[j] = idx < N ? b_limb<EXT>(b, G, idx, q, pos) : 0;
            y1[j] = idx + 1 < N ? b_limb<EXT>(b, G, idx + 1, wrap ? q + 1 : q, wrap ? 0 : pos + 1) : 0;
            pos += step_mod;
            q += step_div;
            if (pos >= n) {
                pos -= n;
                q += 1;
            }
        }
    } else if (full) {
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const u64v2 va = __builtin_nontemporal_load(reinterpret_cast<const u64v2 *>(a + idx0 + (u64)j * 128));
            x0[j] = va.x;
            x1[j] = va.y;
            if (BC) {
                y0[j] = y1[j] = G.bval;
            } else {
                const u64v2 vb = __builtin_nontemporal_load(reinterpret_cast<const u64v2 *>(b + idx0 + (u64)j * 128));
                y0[j] = vb.x;
                y1[j] = vb.y;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const u64 idx = idx0 + (u64)j * 128;
            x0[j] = idx < N ? a[idx] : 0;
            y0[j] = idx < N ? (BC ? G.bval : b[idx]) : 0;
            x1[j] = idx + 1 < N ? a[idx + 1] : 0;
            y1[j] = idx + 1 < N ? (BC ? G.bval : b[idx + 1]) : 0;
        }
    }

    u64 pos0, q0;
    divmod_u64(idx0, n, G.nshift, q0, pos0);

    // ---- phase 2: classify, ballot, wave aggregate with carry-in 0 ----
    u64 Gm[ROWS], Pm[ROWS];
    u32 fl[ROWS];  // bit0 g0, bit1 p0, bit2 g1, bit3 p1 (raw flags of the lane's two limbs)
    u32 wg = 0, wp = 1;
    {
        u64 pos = pos0, q = q0;
        u64 sq = ~0ull;  // EXT_SWAP: the pair whose sign sneg holds
        bool sneg = false;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const u64 idx = idx0 + (u64)j * 128;
            const bool v0 = idx < N, v1 = idx + 1 < N;
            if constexpr ((EXT & EXT_SWAP) != 0) {
                // the pair's operands in the order its sign gives; the lane holding a
                // pair's first limb records the sign
                const bool wrap = pos + 1 == n;
                if (v0 && q != sq) {
                    sq = q;
                    sneg = swap_sign(G.swap, q);
                }
                const bool n0 = v0 && sneg;
                const bool n1 = v1 && (wrap ? swap_sign(G.swap, q + 1) : sneg);
                if (n0) {
                    const u64 t0 = x0[j];
                    x0[j] = y0[j];
                    y0[j] = t0;
                }
                if (n1) {
                    const u64 t1 = x1[j];
                    x1[j] = y1[j];
                    y1[j] = t1;
                }
                if (v0 && pos == 0) G.swap.neg[q] = n0;
                if (v1 && wrap) G.swap.neg[q + 1] = n1;
            }
            u64 s0, s1;
            bool g0, p0, g1, p1;
            limb_gp<SUB>(x0[j], y0[j], s0, g0, p0);
            limb_gp<SUB>(x1[j], y1[j], s1, g1, p1);
            g0 &= v0;
            p0 &= v0;
            g1 &= v1;
            p1 &= v1;
            x0[j] = s0;
            x1[j] = s1;
            fl[j] = (u32)g0 | ((u32)p0 << 1) | ((u32)g1 << 2) | ((u32)p1 << 3);
            const bool st0 = (pos == 0);
            const bool st1 = (pos + 1 == n);
            const bool pp0 = p0 && !st0;  // a segment start does not pass a carry in
            const bool pp1 = p1 && !st1;
            // ... it takes the segment's own carry-in instead (EXT_CIN)
            const bool ge0 = g0 || (st0 && p0 && seg_cin<EXT>(G, q));
            const bool ge1 = g1 || (st1 && p1 && seg_cin<EXT>(G, q + 1));
            const bool Gl = ge1 || (pp1 && ge0);
            const bool Pl = pp0 && pp1;
            Gm[j] = __ballot(Gl);
            Pm[j] = __ballot(Pl);
            u64 co;
            row_resolve(Gm[j], Pm[j], wg, co);
            wg = (u32)co;
            wp &= (Pm[j] == ~0ull) ? 1u : 0u;
            pos += step_mod;
            q += step_div;
            if (pos >= n) {
                pos -= n;
                q += 1;
            }
        }
    }
    if (lane == 0) {
        sh_g[w] = wg;
        sh_p[w] = wp;
    }
    __syncthreads();

    // ---- phase 3: carries into the waves assuming carry-in 0 into the tile; publish ----
    // A tile that does not propagate knows its carry-out now (I0/I1); one that
    // propagates publishes A and learns its carry-in by look-back in phase 5.
    // (never in place: without self-help nobody could get past the silent tile)
    const bool poison = (dbg & 1u) && t == 0 && !G.no_self_help;
    if (threadIdx.x == 0) {
        u32 c = 0, pt = 1;
#pragma unroll
        for (int i = 0; i < WAVES; ++i) {
            sh_cin[i] = c;
            c = sh_g[i] | (sh_p[i] & c);
            pt &= sh_p[i];
        }
        sh_pt = pt;
        if (chain && !poison) st_relaxed(status + t, (epoch << 2) | (pt ? ST_A : (c ? ST_I1 : ST_I0)));
    }
    __syncthreads();

    // Deferred launches: no tile waits for another tile's look-back.  A tile whose every
    // limb propagates holds no information but its carry-in -- its result is the
    // constant the raw limbs turn into (add: all ones with carry-in 0, all zeros with 1;
    // sub: the reverse) -- so it stores nothing and frees its slot at once; its A status
    // stays.  (Reading its window once first and storing the constant when that decides
    // the carry-in was measured slower on every input.)  Every other tile stores its
    // sums for carry-in 0 and reads its window, waiting only for a predecessor that is
    // still loading: if every tile in the window propagates, it leaves the repair (the
    // propagate run at its start) to the fill pass.  After the launch, k_defer_scan
    // finds the carry-in of every tile left over among the final status words and
    // k_defer_fill writes the constants and the repairs.
    if (chain && G.defer && sh_pt) return;

    // The tile's real carry-in by look-back (wave 0), its inclusive status published,
    // and the carry into every wave of the tile.
    auto resolve_cin = [&]() {
        if (w == 0) {
            u32 cin = 0;
            const u64 first_pos = __shfl(pos0, 0);
            if (G.defer) {
                // an undecided carry-in is left to the fill pass (the tile keeps its
                // carry-in-0 sums, and its flag byte says so)
                u32 later = 0;
                if (t > 0 && first_pos != 0) {
                    cin = lookback_defer(status, t, epoch, spin_limit);
                    if (cin > 1u) {
                        cin = 0;
                        later = 1;
                    }
                }
                if (lane == 0) G.codes[t] = (uint8_t)later;
            } else if (t > 0 && first_pos != 0) {
                u64 dist;
                cin = lookback<SUB, EXT>(status, t, epoch, spin_limit, &ctl->err, a, b, G, dist);
                if ((dbg & 2u) && lane == 0)
                    __hip_atomic_fetch_add(ctl->hist + (63 - __clzll((long long)dist)), 1ull, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
            if (lane == 0) {
                if (sh_pt && !poison) st_relaxed(status + t, (epoch << 2) | (cin ? ST_I1 : ST_I0));
                u32 c = cin;
#pragma unroll
                for (int i = 0; i < WAVES; ++i) {
                    sh_cin_true[i] = c;
                    c = sh_g[i] | (sh_p[i] & c);
                }
            }
        }
    };
    // A tile that propagates its carry-in through every limb would have every limb
    // rewritten after an optimistic store, so it looks back first (its A status is
    // already published, so the tiles behind it can walk past it meanwhile).
    const bool early = chain && sh_pt;
    if (early) {
        resolve_cin();
        __syncthreads();
    }

    // ---- phase 4: apply the carries, store sums and per-segment carry-outs ----
    // Stored optimistically: in a chained launch the tile's real carry-in is not
    // known yet (unless looked up early above); phase 5 rewrites the few limbs it
    // changes (DoT's rare fix-up).
    const u32 c_assumed = early ? sh_cin_true[w] : sh_cin[w];
    {
        u64 c = c_assumed;
        u64 pos = pos0, q = q0;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const u64 idx = idx0 + (u64)j * 128;
            u64 co;
            const u64 C = row_resolve(Gm[j], Pm[j], c, co);
            c = co;
            const bool cb = (C >> lane) & 1ull;
            const bool g0 = fl[j] & 1u, p0 = fl[j] & 2u, g1 = fl[j] & 4u, p1 = fl[j] & 8u;
            const bool st0 = (pos == 0);
            const bool st1 = (pos + 1 == n);
            const bool en1 = (n == 1) || (pos + 2 == n);
            const bool ci0 = st0 ? seg_cin<EXT>(G, q) : cb;
            const bool co0 = g0 || (p0 && ci0);
            const bool ci1 = st1 ? seg_cin<EXT>(G, q + 1) : co0;
            const bool co1 = g1 || (p1 && ci1);
            const u64 r0 = SUB ? x0[j] - (u64)ci0 : x0[j] + (u64)ci0;
            const u64 r1 = SUB ? x1[j] - (u64)ci1 : x1[j] + (u64)ci1;
            if (full) {
                const u64v2 rv = {r0, r1};
                __builtin_nontemporal_store(rv, reinterpret_cast<u64v2 *>(r + idx));
            } else {
                if (idx < N) r[idx] = r0;
                if (idx + 1 < N) r[idx + 1] = r1;
            }
            if (carry) {
                if (idx < N && st1) carry[q] = co0;                        // limb idx ends a segment
                if (idx + 1 < N && en1) carry[q + (st1 ? 1 : 0)] = co1;
            }
            pos += step_mod;
            q += step_div;
            if (pos >= n) {
                pos -= n;
                q += 1;
            }
        }
    }
    if (!chain) return;

    // ---- phase 5: the tile's real carry-in (look-back), publish, repair ----
    if (!early) {
        resolve_cin();
        __syncthreads();  // also orders the optimistic stores before their rewrites
    }
    const u32 c_true = sh_cin_true[w];
    if (c_true != c_assumed) {
        // Replay the rows with both carries; lanes whose carry differs rewrite the
        // limbs (and segment carry-outs) that change; stop once the chains agree.
        u64 ca = c_assumed, ct = c_true;
        u64 pos = pos0, q = q0;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const u64 idx = idx0 + (u64)j * 128;
            u64 coa = ca, cot = ct;
            u64 Ca = 0, Ct = 0;
            if (ca != ct) {  // wave-uniform; once the chains agree every later row is unchanged
                Ca = row_resolve(Gm[j], Pm[j], ca, coa);
                Ct = row_resolve(Gm[j], Pm[j], ct, cot);
            }
            if (((Ca ^ Ct) >> lane) & 1ull) {
                const bool g0 = fl[j] & 1u, p0 = fl[j] & 2u, g1 = fl[j] & 4u, p1 = fl[j] & 8u;
                const bool st0 = (pos == 0);
                const bool st1 = (pos + 1 == n);
                const bool en1 = (n == 1) || (pos + 2 == n);
                const bool cs0 = seg_cin<EXT>(G, q), cs1 = st1 && seg_cin<EXT>(G, q + 1);
                const bool ci0a = st0 ? cs0 : ((Ca >> lane) & 1ull), ci0t = st0 ? cs0 : ((Ct >> lane) & 1ull);
                const bool co0a = g0 || (p0 && ci0a), co0t = g0 || (p0 && ci0t);
                const bool ci1a = st1 ? cs1 : co0a, ci1t = st1 ? cs1 : co0t;
                const bool co1a = g1 || (p1 && ci1a), co1t = g1 || (p1 && ci1t);
                if (ci0a != ci0t && idx < N) r[idx] = SUB ? x0[j] - (u64)ci0t : x0[j] + (u64)ci0t;
                if (ci1a != ci1t && idx + 1 < N) r[idx + 1] = SUB ? x1[j] - (u64)ci1t : x1[j] + (u64)ci1t;
                if (carry) {
                    if (idx < N && st1 && co0a != co0t) carry[q] = co0t;
                    if (idx + 1 < N && en1 && co1a != co1t) carry[q + (st1 ? 1 : 0)] = co1t;
                }
            }
            ca = coa;
            ct = cot;
            pos += step_mod;
            q += step_div;
            if (pos >= n) {
                pos -= n;
                q += 1;
            }
        }
    }
}

// After a deferred launch (every workgroup done): the carry into every tile that left
// its result to the fill pass -- tiles that propagate through all of their limbs, and
// tiles whose look-back window did not decide their carry-in.  A tile's carry-in is
// the carry out of the nearest tile below it that does not propagate (tile 0 starts a
// segment, so there is one).  Codes written: 0 = nothing to do, 1 + c = fill with
// carry-in c, 3 = repair with carry-in 1.  One workgroup; blocks of 16384 tiles,
// thread i taking 16 consecutive tiles; the "last known carry-out" runs across threads
// by ballots within each wave and across the 16 wave aggregates.
constexpr int DS_THREADS = 1024, DS_PER = 16;
__global__ __launch_bounds__(DS_THREADS) void k_defer_scan(const u64 *__restrict__ status, uint8_t *__restrict__ code,
                                                           u64 ntiles, u64 epoch_arg, const ScanCtl *__restrict__ ctl) {
    __shared__ u32 sh_def[DS_THREADS / 64], sh_val[DS_THREADS / 64];
    const u64 epoch = epoch_arg ? epoch_arg : ctl->epoch;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    u32 carry_blocks = 0;  // carry out of the blocks before this one (uniform)
    for (u64 base = 0; base < ntiles; base += (u64)DS_THREADS * DS_PER) {
        const u64 t0 = base + (u64)threadIdx.x * DS_PER;
        const bool whole = t0 + DS_PER <= ntiles;
        u32 state[DS_PER];
        u64 flags[DS_PER / 8];  // this thread's flag bytes, packed
        if (whole) {  // status + t0 is 128-byte aligned, code + t0 8-byte aligned
#pragma unroll
            for (int j = 0; j < DS_PER; j += 2) {
                const u64v2 v = *reinterpret_cast<const u64v2 *>(status + t0 + j);
                state[j] = (v.x >> 2) == epoch ? (u32)(v.x & 3) : 0u;
                state[j + 1] = (v.y >> 2) == epoch ? (u32)(v.y & 3) : 0u;
            }
#pragma unroll
            for (int k = 0; k < DS_PER / 8; ++k) flags[k] = *reinterpret_cast<const u64 *>(code + t0 + 8 * k);
        } else {
#pragma unroll
            for (int k = 0; k < DS_PER / 8; ++k) flags[k] = 0;
#pragma unroll
            for (int j = 0; j < DS_PER; ++j) {
                const u64 st = t0 + j < ntiles ? status[t0 + j] : 0ull;
                state[j] = (st >> 2) == epoch ? (u32)(st & 3) : 0u;
                if (t0 + j < ntiles) flags[j / 8] |= (u64)code[t0 + j] << (8 * (j % 8));
            }
        }
        bool def = false;
        u32 val = 0;
#pragma unroll
        for (int j = 0; j < DS_PER; ++j)
            if (state[j] >= ST_I0) {
                def = true;
                val = state[j] & 1u;
            }
        const u64 D = __ballot(def), V = __ballot(def && val);
        __syncthreads();  // the previous block's readers are done with sh_def / sh_val
        if (lane == 0) {
            sh_def[w] = D != 0;
            sh_val[w] = D ? (u32)((V >> (63 - __clzll((long long)D))) & 1ull) : 0u;
        }
        __syncthreads();
        u32 c = carry_blocks, block_out = carry_blocks;
#pragma unroll
        for (int k = 0; k < DS_THREADS / 64; ++k)
            if (sh_def[k]) {
                if (k < w) c = sh_val[k];
                block_out = sh_val[k];
            }
        const u64 below = D & ((1ull << lane) - 1ull);
        if (below) c = (u32)((V >> (63 - __clzll((long long)below))) & 1ull);
        u64 out[DS_PER / 8] = {};
#pragma unroll
        for (int j = 0; j < DS_PER; ++j) {
            u64 o = 0;
            if (state[j] == ST_A) {
                o = 1u + c;
            } else {
                if (((flags[j / 8] >> (8 * (j % 8))) & 0xff) != 0 && c) o = 3;
                if (state[j] >= ST_I0) c = state[j] & 1u;
            }
            out[j / 8] |= o << (8 * (j % 8));
        }
        if (whole) {
#pragma unroll
            for (int k = 0; k < DS_PER / 8; ++k) *reinterpret_cast<u64 *>(code + t0 + 8 * k) = out[k];
        } else {
#pragma unroll
            for (int j = 0; j < DS_PER; ++j)
                if (t0 + j < ntiles) code[t0 + j] = (uint8_t)(out[j / 8] >> (8 * (j % 8)));
        }
        carry_blocks = block_out;
    }
}

// The fill pass of a deferred launch, a grid-stride loop over the tiles' codes.
//   1 + c (c = 0, 1): the tile propagates through every limb; its result is the constant
//     the raw limbs turn into with carry-in c (add: all ones with 0, zeros with 1; sub:
//     zeros with 0, all ones with 1).  No segment starts inside such a tile, but its top
//     limb may end one (the next starts in the next tile, or it is the last limb): that
//     segment's carry-out is c, passed through every limb.
//   3: the tile holds its sums for carry-in 0 and its carry-in is 1: the carry runs up
//     from its first limb through the limbs still holding the propagate value (add: all
//     ones, sub: 0), which flip, to the first other limb, which moves by one -- or to a
//     segment start, in which case the segment below it gets carry-out 1.
// One tile's work (code c) on the whole workgroup.
template <bool SUB>
__device__ __forceinline__ void defer_fill_tile(u64 *__restrict__ r, u32 c, u64 lo, u64 hi, u64 n,
                                                u64 *__restrict__ carry, u32 &sh_stop) {
    constexpr u64 PV = SUB ? 0ull : ~0ull;  // a propagating limb's value for carry-in 0
    if (c <= 2) {
        const u64 v = ((c - 1u) ^ (SUB ? 1u : 0u)) ? 0ull : ~0ull;
        if (carry && threadIdx.x == 0 && hi % n == 0) carry[hi / n - 1] = c - 1u;
        if ((((uintptr_t)(r + lo)) & 15u) == 0 && ((hi - lo) & 1u) == 0) {
            const u64v2 vv = {v, v};
            for (u64 i = lo + 2 * (u64)threadIdx.x; i < hi; i += 512)
                __builtin_nontemporal_store(vv, reinterpret_cast<u64v2 *>(r + i));
        } else {
            for (u64 i = lo + threadIdx.x; i < hi; i += 256) r[i] = v;
        }
        return;
    }
    // repair with carry-in 1: where the carry stops (offset from lo), 256 limbs a pass
    if (threadIdx.x == 0) sh_stop = (u32)(hi - lo);
    __syncthreads();
    for (u64 base = lo; base < hi; base += 256) {
        const u64 i = base + threadIdx.x;
        if (i < hi && ((i > lo && i % n == 0) || r[i] != PV)) atomicMin(&sh_stop, (u32)(i - lo));
        __syncthreads();
        // later passes only lower sh_stop to values past this pass, so every thread
        // takes the same decision here
        if (sh_stop < (u32)(base + 256 - lo)) break;
    }
    const u64 stop = lo + sh_stop;
    for (u64 i = lo + threadIdx.x; i < stop; i += 256) r[i] = ~PV;
    if (threadIdx.x == 0) {
        if (stop < hi && stop % n != 0) r[stop] = SUB ? r[stop] - 1u : r[stop] + 1u;
        else if (carry && stop % n == 0) carry[stop / n - 1] = 1;
    }
    __syncthreads();  // sh_stop is reused by the next tile
}

// Workgroup b takes tiles b, b + G, b + 2G, ... (G = gridDim.x); the codes of 64 of them
// are read at once, one per lane (every wave reads the same ones, so the workgroup
// branches alike), and only the tiles with work are visited.
template <bool SUB>
__global__ __launch_bounds__(256) void k_defer_fill(u64 *__restrict__ r, const uint8_t *__restrict__ code, u64 ntiles,
                                                    u64 TL, u64 N, u64 n, u64 *__restrict__ carry) {
    __shared__ u32 sh_stop;
    const int lane = threadIdx.x & 63;
    for (u64 t0 = blockIdx.x; t0 < ntiles; t0 += 64 * (u64)gridDim.x) {
        const u64 tk = t0 + (u64)lane * gridDim.x;
        const u32 ck = tk < ntiles ? code[tk] : 0u;
        for (u64 m = __ballot(ck != 0); m; m &= m - 1) {
            const int k = __ffsll((unsigned long long)m) - 1;
            const u32 c = (u32)__shfl((int)ck, k);
            const u64 lo = (t0 + (u64)k * gridDim.x) * TL;
            defer_fill_tile<SUB>(r, c, lo, lo + TL < N ? lo + TL : N, n, carry, sh_stop);
        }
    }
}

// After a chained launch: move to a fresh epoch so that the next launch never
// mistakes this launch's status words for its own.  Stream order puts it after
// every workgroup of the scan.
__global__ void k_bump_epoch(ScanCtl *ctl) { ctl->epoch += 1; }

__global__ void k_fill_u64(u64 *p, u64 count, u64 value) {
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < count; i += (u64)gridDim.x * blockDim.x)
        p[i] = value;
}

typedef void (*scan_fn)(u64 *, const u64 *, const u64 *, ScanGeom, u64, u64, u64 *, ScanCtl *, u64 *, u32, u32);

template <bool SUB, bool CHAIN>
scan_fn pick(int waves, int rows) {
#define BN_SHAPE(W, R) \
    if (waves == W && rows == R) return k_flat_scan<SUB, W, R, true, CHAIN>;
#define BN_ROWS(W) BN_SHAPE(W, 1) BN_SHAPE(W, 2) BN_SHAPE(W, 4) BN_SHAPE(W, 8)
    BN_ROWS(1)
    BN_ROWS(2)
    BN_ROWS(4)
    BN_ROWS(8)
    BN_SHAPE(1, 16)
    BN_SHAPE(2, 16)
    BN_SHAPE(4, 16)  // 8 x 16 would not fit the register file
#undef BN_ROWS
#undef BN_SHAPE
    return nullptr;
}

// Operands that are only 8-byte aligned take 8-byte loads and fixed shapes.
constexpr int UNALIGNED_BATCH_WAVES = 1, UNALIGNED_BATCH_ROWS = 1;
constexpr int UNALIGNED_CHAIN_WAVES = 4, UNALIGNED_CHAIN_ROWS = 4;

// [x, x + xn) and [y, y + yn) (limbs) share a limb
bool ranges_overlap(const u64 *x, u64 xn, const u64 *y, u64 yn) {
    const uintptr_t x0 = (uintptr_t)x, y0 = (uintptr_t)y;
    return x && y && xn && yn && x0 < y0 + 8 * yn && y0 < x0 + 8 * xn;
}

}  // namespace

bool flat_scan_shape_ok(int waves, int rows) { return pick<false, false>(waves, rows) != nullptr; }

// Shape for a launch over N limbs in segments of n: the independent-tile shape when
// its tile length is a multiple of n, else the chained (look-back) shape, with its
// rows halved (aligned operands) until the launch has at least 8 tiles per CU -- a
// 2^20-limb chained launch in 4096-limb tiles would leave most of the device idle.
static void flat_scan_shape(const bn_ctx *ctx, u64 n, u64 N, bool vec, int &waves, int &rows, bool &chain) {
    const int bw = vec ? ctx->tune.batch_waves : UNALIGNED_BATCH_WAVES;
    const int br = vec ? ctx->tune.batch_rows : UNALIGNED_BATCH_ROWS;
    const u64 tl = (u64)bw * br * 128;
    chain = !(n && tl % n == 0);
    if (!chain) {
        waves = bw;
        rows = br;
    } else {
        waves = vec ? ctx->tune.chain_waves : UNALIGNED_CHAIN_WAVES;
        rows = vec ? ctx->tune.chain_rows : UNALIGNED_CHAIN_ROWS;
        const u64 want = 8 * (u64)std::max(1, ctx->num_cu);
        while (vec && rows > 1 && (N + (u64)waves * rows * 128 - 1) / ((u64)waves * rows * 128) < want) rows /= 2;
    }
}

// Look-back state of a chained launch over `tiles` tiles: one status word per tile,
// then one fill code byte per tile (deferred launches).
size_t scan_state_bytes(u64 tiles) { return (size_t)(tiles + (tiles + 7) / 8) * sizeof(u64); }

// Status words needed by a launch over N limbs in segments of n (the larger count
// of the aligned and the unaligned shape, so a reservation covers both).
size_t flat_scan_status_bytes(const bn_ctx *ctx, u64 n, u64 N) {
    u64 tiles = 0;
    for (int v = 0; v < 2; ++v) {
        int waves = 1, rows = 1;
        bool chain = false;
        flat_scan_shape(ctx, n, N, v == 1, waves, rows, chain);
        if (!chain) continue;  // independent tiles publish nothing
        const u64 TL = (u64)waves * rows * 128;
        tiles = std::max<u64>(tiles, (N + TL - 1) / TL);
    }
    return scan_state_bytes(tiles);
}

size_t flat_scan_ext_status_bytes(u64 n, u64 N) {
    if (n == 0 || 128 % n == 0) return 0;  // independent tiles: no status words
    const u64 TL = 4 * 128;  // the smallest chained tile
    return scan_state_bytes((N + TL - 1) / TL);
}

bn_status launch_fill_u64(u64 *p, u64 count, u64 value, hipStream_t s) {
    if (count == 0) return BN_OK;
    u64 blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((u32)blocks), dim3(256), 0, s, p, count, value);
    return bn_launch_status();
}

// The extended variants (carry-in, constant b) come in fixed shapes: 1 x 1 independent
// tiles, 4 x 8 (4 x 4 unaligned) chained tiles; aligned chained launches of the
// constant-b variant alone (the operand conversion of products) also take 4 x 4, 4 x 2
// and 4 x 1 tiles, so that a small launch still spreads over the device.
template <bool SUB, int EXT>
static scan_fn pick_ext(bool vec, bool chain, int rows = 8) {
    if constexpr (EXT == EXT_COMB) {  // at most 4 rows: every row's term loads are held at once
        if (vec && chain) {
            if (rows == 1) return k_flat_scan<SUB, 4, 1, true, true, EXT>;
            if (rows == 2) return k_flat_scan<SUB, 4, 2, true, true, EXT>;
            return k_flat_scan<SUB, 4, 4, true, true, EXT>;
        }
        if (vec) return k_flat_scan<SUB, 1, 1, true, false, EXT>;
        return chain ? k_flat_scan<SUB, UNALIGNED_CHAIN_WAVES, UNALIGNED_CHAIN_ROWS, false, true, EXT>
                     : k_flat_scan<SUB, UNALIGNED_BATCH_WAVES, UNALIGNED_BATCH_ROWS, false, false, EXT>;
    }
    if (vec && chain && (EXT == EXT_BCONST || EXT == EXT_SWAP)) {
        if (rows == 1) return k_flat_scan<SUB, 4, 1, true, true, EXT>;
        if (rows == 2) return k_flat_scan<SUB, 4, 2, true, true, EXT>;
        if (rows == 4) return k_flat_scan<SUB, 4, 4, true, true, EXT>;
    }
    if (vec) return chain ? k_flat_scan<SUB, 4, 8, true, true, EXT> : k_flat_scan<SUB, 1, 1, true, false, EXT>;
    return chain ? k_flat_scan<SUB, UNALIGNED_CHAIN_WAVES, UNALIGNED_CHAIN_ROWS, false, true, EXT>
                 : k_flat_scan<SUB, UNALIGNED_BATCH_WAVES, UNALIGNED_BATCH_ROWS, false, false, EXT>;
}

bn_status launch_flat_scan_mem(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs,
                             const u64 *cin, bool bconst, u64 bval, u64 *carry, hipStream_t s, const ScanMem *fixed,
                             i64 nbz, const ScanComb *comb, const ScanPart2 *part2, const ScanSwap *swap) {
    if (part2 && part2->npairs == 0) part2 = nullptr;
    // the second part on its own: its pairs' carries, carry-ins and signs follow the first part's
    auto second_alone = [&](u64 np1) {
        ScanSwap sw2;
        if (swap) {
            sw2 = *swap;
            sw2.keys += np1 * swap->npieces;
            sw2.neg += np1;
        }
        return launch_flat_scan_mem(ctx, sub, part2->r, part2->a, part2->b, n, part2->npairs, cin ? cin + np1 : nullptr,
                                    bconst, bval, carry ? carry + np1 : nullptr, s, fixed, nbz, comb, nullptr,
                                    swap ? &sw2 : nullptr);
    };
    if (part2 && (npairs == 0 || n == 0 || cin || nbz >= 0 || comb)) {  // one launch per part
        bn_status st =
            launch_flat_scan_mem(ctx, sub, r, a, b, n, npairs, cin, bconst, bval, carry, s, fixed, nbz, comb, nullptr, swap);
        if (st != BN_OK) return st;
        return second_alone(npairs);
    }
    const u64 N1 = part2 ? n * npairs : 0;
    const u64 N = n * (npairs + (part2 ? part2->npairs : 0));
    npairs += part2 ? part2->npairs : 0;
    if (N == 0) return carry ? launch_fill_u64(carry, npairs, 0, s) : BN_OK;
    const bool bzx = nbz >= 0;
    const bool vec =
        (((uintptr_t)r | (uintptr_t)a | (uintptr_t)(bconst || bzx ? nullptr : b) |
          (part2 ? ((uintptr_t)part2->r | (uintptr_t)part2->a | (uintptr_t)(bconst ? nullptr : part2->b)) : 0)) &
         15u) == 0;
    const int ext = (cin ? EXT_CIN : 0) | (bconst ? EXT_BCONST : 0) | (bzx ? EXT_BZX : 0) | (comb ? EXT_COMB : 0) |
                    (swap ? EXT_SWAP : 0);
    int waves, rows;
    bool chain;
    if (ext == 0) {
        flat_scan_shape(ctx, n, N, vec, waves, rows, chain);
    } else {
        chain = (128 % n) != 0;
        waves = chain ? (vec ? 4 : UNALIGNED_CHAIN_WAVES) : 1;
        rows = chain ? (vec ? (ext == EXT_COMB ? 4 : 8) : UNALIGNED_CHAIN_ROWS) : 1;
        if ((ext == EXT_BCONST || ext == EXT_COMB || ext == EXT_SWAP) && chain && vec) {  // >= 8 tiles per CU where rows allow
            const u64 want = 8 * (u64)std::max(1, ctx->num_cu);
            while (rows > 1 && (N + (u64)waves * rows * 128 - 1) / ((u64)waves * rows * 128) < want) rows /= 2;
        }
    }
    const u64 TL = (u64)waves * rows * 128;
    if (part2) {
        // one launch only if the first part ends on a tile boundary and every array is
        // apart from every other (a tile of one part never touches the other's arrays)
        const u64 N2 = N - N1;
        const bool apart = !ranges_overlap(r, N1, part2->r, N2) && !ranges_overlap(r, N1, a, N1) &&
                           !ranges_overlap(r, N1, part2->a, N2) && !ranges_overlap(part2->r, N2, a, N1) &&
                           !ranges_overlap(part2->r, N2, part2->a, N2) &&
                           (bconst || (!ranges_overlap(r, N1, b, N1) && !ranges_overlap(r, N1, part2->b, N2) &&
                                       !ranges_overlap(part2->r, N2, b, N1) &&
                                       !ranges_overlap(part2->r, N2, part2->b, N2)));
        if (N1 % TL != 0 || !apart) {
            const u64 np1 = N1 / n;
            bn_status st = launch_flat_scan_mem(ctx, sub, r, a, b, n, np1, nullptr, bconst, bval, carry, s, fixed, -1,
                                                nullptr, nullptr, swap);
            if (st != BN_OK) return st;
            return second_alone(np1);
        }
    }
    const u64 ntiles = (N + TL - 1) / TL;
    if (chain) {
        if (fixed) {
            if (ntiles > fixed->max_tiles) return BN_ERANGE;
        } else {
            bn_status st = bn_ensure(ctx, ctx->status, scan_state_bytes(ntiles), s);
            if (st != BN_OK) return st;
        }
    }
    if (ntiles > 0x7fffffffull) return BN_ERANGE;
    scan_fn f = nullptr;
    if (ext == EXT_CIN)
        f = sub ? pick_ext<true, EXT_CIN>(vec, chain) : pick_ext<false, EXT_CIN>(vec, chain);
    else if (ext == (EXT_CIN | EXT_BCONST))
        f = sub ? pick_ext<true, EXT_CIN | EXT_BCONST>(vec, chain) : pick_ext<false, EXT_CIN | EXT_BCONST>(vec, chain);
    else if (ext == EXT_BCONST && !sub)
        f = pick_ext<false, EXT_BCONST>(vec, chain, rows);
    else if (ext == EXT_BZX)
        f = sub ? pick_ext<true, EXT_BZX>(vec, chain) : pick_ext<false, EXT_BZX>(vec, chain);
    else if (ext == EXT_COMB && !sub)
        f = pick_ext<false, EXT_COMB>(vec, chain, rows);
    else if (ext == EXT_SWAP && sub)
        f = pick_ext<true, EXT_SWAP>(vec, chain, rows);
    else if (ext != 0)
        return BN_EINVAL;
    else if (vec)
        f = sub ? (chain ? pick<true, true>(waves, rows) : pick<true, false>(waves, rows))
                : (chain ? pick<false, true>(waves, rows) : pick<false, false>(waves, rows));
    else if (chain)
        f = sub ? k_flat_scan<true, UNALIGNED_CHAIN_WAVES, UNALIGNED_CHAIN_ROWS, false, true>
                : k_flat_scan<false, UNALIGNED_CHAIN_WAVES, UNALIGNED_CHAIN_ROWS, false, true>;
    else
        f = sub ? k_flat_scan<true, UNALIGNED_BATCH_WAVES, UNALIGNED_BATCH_ROWS, false, false>
                : k_flat_scan<false, UNALIGNED_BATCH_WAVES, UNALIGNED_BATCH_ROWS, false, false>;
    if (!f) return BN_EINVAL;
    // Chained launches outside a stream capture take a fresh epoch from a host counter
    // (its range, from 2^61 up, is disjoint from the control block's, which counts up
    // from its initial value); captured ones read the control block and bump it after.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (chain && hipStreamIsCapturing(s, &cs) != hipSuccess) return BN_EHIP;
    const bool captured = cs != hipStreamCaptureStatusNone;
    u64 epoch = 0;
    if (chain && !captured) epoch = fixed ? fixed->host_epoch->fetch_add(1) + 1 : ++ctx->host_epoch;
    // r overlapping an operand: a waiting tile must not read another tile's operands
    const bool inplace =  // (two-part launches: every array is apart, checked above)
        !part2 && (ranges_overlap(r, N, a, N) || (!bconst && ranges_overlap(r, N, b, bzx ? (u64)nbz * npairs : N)));
    u32 dbg = ctx->tune.debug_flags & (fixed ? fixed->dbg_mask : ~0u);
    if (inplace) dbg &= ~1u;
    // deferred all-propagate tiles from `addsub.defer_tiles` tiles up (the silent-tile-0
    // debug mode keeps the waiting form: the status scan needs every tile's word)
    const u64 dt = ctx->tune.defer_tiles;
    const bool defer = chain && dt > 0 && ntiles >= dt && (dbg & 1u) == 0 && !part2;
    ScanCtl *ctl = fixed ? fixed->ctl : ctx->ctl;
    u64 *status = fixed ? fixed->status : (u64 *)ctx->status.ptr;
    uint8_t *codes = chain ? reinterpret_cast<uint8_t *>(status + (fixed ? fixed->max_tiles : ntiles)) : nullptr;
    ScanGeom G{N, n, -1, TL, epoch, cin, npairs, bval, inplace ? 1u : 0u, bzx ? (u64)nbz : 0, defer ? 1u : 0u, codes};
    if ((n & (n - 1)) == 0) G.nshift = __builtin_ctzll(n);
    if (comb) G.comb = *comb;
    if (swap) G.swap = *swap;
    if (part2) {
        G.N1 = N1;
        G.r2 = part2->r;
        G.a2 = part2->a;
        G.b2 = bconst ? nullptr : part2->b;
    }
    hipLaunchKernelGGL(f, dim3((u32)ntiles), dim3(waves * 64), 0, s, r, a, b, G, (u64)(128 % n), (u64)(128 / n), carry,
                       ctl, status, ctx->tune.spin_limit, dbg);
    bn_status st = bn_launch_status();
    if (st == BN_OK && defer) {
        hipLaunchKernelGGL(k_defer_scan, dim3(1), dim3(DS_THREADS), 0, s, status, codes, ntiles, epoch, ctl);
        if ((st = bn_launch_status()) != BN_OK) return st;
        const u64 fill_blocks = std::min<u64>(ntiles, 8 * (u64)std::max(1, ctx->num_cu));
        hipLaunchKernelGGL(sub ? k_defer_fill<true> : k_defer_fill<false>, dim3((u32)fill_blocks), dim3(256), 0, s, r,
                           codes, ntiles, TL, N, n, carry);
        st = bn_launch_status();
    }
    if (st != BN_OK || !chain || !captured) return st;
    hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(1), 0, s, ctl);
    return bn_launch_status();
}

bn_status launch_flat_scan_ext(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs,
                               const u64 *cin, bool bconst, u64 bval, u64 *carry, hipStream_t s) {
    return launch_flat_scan_mem(ctx, sub, r, a, b, n, npairs, cin, bconst, bval, carry, s, nullptr, -1);
}

bn_status launch_flat_scan_comb(bn_ctx *ctx, u64 *r, const ScanComb &comb, u64 out, u64 N, hipStream_t s) {
    return launch_flat_scan_mem(ctx, false, r, nullptr, nullptr, out, N, nullptr, false, 0, nullptr, s, nullptr, -1,
                                &comb);
}

bn_status launch_flat_scan_bzx(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, u64 na, const u64 *b, u64 nb,
                               u64 npairs, u64 *carry, hipStream_t s) {
    return launch_flat_scan_mem(ctx, sub, r, a, b, na, npairs, nullptr, false, 0, carry, s, nullptr, (i64)nb);
}

bn_status launch_flat_scan(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs, u64 *carry,
                           hipStream_t s) {
    return launch_flat_scan_ext(ctx, sub, r, a, b, n, npairs, nullptr, false, 0, carry, s);
}
