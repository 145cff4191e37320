// dot_host.c -- DoT addition and subtraction on x86-64 SIMD (Sec. 3.1, Algorithm 1).
//
// One step handles w limb pairs held in one vector register:
//   phase 1  r = a + b lane by lane;
//   phase 2  g = lanes whose sum wrapped (r < a), as a bit mask; the carry out of the
//            step is g's top bit, and the carries to add are (g << 1) | c_in;
//   phase 3  r' = r + those carries; a lane wraps again only if it held 2^64 - 1;
//   phase 4  (rare) the lanes wrapped by phase 3 start a cascade through the lanes
//            equal to 2^64 - 1.  With s = (wrap << 1) + m, m the mask of such lanes,
//            the lanes that receive a carry are s ^ m and the carry out of the step
//            also takes s >> w: the Kogge-Stone integer-add trick on the masks.
// Subtraction is the mirror image: borrows are [a < b], the cascade runs through
// zero limbs.  Steps are chained by their carry, w = 8 limbs with AVX-512 (mask
// registers) and w = 4 with AVX2 (bit masks from movemask, lane vectors from a
// table); the last partial step uses masked loads and stores.  Functions carry
// their own target attributes, so the library builds without -march flags and picks
// the ISA at run time.
#include "bn_host.h"

#include <immintrin.h>
#include <pthread.h>
#include <stdlib.h>

typedef uint64_t (*step_fn)(uint64_t *, const uint64_t *, const uint64_t *, size_t, uint64_t);

// ------------------------------------------------------------------ scalar ----
static uint64_t add_scalar(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t c) {
    unsigned char cf = (unsigned char)c;
    for (size_t i = 0; i < n; ++i) {
        unsigned long long t;
        cf = _addcarry_u64(cf, a[i], b[i], &t);
        r[i] = t;
    }
    return cf;
}

static uint64_t sub_scalar(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t c) {
    unsigned char bf = (unsigned char)c;
    for (size_t i = 0; i < n; ++i) {
        unsigned long long t;
        bf = _subborrow_u64(bf, a[i], b[i], &t);
        r[i] = t;
    }
    return bf;
}

// ----------------------------------------------------------------- AVX-512 ----
// One step over the lanes in `lanes` (all 8 but in the last step).  `w` is the
// number of valid lanes; invalid lanes load as zero and are never stored.
__attribute__((target("avx512f"))) static inline uint64_t add8(uint64_t *r, const uint64_t *a, const uint64_t *b,
                                                               uint64_t c, unsigned w, __mmask8 lanes) {
    const __m512i ones = _mm512_set1_epi64(-1);
    const __m512i va = _mm512_maskz_loadu_epi64(lanes, a), vb = _mm512_maskz_loadu_epi64(lanes, b);
    const __m512i vr = _mm512_add_epi64(va, vb);                               // phase 1
    const unsigned g = _mm512_cmplt_epu64_mask(vr, va);                          // phase 2
    uint64_t cout = (g >> (w - 1)) & 1u;
    const __mmask8 cm = (__mmask8)(((g << 1) | (unsigned)c) & lanes);
    __m512i vr2 = _mm512_mask_sub_epi64(vr, cm, vr, ones);                      // phase 3: +1
    const unsigned wrap = _mm512_mask_cmplt_epu64_mask(cm, vr2, vr);
    if (wrap) {                                                                  // phase 4
        const unsigned m = _mm512_mask_cmpeq_epi64_mask(lanes, vr2, ones);
        const unsigned s = (wrap << 1) + m;
        cout |= (s >> w) != 0;
        vr2 = _mm512_mask_sub_epi64(vr2, (__mmask8)((s ^ m) & lanes), vr2, ones);
    }
    _mm512_mask_storeu_epi64(r, lanes, vr2);
    return cout;
}

__attribute__((target("avx512f"))) static inline uint64_t sub8(uint64_t *r, const uint64_t *a, const uint64_t *b,
                                                               uint64_t c, unsigned w, __mmask8 lanes) {
    const __m512i ones = _mm512_set1_epi64(-1), zero = _mm512_setzero_si512();
    const __m512i va = _mm512_maskz_loadu_epi64(lanes, a), vb = _mm512_maskz_loadu_epi64(lanes, b);
    const __m512i vr = _mm512_sub_epi64(va, vb);
    const unsigned g = _mm512_cmplt_epu64_mask(va, vb);  // borrows
    uint64_t cout = (g >> (w - 1)) & 1u;
    const __mmask8 cm = (__mmask8)(((g << 1) | (unsigned)c) & lanes);
    __m512i vr2 = _mm512_mask_add_epi64(vr, cm, vr, ones);  // -1
    const unsigned wrap = _mm512_mask_cmplt_epu64_mask(cm, vr, vr2);  // 0 became 2^64 - 1
    if (wrap) {
        const unsigned m = _mm512_mask_cmpeq_epi64_mask(lanes, vr2, zero);
        const unsigned s = (wrap << 1) + m;
        cout |= (s >> w) != 0;
        vr2 = _mm512_mask_add_epi64(vr2, (__mmask8)((s ^ m) & lanes), vr2, ones);
    }
    _mm512_mask_storeu_epi64(r, lanes, vr2);
    return cout;
}

__attribute__((target("avx512f"))) static uint64_t add_avx512(uint64_t *r, const uint64_t *a, const uint64_t *b,
                                                              size_t n, uint64_t c) {
    size_t i = 0;
    for (; i + 8 <= n; i += 8) c = add8(r + i, a + i, b + i, c, 8, 0xff);
    if (i < n) c = add8(r + i, a + i, b + i, c, (unsigned)(n - i), (__mmask8)((1u << (n - i)) - 1));
    return c;
}

__attribute__((target("avx512f"))) static uint64_t sub_avx512(uint64_t *r, const uint64_t *a, const uint64_t *b,
                                                              size_t n, uint64_t c) {
    size_t i = 0;
    for (; i + 8 <= n; i += 8) c = sub8(r + i, a + i, b + i, c, 8, 0xff);
    if (i < n) c = sub8(r + i, a + i, b + i, c, (unsigned)(n - i), (__mmask8)((1u << (n - i)) - 1));
    return c;
}

// -------------------------------------------------------------------- AVX2 ----
// LANE[k]: all-ones in the lanes whose bit is set in k.
static const int64_t LANE[16][4] __attribute__((aligned(32))) = {
    {0, 0, 0, 0},   {-1, 0, 0, 0},   {0, -1, 0, 0},   {-1, -1, 0, 0},   {0, 0, -1, 0},   {-1, 0, -1, 0},
    {0, -1, -1, 0}, {-1, -1, -1, 0}, {0, 0, 0, -1},   {-1, 0, 0, -1},   {0, -1, 0, -1},  {-1, -1, 0, -1},
    {0, 0, -1, -1}, {-1, 0, -1, -1}, {0, -1, -1, -1}, {-1, -1, -1, -1}};

__attribute__((target("avx2"))) static inline __m256i lane_vec(unsigned k) {
    return _mm256_load_si256((const __m256i *)LANE[k & 15u]);
}

// bit i set iff x_i < y_i as unsigned 64-bit numbers
__attribute__((target("avx2"))) static inline unsigned ltu4(__m256i x, __m256i y) {
    const __m256i sb = _mm256_set1_epi64x(INT64_MIN);
    const __m256i gt = _mm256_cmpgt_epi64(_mm256_xor_si256(y, sb), _mm256_xor_si256(x, sb));
    return (unsigned)_mm256_movemask_pd(_mm256_castsi256_pd(gt));
}

__attribute__((target("avx2"))) static inline unsigned eq4(__m256i x, __m256i y) {
    return (unsigned)_mm256_movemask_pd(_mm256_castsi256_pd(_mm256_cmpeq_epi64(x, y)));
}

__attribute__((target("avx2"))) static inline uint64_t add4(uint64_t *r, const uint64_t *a, const uint64_t *b,
                                                            uint64_t c, unsigned w, unsigned lanes) {
    const __m256i lv = lane_vec(lanes);
    const __m256i va = _mm256_maskload_epi64((const long long *)a, lv);
    const __m256i vb = _mm256_maskload_epi64((const long long *)b, lv);
    const __m256i vr = _mm256_add_epi64(va, vb);
    const unsigned g = ltu4(vr, va);
    uint64_t cout = (g >> (w - 1)) & 1u;
    const unsigned cm = ((g << 1) | (unsigned)c) & lanes;
    __m256i vr2 = _mm256_sub_epi64(vr, lane_vec(cm));  // +1 in the carry lanes
    const unsigned wrap = ltu4(vr2, vr) & cm;
    if (wrap) {
        const unsigned m = eq4(vr2, _mm256_set1_epi64x(-1)) & lanes;
        const unsigned s = (wrap << 1) + m;
        cout |= (s >> w) != 0;
        vr2 = _mm256_sub_epi64(vr2, lane_vec((s ^ m) & lanes));
    }
    _mm256_maskstore_epi64((long long *)r, lv, vr2);
    return cout;
}

__attribute__((target("avx2"))) static inline uint64_t sub4(uint64_t *r, const uint64_t *a, const uint64_t *b,
                                                            uint64_t c, unsigned w, unsigned lanes) {
    const __m256i lv = lane_vec(lanes);
    const __m256i va = _mm256_maskload_epi64((const long long *)a, lv);
    const __m256i vb = _mm256_maskload_epi64((const long long *)b, lv);
    const __m256i vr = _mm256_sub_epi64(va, vb);
    const unsigned g = ltu4(va, vb);
    uint64_t cout = (g >> (w - 1)) & 1u;
    const unsigned cm = ((g << 1) | (unsigned)c) & lanes;
    __m256i vr2 = _mm256_add_epi64(vr, lane_vec(cm));  // -1 in the borrow lanes
    const unsigned wrap = ltu4(vr, vr2) & cm;
    if (wrap) {
        const unsigned m = eq4(vr2, _mm256_setzero_si256()) & lanes;
        const unsigned s = (wrap << 1) + m;
        cout |= (s >> w) != 0;
        vr2 = _mm256_add_epi64(vr2, lane_vec((s ^ m) & lanes));
    }
    _mm256_maskstore_epi64((long long *)r, lv, vr2);
    return cout;
}

__attribute__((target("avx2"))) static uint64_t add_avx2(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                                                         uint64_t c) {
    size_t i = 0;
    for (; i + 4 <= n; i += 4) c = add4(r + i, a + i, b + i, c, 4, 0xf);
    if (i < n) c = add4(r + i, a + i, b + i, c, (unsigned)(n - i), (1u << (n - i)) - 1);
    return c;
}

__attribute__((target("avx2"))) static uint64_t sub_avx2(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                                                         uint64_t c) {
    size_t i = 0;
    for (; i + 4 <= n; i += 4) c = sub4(r + i, a + i, b + i, c, 4, 0xf);
    if (i < n) c = sub4(r + i, a + i, b + i, c, (unsigned)(n - i), (1u << (n - i)) - 1);
    return c;
}

// ---------------------------------------------------------------- dispatch ----
int bnh_isa_best(void) {
    __builtin_cpu_init();
    if (__builtin_cpu_supports("avx512f")) return BNH_ISA_AVX512;
    if (__builtin_cpu_supports("avx2")) return BNH_ISA_AVX2;
    return BNH_ISA_SCALAR;
}

static int pick(int isa, int sub, step_fn *f) {
    if (isa < BNH_ISA_SCALAR || isa > BNH_ISA_AVX512) return BNH_EINVAL;
    if (isa > bnh_isa_best()) return BNH_EUNSUPPORTED;
    static const step_fn table[2][3] = {{add_scalar, add_avx2, add_avx512}, {sub_scalar, sub_avx2, sub_avx512}};
    *f = table[sub][isa];
    return BNH_OK;
}

static int one(int sub, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t cin, uint64_t *cout,
               int isa) {
    step_fn f;
    const int st = pick(isa, sub, &f);
    if (st != BNH_OK) return st;
    if (n && (!r || !a || !b)) return BNH_EINVAL;
    if (cin > 1) return BNH_EINVAL;
    const uint64_t c = f(r, a, b, n, cin);
    if (cout) *cout = c;
    return BNH_OK;
}

int bnh_add_n(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t carry_in, uint64_t *carry_out,
              int isa) {
    return one(0, r, a, b, n, carry_in, carry_out, isa);
}

int bnh_sub_n(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t borrow_in, uint64_t *borrow_out,
              int isa) {
    return one(1, r, a, b, n, borrow_in, borrow_out, isa);
}

typedef struct {
    step_fn f;
    uint64_t *r, *carry;
    const uint64_t *a, *b;
    size_t n, p0, p1;
    pthread_t tid;
    int running;  // on a thread of its own (else run on the calling thread)
} range_job;

static void *run_range(void *arg) {
    const range_job *j = (const range_job *)arg;
    for (size_t p = j->p0; p < j->p1; ++p) {
        const uint64_t c = j->f(j->r + p * j->n, j->a + p * j->n, j->b + p * j->n, j->n, 0);
        if (j->carry) j->carry[p] = c;
    }
    return NULL;
}

static int batch(int sub, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs, uint64_t *carry,
                 int isa, int threads) {
    step_fn f;
    const int st = pick(isa, sub, &f);
    if (st != BNH_OK) return st;
    if (threads < 1) return BNH_EINVAL;
    if (npairs && n && (!r || !a || !b)) return BNH_EINVAL;
    if ((size_t)threads > npairs) threads = npairs ? (int)npairs : 1;
    range_job *jobs = (range_job *)calloc((size_t)threads, sizeof(range_job));
    if (!jobs) return BNH_EINVAL;
    for (int t = 0; t < threads; ++t) {
        jobs[t].f = f;
        jobs[t].r = r;
        jobs[t].carry = carry;
        jobs[t].a = a;
        jobs[t].b = b;
        jobs[t].n = n;
        jobs[t].p0 = npairs * (size_t)t / (size_t)threads;
        jobs[t].p1 = npairs * (size_t)(t + 1) / (size_t)threads;
    }
    for (int t = 1; t < threads; ++t) jobs[t].running = pthread_create(&jobs[t].tid, NULL, run_range, &jobs[t]) == 0;
    run_range(&jobs[0]);
    for (int t = 1; t < threads; ++t) {
        if (jobs[t].running)
            pthread_join(jobs[t].tid, NULL);
        else
            run_range(&jobs[t]);  // no thread could be started: run the range here
    }
    free(jobs);
    return BNH_OK;
}

int bnh_add_n_batch(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs, uint64_t *carry_out,
                    int isa, int threads) {
    return batch(0, r, a, b, n, npairs, carry_out, isa, threads);
}

int bnh_sub_n_batch(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs, uint64_t *carry_out,
                    int isa, int threads) {
    return batch(1, r, a, b, n, npairs, carry_out, isa, threads);
}
