// tune.hip -- in-library autotuner: times candidate tile shapes and the mad/MFMA
// crossover on the current device and stores the winners in the context.
#include <stdio.h>

#include <algorithm>
#include <string>
#include <vector>

#include "bn_internal.h"
#include "bn_mul_dev.h"

namespace {

// Random 32-bit words for the probes' operands (the rates depend on the data).
__device__ __forceinline__ int rate_hash(u32 x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return (int)x;
}

// Rate probes.  k_rate_mac96: eight independent chains per lane of the plain form's
// instruction pair (v_mad_u64_u32 + v_addc_co_u32, one 32x32 -> 96-bit accumulate), on
// random digits as in a product: the wave-uniform digit changes every iteration, the
// lanes' digits are random.
__global__ __launch_bounds__(256) void k_rate_mac96(u64 *out, u32 x, u32 y, int iters) {
    const u32 l = threadIdx.x + 256u * blockIdx.x;
    u64 lo[8];
    u32 hi[8], yk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        lo[k] = threadIdx.x + k;
        hi[k] = 0;
        yk[k] = (u32)rate_hash(l * 8 + k + y);
    }
    for (int i = 0; i < iters; ++i) {
        const u32 xi = x ^ ((u32)i * 0x9e3779b9u);
#pragma unroll
        for (int k = 0; k < 8; ++k) mac96(lo[k], hi[k], xi, yk[k]);
    }
    u64 sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) sum += lo[k] + hi[k];
    out[blockIdx.x * (u64)blockDim.x + threadIdx.x] = sum;
}

// k_rate_mfma: four independent accumulators per wave of v_mfma_i32_32x32x32_i8 on
// operand bytes that look like a product's digits: hashed (random) bytes, two operand
// sets alternating so that consecutive MFMAs see different bits.  The rate depends on
// the data: the same loop on small constant bytes (mostly zero) runs about 25% faster
// (the part draws less power and holds a higher clock).
__global__ __launch_bounds__(256) void k_rate_mfma(int *out, int iters) {
    const u32 l = threadIdx.x + 256u * blockIdx.x;
    const v4i p{rate_hash(l), rate_hash(l + 77), rate_hash(l + 991), rate_hash(l + 12345)};
    const v4i q{rate_hash(3 * l + 1), rate_hash(5 * l + 2), rate_hash(7 * l + 3), rate_hash(11 * l + 4)};
    const v4i p2 = p ^ v4i{0x5a5a5a5a, (int)0xa5a5a5a5, 0x3c3c3c3c, (int)0xc3c3c3c3};
    v16i acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = v16i{0};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8((k & 1) ? p2 : p, q, acc[k], 0, 0, 0);
    u32 sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < 16; ++e) sum += (u32)acc[k][e];
    out[blockIdx.x * (u64)blockDim.x + threadIdx.x] = (int)sum;
}

__global__ void k_fill_random(u64 *p, u64 n, u64 seed) {
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        // splitmix64 of (seed, i): scratch operands only
        u64 z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        p[i] = z ^ (z >> 31);
    }
}

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Timer() {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
    }
    ~Timer() {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
};

// median of `reps` timed runs of f (after one warm-up), in ms
template <class F>
float time_ms(F &&f, int reps = 5) {
    Timer t;
    std::vector<float> v;
    f();
    (void)hipDeviceSynchronize();
    for (int i = 0; i < reps; ++i) {
        (void)hipEventRecord(t.e0, nullptr);
        f();
        (void)hipEventRecord(t.e1, nullptr);
        (void)hipEventSynchronize(t.e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, t.e0, t.e1);
        v.push_back(ms);
    }
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
}

// k_rate_copy: the streaming reference for the add/sub roofline -- 16 bytes per lane,
// non-temporal loads and stores, as the scan kernel moves its operands.  A workgroup
// copies one tile of 256 U vectors: U coalesced loads in flight per lane, then the
// stores.  The grid covers the array exactly (n a multiple of 256 U).
typedef u64 u64v2t __attribute__((ext_vector_type(2)));
template <int U>
__global__ __launch_bounds__(256) void k_rate_copy(u64v2t *__restrict__ dst, const u64v2t *__restrict__ src) {
    const u64 base = (u64)blockIdx.x * 256 * U + threadIdx.x;
    u64v2t v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = __builtin_nontemporal_load(src + base + 256 * j);
#pragma unroll
    for (int j = 0; j < U; ++j) __builtin_nontemporal_store(v[j], dst + base + 256 * j);
}

}  // namespace

extern "C" bn_status bn_probe_rates(bn_ctx *ctx, double *mac96_per_s, double *mfma_i8_ops_per_s,
                                    double *copy_bytes_per_s) {
    if (!ctx || !mac96_per_s || !mfma_i8_ops_per_s || !copy_bytes_per_s) return BN_EINVAL;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(ctx->device) != hipSuccess) return BN_EHIP;
    const u64 cus = (u64)std::max(1, ctx->num_cu);
    const u64 bm = cus * 16, bf = cus * 8;  // resident waves: 16 and 8 per CU
    const int im = 4096, iff = 1024;
    void *out = nullptr;
    if (hipMalloc(&out, bm * 256 * sizeof(u64)) != hipSuccess) {
        (void)hipSetDevice(prev);
        return BN_ENOMEM;
    }
    const float tm = time_ms([&] {
        hipLaunchKernelGGL(k_rate_mac96, dim3((u32)bm), dim3(256), 0, nullptr, (u64 *)out, 3u, 5u, im);
    });
    const float tf = time_ms([&] {
        hipLaunchKernelGGL(k_rate_mfma, dim3((u32)bf), dim3(256), 0, nullptr, (int *)out, iff);
    });
    bool ok = hipGetLastError() == hipSuccess;
    (void)hipDeviceSynchronize();
    (void)hipFree(out);
    // streaming copy of 512 MiB
    const u64 nv = (512ull << 20) / 16;
    void *src = nullptr, *dst = nullptr;
    float tc = 0;
    if (hipMalloc(&src, nv * 16) != hipSuccess || hipMalloc(&dst, nv * 16) != hipSuccess) {
        if (src) (void)hipFree(src);
        (void)hipSetDevice(prev);
        return BN_ENOMEM;
    }
    (void)hipMemset(src, 0x5a, nv * 16);
    // the fastest of three tile depths
    auto run_copy = [&](auto kernel, u64 per_block) {
        return time_ms([&] {
            hipLaunchKernelGGL(kernel, dim3((u32)(nv / per_block)), dim3(256), 0, nullptr, (u64v2t *)dst,
                               (const u64v2t *)src);
        });
    };
    tc = std::min({run_copy(k_rate_copy<2>, 512), run_copy(k_rate_copy<4>, 1024), run_copy(k_rate_copy<8>, 2048)});
    ok = ok && hipGetLastError() == hipSuccess;
    (void)hipDeviceSynchronize();
    (void)hipFree(src);
    (void)hipFree(dst);
    (void)hipSetDevice(prev);
    if (!ok || tm <= 0 || tf <= 0 || tc <= 0) return BN_EHIP;
    *mac96_per_s = (double)bm * 256 * im * 8 / (tm * 1e-3);
    // per wave and iteration: 4 MFMAs of 32 x 32 x 32 multiply-adds, 2 ops each
    *mfma_i8_ops_per_s = (double)bf * 4 * iff * 4 * 32768.0 * 2 / (tf * 1e-3);
    *copy_bytes_per_s = 2.0 * nv * 16 / (tc * 1e-3);  // bytes read + bytes written
    return BN_OK;
}

// The autotuner's own calls may grow the context's workspace (it is synchronous and
// never captured); the scope ends with the call.
struct GrowScope {
    bn_ctx *ctx;
    explicit GrowScope(bn_ctx *c) : ctx(c) { ctx->grow_scope = true; }
    ~GrowScope() { ctx->grow_scope = false; }
};

extern "C" bn_status bn_autotune(bn_ctx *ctx, const char *out_json) {
    if (!ctx) return BN_EINVAL;
    GrowScope grow(ctx);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    const u64 NBIG = 1ull << 24;  // limbs per operand for the add/sub sweep
    u64 *a = nullptr, *b = nullptr, *r = nullptr;
    if (hipMalloc(&a, NBIG * 8) != hipSuccess || hipMalloc(&b, NBIG * 8) != hipSuccess ||
        hipMalloc(&r, 2 * NBIG * 8) != hipSuccess) {
        (void)hipFree(a);
        (void)hipFree(b);
        (void)hipFree(r);
        (void)hipSetDevice(prev);
        return BN_ENOMEM;
    }
    hipLaunchKernelGGL(k_fill_random, dim3(1024), dim3(256), 0, nullptr, a, NBIG, 1ull);
    hipLaunchKernelGGL(k_fill_random, dim3(1024), dim3(256), 0, nullptr, b, NBIG, 2ull);
    (void)hipDeviceSynchronize();
    Tuning &t = ctx->tune;
    std::string log;

    // 1) add/sub tile shapes: independent tiles (64-limb pairs) and chained tiles (one
    //    operand pair spanning the whole array).  Chained shapes are scored on random
    //    operands and on the all-propagate worst case (all-ones + 1: the carry crosses
    //    every tile), by the sum of times relative to each input's best shape.
    const int shapes[][2] = {{1, 1}, {1, 2}, {2, 1}, {4, 1}, {8, 1}, {8, 2}, {2, 8}, {4, 4}, {4, 8}, {8, 4}};
    constexpr int NS = sizeof shapes / sizeof shapes[0];
    {
        float best = 1e30f;
        int bw = 1, br = 1;
        for (auto &sh : shapes) {
            t.batch_waves = sh[0];
            t.batch_rows = sh[1];
            const float ms = time_ms([&] { launch_flat_scan(ctx, false, r, a, b, 64, NBIG / 64, nullptr, nullptr); });
            if (ms < best) {
                best = ms;
                bw = sh[0];
                br = sh[1];
            }
        }
        t.batch_waves = bw;
        t.batch_rows = br;
    }
    {
        u64 *wa = nullptr, *wb = nullptr;
        if (hipMalloc(&wa, NBIG * 8) != hipSuccess || hipMalloc(&wb, NBIG * 8) != hipSuccess) {
            (void)hipFree(wa);
            (void)hipFree(wb);
            (void)hipFree(a);
            (void)hipFree(b);
            (void)hipFree(r);
            (void)hipSetDevice(prev);
            return BN_ENOMEM;
        }
        (void)launch_fill_u64(wa, NBIG, ~0ull, nullptr);
        (void)launch_fill_u64(wb, NBIG, 0ull, nullptr);
        (void)launch_fill_u64(wb, 1, 1ull, nullptr);
        float tms[2][NS] = {};
        for (int in = 0; in < 2; ++in)
            for (int k = 0; k < NS; ++k) {
                t.chain_waves = shapes[k][0];
                t.chain_rows = shapes[k][1];
                tms[in][k] = time_ms(
                    [&] { launch_flat_scan(ctx, false, r, in ? wa : a, in ? wb : b, NBIG, 1, nullptr, nullptr); });
            }
        (void)hipDeviceSynchronize();
        (void)hipFree(wa);
        (void)hipFree(wb);
        float best[2] = {1e30f, 1e30f};
        for (int in = 0; in < 2; ++in)
            for (int k = 0; k < NS; ++k) best[in] = std::min(best[in], tms[in][k]);
        int bk = 0;
        float bscore = 1e30f;
        for (int k = 0; k < NS; ++k) {
            const float score = tms[0][k] / best[0] + tms[1][k] / best[1];
            if (score < bscore) {
                bscore = score;
                bk = k;
            }
        }
        t.chain_waves = shapes[bk][0];
        t.chain_rows = shapes[bk][1];
    }

    // 2) mad vs MFMA crossovers, equal total work per shape.  The one-wave range
    // (mul_small_range) from square products, the larger range from products of a
    // 2048-limb operand with a shorter one of s limbs (the crossover is a bound on the
    // shorter length, and squares of more than 512 limbs would only test it from 1024
    // up); each range gets the smallest length from which MFMA wins at every larger one.
    i64 crossover = -1, small_crossover = -1;
    for (u64 n = 4; n <= 4096; n *= 2) {
        u64 npairs = std::max<u64>(1, std::min<u64>((1ull << 26) / (n * n), NBIG / n));
        npairs = std::min<u64>(npairs, 65535);
        const float tm = time_ms([&] { launch_mul_batch(ctx, r, a, b, n, n, npairs, BN_MUL_MAD, nullptr); }, 3);
        const float tf = time_ms([&] { launch_mul_batch(ctx, r, a, b, n, n, npairs, BN_MUL_MFMA, nullptr); }, 3);
        char line[160];
        snprintf(line, sizeof line, "    \"sweep.n%llu\": \"mad %.4f ms, mfma %.4f ms, pairs %llu\",\n",
                 (unsigned long long)n, tm, tf, (unsigned long long)npairs);
        log += line;
        if (!mul_small_range(2 * n)) continue;
        if (tf < tm) {
            if (small_crossover < 0) small_crossover = (i64)n;
        } else {
            small_crossover = -1;
        }
    }
    for (u64 sl = 1; sl <= 2048; sl *= 2) {
        const u64 nl = 2048;
        u64 npairs = std::max<u64>(1, std::min<u64>((1ull << 26) / (nl * sl), NBIG / nl));
        npairs = std::min<u64>(npairs, 65535);
        const float tm = time_ms([&] { launch_mul_batch(ctx, r, a, b, nl, sl, npairs, BN_MUL_MAD, nullptr); }, 3);
        const float tf = time_ms([&] { launch_mul_batch(ctx, r, a, b, nl, sl, npairs, BN_MUL_MFMA, nullptr); }, 3);
        char line[160];
        snprintf(line, sizeof line, "    \"sweep.n2048x%llu\": \"mad %.4f ms, mfma %.4f ms, pairs %llu\",\n",
                 (unsigned long long)sl, tm, tf, (unsigned long long)npairs);
        log += line;
        if (tf < tm) {
            if (crossover < 0) crossover = (i64)sl;
        } else {
            crossover = -1;
        }
    }
    t.mul_crossover_limbs = crossover > 0 ? crossover : (i64)1 << 40;
    t.mul_small_crossover_limbs = small_crossover > 0 ? small_crossover : (i64)1 << 40;

    // 3) staging window of the large MFMA kernel: by size (0) or one fixed window, on
    // 64 products of 16384 limbs and 576 of 4096 limbs (the bottom of two Karatsuba
    // levels on C5), candidates interleaved over five rounds; the winner has the lowest
    // sum of times relative to the best time of each shape, and a fixed window replaces
    // the size rule only when it is better by more than 1% (the noise of this sweep)
    {
        const int cand[] = {0, 192, 224, 234, 256};
        constexpr int NC = sizeof cand / sizeof cand[0];
        const u64 shape[2][2] = {{16384, 64}, {4096, 576}};
        float tms[2][NC] = {};
        // (the first timing after a change of shape ran a few percent slow: an untimed
        // launch goes first, and the candidates' order rotates from round to round)
        constexpr int ROUNDS = NC;
        for (int round = 0; round < ROUNDS; ++round)
            for (int sh = 0; sh < 2; ++sh) {
                const u64 n = shape[sh][0], np = shape[sh][1];
                (void)launch_mul_batch(ctx, r, a, b, n, n, np, BN_MUL_MFMA, nullptr);
                for (int k = 0; k < NC; ++k) {
                    const int c = (k + round) % NC;
                    t.mfma_chunk = cand[c];
                    tms[sh][c] += time_ms([&] { launch_mul_batch(ctx, r, a, b, n, n, np, BN_MUL_MFMA, nullptr); }, 3);
                }
            }
        float best[2] = {1e30f, 1e30f};
        for (int sh = 0; sh < 2; ++sh)
            for (int c = 0; c < NC; ++c) best[sh] = std::min(best[sh], tms[sh][c]);
        int bc = 0;
        float bscore = 1e30f;
        for (int c = 0; c < NC; ++c) {
            const float score = tms[0][c] / best[0] + tms[1][c] / best[1];
            char line[128];
            snprintf(line, sizeof line, "    \"sweep.mfma_chunk%d\": \"%.4f ms (16384 x 64), %.4f ms (4096 x 576)\",\n",
                     cand[c], tms[0][c] / ROUNDS, tms[1][c] / ROUNDS);
            log += line;
            if (c == 0 || score < bscore - 0.02f) {
                bscore = score;
                bc = c;
            }
        }
        t.mfma_chunk = cand[bc];
    }
    (void)hipDeviceSynchronize();
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(r);
    (void)hipSetDevice(prev);
    if (out_json) {
        FILE *f = fopen(out_json, "w");
        if (!f) return BN_EINVAL;
        fprintf(f, "{\n%s", log.c_str());
        fprintf(f, "    \"addsub.batch_waves\": %d,\n    \"addsub.batch_rows\": %d,\n", t.batch_waves, t.batch_rows);
        fprintf(f, "    \"addsub.chain_waves\": %d,\n    \"addsub.chain_rows\": %d,\n", t.chain_waves, t.chain_rows);
        fprintf(f, "    \"mul.crossover_limbs\": %lld,\n", (long long)t.mul_crossover_limbs);
        fprintf(f, "    \"mul.small_crossover_limbs\": %lld,\n", (long long)t.mul_small_crossover_limbs);
        fprintf(f, "    \"mul.mad_xchunk\": %d,\n    \"mul.mfma_chunk\": %d,\n    \"mul.mfma_rows\": %d\n}\n",
                t.mad_xchunk, t.mfma_chunk, t.mfma_rows);
        fclose(f);
    }
    return BN_OK;
}
