// tune.hip -- in-library autotuner: times candidate tile shapes and the mad/MFMA
// crossover on the current device and stores the winners in the context.
#include <stdio.h>

#include <algorithm>
#include <string>
#include <vector>

#include "bn_internal.h"

namespace {

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

}  // namespace

extern "C" bn_status bn_autotune(bn_ctx *ctx, const char *out_json) {
    if (!ctx) return BN_EINVAL;
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

    // 1) add/sub tile shapes: independent tiles (64-limb pairs) and chained tiles
    //    (one operand pair spanning the whole array)
    const int shapes[][2] = {{1, 1}, {1, 2}, {2, 1}, {4, 1}, {8, 1}, {8, 2}, {2, 8}, {4, 4}, {4, 8}, {8, 4}};
    for (int mode = 0; mode < 2; ++mode) {
        float best = 1e30f;
        int bw = 1, br = 1;
        for (auto &sh : shapes) {
            if (mode == 0) {
                t.batch_waves = sh[0];
                t.batch_rows = sh[1];
            } else {
                t.chain_waves = sh[0];
                t.chain_rows = sh[1];
            }
            const u64 n = mode == 0 ? 64 : NBIG;
            const float ms =
                time_ms([&] { launch_flat_scan(ctx, false, r, a, b, n, NBIG / n, nullptr, nullptr); });
            if (ms < best) {
                best = ms;
                bw = sh[0];
                br = sh[1];
            }
        }
        if (mode == 0) {
            t.batch_waves = bw;
            t.batch_rows = br;
        } else {
            t.chain_waves = bw;
            t.chain_rows = br;
        }
    }

    // 2) mad vs MFMA crossover: square products, equal total work per size
    i64 crossover = -1;
    bool mfma_wins_all_after = true;
    for (u64 n = 8; n <= 4096; n *= 2) {
        u64 npairs = std::max<u64>(1, std::min<u64>((1ull << 26) / (n * n), NBIG / n));
        npairs = std::min<u64>(npairs, 65535);
        const float tm = time_ms([&] { launch_mul_batch(ctx, r, a, b, n, n, npairs, BN_MUL_MAD, nullptr); }, 3);
        const float tf = time_ms([&] { launch_mul_batch(ctx, r, a, b, n, n, npairs, BN_MUL_MFMA, nullptr); }, 3);
        char line[160];
        snprintf(line, sizeof line, "    \"sweep.n%llu\": \"mad %.4f ms, mfma %.4f ms, pairs %llu\",\n",
                 (unsigned long long)n, tm, tf, (unsigned long long)npairs);
        log += line;
        if (tf < tm) {
            if (crossover < 0) crossover = (i64)n;
        } else if (crossover >= 0) {
            mfma_wins_all_after = false;
            crossover = -1;
        }
    }
    (void)mfma_wins_all_after;
    t.mul_crossover_limbs = crossover > 0 ? crossover : (i64)1 << 40;
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
        fprintf(f, "    \"mul.mad_xchunk\": %d,\n    \"mul.mfma_chunk\": %d\n}\n", t.mad_xchunk, t.mfma_chunk);
        fclose(f);
    }
    return BN_OK;
}
