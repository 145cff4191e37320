/* bn_c_check.c -- the library's C ABI driven from plain C (no Python, no torch): a
 * context, device buffers from the HIP runtime's C API, a caller-created stream, and
 * uniform-batch add, subtract and multiply calls checked against closed forms:
 *   (X^n - 1) + v          = v - 1 with carry 1             (Theorem 1, full carry chain)
 *   0 - v                  = X^n - v with borrow 1           (the borrow mirror)
 *   (X^n - 1)^2            = X^(2n) - 2 X^n + 1              (Theorem 2, both forms)
 * with X = 2^64, plus the synchronous argument errors.  Prints "ok" and returns 0 when
 * every check holds; otherwise prints the first failure and returns 1. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "bn.h"

#define ONES UINT64_MAX

static int fail(const char *what, size_t i, uint64_t got, uint64_t want) {
    printf("FAIL %s at %zu: got %016llx want %016llx\n", what, i, (unsigned long long)got, (unsigned long long)want);
    return 1;
}

#define HIP_OK(x)                                                      \
    do {                                                               \
        if ((x) != hipSuccess) {                                       \
            printf("FAIL hip call %s\n", #x);                          \
            return 1;                                                  \
        }                                                              \
    } while (0)
#define BN_OK_(x)                                                      \
    do {                                                               \
        bn_status s_ = (x);                                            \
        if (s_ != BN_OK) {                                             \
            printf("FAIL %s: %s\n", #x, bn_strerror(s_));              \
            return 1;                                                  \
        }                                                              \
    } while (0)

/* Batched add and subtract of npairs pairs of n limbs. */
static int check_addsub(bn_ctx *ctx, hipStream_t st, size_t n, size_t npairs) {
    const size_t N = n * npairs;
    uint64_t *ha = malloc(N * 8), *hb = malloc(N * 8), *hr = malloc(N * 8), *hc = malloc(npairs * 8);
    uint64_t *da, *db, *dr, *dc;
    if (!ha || !hb || !hr || !hc) return 1;
    HIP_OK(hipMalloc((void **)&da, N * 8));
    HIP_OK(hipMalloc((void **)&db, N * 8));
    HIP_OK(hipMalloc((void **)&dr, N * 8));
    HIP_OK(hipMalloc((void **)&dc, npairs * 8));
    BN_OK_(bn_reserve_for(ctx, BN_OP_ADDSUB, n, 0, npairs, BN_MUL_AUTO, 0));
    /* add: a = X^n - 1, b = p + 1 (one limb) */
    for (size_t p = 0; p < npairs; ++p)
        for (size_t i = 0; i < n; ++i) {
            ha[p * n + i] = ONES;
            hb[p * n + i] = i == 0 ? (uint64_t)p + 1 : 0;
        }
    HIP_OK(hipMemcpy(da, ha, N * 8, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(db, hb, N * 8, hipMemcpyHostToDevice));
    BN_OK_(bn_add_n_batch(ctx, dr, da, db, n, npairs, dc, (bn_stream)st));
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipMemcpy(hr, dr, N * 8, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hc, dc, npairs * 8, hipMemcpyDeviceToHost));
    for (size_t p = 0; p < npairs; ++p) {
        if (hc[p] != 1) return fail("add carry", p, hc[p], 1);
        for (size_t i = 0; i < n; ++i) {
            const uint64_t want = i == 0 ? (uint64_t)p : 0;
            if (hr[p * n + i] != want) return fail("add", p * n + i, hr[p * n + i], want);
        }
    }
    /* sub: a = 0, b = p + 1 */
    memset(ha, 0, N * 8);
    HIP_OK(hipMemcpy(da, ha, N * 8, hipMemcpyHostToDevice));
    BN_OK_(bn_sub_n_batch(ctx, dr, da, db, n, npairs, dc, (bn_stream)st));
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipMemcpy(hr, dr, N * 8, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hc, dc, npairs * 8, hipMemcpyDeviceToHost));
    for (size_t p = 0; p < npairs; ++p) {
        if (hc[p] != 1) return fail("sub borrow", p, hc[p], 1);
        for (size_t i = 0; i < n; ++i) {
            const uint64_t want = i == 0 ? (uint64_t)0 - ((uint64_t)p + 1) : ONES;
            if (hr[p * n + i] != want) return fail("sub", p * n + i, hr[p * n + i], want);
        }
    }
    /* argument errors return at once and enqueue nothing */
    if (bn_add_n_batch(ctx, dr, NULL, db, n, npairs, dc, (bn_stream)st) != BN_EINVAL)
        return fail("NULL operand refused", 0, 0, 0);
    if (bn_add_n_batch(ctx, (uint64_t *)((char *)dr + 4), da, db, n, npairs, dc, (bn_stream)st) != BN_EINVAL)
        return fail("misaligned result refused", 0, 0, 0);
    HIP_OK(hipFree(da));
    HIP_OK(hipFree(db));
    HIP_OK(hipFree(dr));
    HIP_OK(hipFree(dc));
    free(ha);
    free(hb);
    free(hr);
    free(hc);
    return 0;
}

/* (X^n - 1)^2 for npairs pairs on the given form. */
static int check_square(bn_ctx *ctx, hipStream_t st, size_t n, size_t npairs, int form) {
    const size_t N = n * npairs, R = 2 * n * npairs;
    uint64_t *ha = malloc(N * 8), *hr = malloc(R * 8);
    uint64_t *da, *dr;
    if (!ha || !hr) return 1;
    for (size_t i = 0; i < N; ++i) ha[i] = ONES;
    HIP_OK(hipMalloc((void **)&da, N * 8));
    HIP_OK(hipMalloc((void **)&dr, R * 8));
    HIP_OK(hipMemcpy(da, ha, N * 8, hipMemcpyHostToDevice));
    BN_OK_(bn_reserve_for(ctx, BN_OP_MUL, n, n, npairs, form, 0));
    BN_OK_(bn_mul_n_batch(ctx, dr, da, da, n, n, npairs, form, (bn_stream)st));
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipMemcpy(hr, dr, R * 8, hipMemcpyDeviceToHost));
    for (size_t p = 0; p < npairs; ++p)
        for (size_t j = 0; j < 2 * n; ++j) {
            const uint64_t want = j == 0 ? 1 : j < n ? 0 : j == n ? ONES - 1 : ONES;
            if (hr[p * 2 * n + j] != want) {
                printf("form %d n %zu: ", form, n);
                return fail("square", p * 2 * n + j, hr[p * 2 * n + j], want);
            }
        }
    HIP_OK(hipFree(da));
    HIP_OK(hipFree(dr));
    free(ha);
    free(hr);
    return 0;
}

int main(void) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        printf("FAIL no GPU\n");
        return 1;
    }
    printf("%s\n", bn_version());
    bn_ctx *ctx = NULL;
    BN_OK_(bn_create(&ctx, 0, NULL));
    hipStream_t st;
    HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    int bad = 0;
    bad |= check_addsub(ctx, st, 37, 300);       /* pairs cross tiles: look-back */
    bad |= check_addsub(ctx, st, 64, 4096);      /* independent tiles */
    bad |= check_addsub(ctx, st, 1 << 20, 1);    /* one pair over many workgroups */
    bad |= check_square(ctx, st, 100, 7, BN_MUL_MAD);
    bad |= check_square(ctx, st, 100, 7, BN_MUL_MFMA);
    bad |= check_square(ctx, st, 1500, 2, BN_MUL_MAD);
    bad |= check_square(ctx, st, 1500, 2, BN_MUL_MFMA);
    if (bn_create(NULL, 0, NULL) != BN_EINVAL) bad |= fail("NULL context pointer refused", 0, 0, 0);
    HIP_OK(hipStreamDestroy(st));
    BN_OK_(bn_destroy(ctx));
    if (bad) return 1;
    printf("ok\n");
    return 0;
}
