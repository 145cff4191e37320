// k_addsub_ext.hip -- add/sub beyond equal-length pairs without carry-in: a carry
// (borrow) into limb 0, unequal operand lengths, and |a - b| with its sign.  All of
// them run on the flat scan kernel (its carry-in and zero-extended-b variants) plus one
// streaming select kernel.
#include "bn_internal.h"

#include <algorithm>

namespace {

// r[p] = neg[p] ? alt[p] : r[p] for N = n * npairs limbs (pair p = limbs [p n, (p+1) n)).
__global__ void k_select_pairs(u64 *__restrict__ r, const u64 *__restrict__ alt, const u64 *__restrict__ neg, u64 n,
                               u64 N) {
    for (u64 idx = blockIdx.x * (u64)blockDim.x + threadIdx.x; idx < N; idx += (u64)gridDim.x * blockDim.x)
        if (neg[idx / n] & 1ull) r[idx] = alt[idx];
}

}  // namespace

bn_status launch_addsub_nc(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs,
                           const u64 *cin, u64 *carry, hipStream_t s) {
    return launch_flat_scan_ext(ctx, sub, r, a, b, n, npairs, cin, false, 0, carry, s);
}

// r_p[0, na) = a_p +- b_p with b_p zero-extended to na limbs (na >= nb), for every
// pair: equal lengths take the plain scan, otherwise one pass of the scan whose b
// reads as zero past nb limbs per pair.
bn_status launch_addsub_unequal(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, u64 na, const u64 *b, u64 nb,
                                u64 npairs, u64 *carry, hipStream_t s) {
    if (na == nb) return launch_flat_scan(ctx, sub, r, a, b, na, npairs, carry, s);
    return launch_flat_scan_bzx(ctx, sub, r, a, na, b, nb, npairs, carry, s);
}

// Status words of an unequal-length add/sub batch.
WsNeed unequal_need(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs) {
    WsNeed w;
    if (npairs == 0 || na == 0) return w;
    w.status = na == nb ? flat_scan_status_bytes(ctx, na, na * npairs) : flat_scan_ext_status_bytes(na, na * npairs);
    return w;
}

// r = |a - b| per pair, sign[p] = [a_p < b_p].  b - a goes to a scratch array first,
// so r may be a or b exactly.
bn_status launch_sub_abs(bn_ctx *ctx, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs, u64 *sign,
                         hipStream_t s) {
    const u64 N = n * npairs;
    if (N == 0) return sign ? launch_fill_u64(sign, npairs, 0, s) : BN_OK;
    bn_status st = bn_ensure(ctx, ctx->kwork, (N + npairs) * sizeof(u64), s);
    if (st != BN_OK) return st;
    u64 *alt = static_cast<u64 *>(ctx->kwork.ptr);
    u64 *neg = sign ? sign : alt + N;
    if ((st = launch_flat_scan(ctx, true, alt, b, a, n, npairs, nullptr, s)) != BN_OK) return st;
    if ((st = launch_flat_scan(ctx, true, r, a, b, n, npairs, neg, s)) != BN_OK) return st;
    const u64 blocks = std::max<u64>(1, std::min<u64>((N + 255) / 256, 65536));
    hipLaunchKernelGGL(k_select_pairs, dim3((u32)blocks), dim3(256), 0, s, r, alt, neg, n, N);
    return bn_launch_status();
}
