// bn_api.hip -- the C ABI: contexts, argument validation, workspace, dispatch,
// parameters, HIP-graph capture.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <string>

#include "bn_internal.h"

#define BN_VERSION_STRING "bn-mi355x 0.1.0 (gfx950)"

bool flat_scan_shape_ok(int waves, int rows);

bn_status bn_launch_status() { return hipGetLastError() == hipSuccess ? BN_OK : BN_EHIP; }

bn_status bn_grow(bn_ctx *ctx, DevBuf &buf, size_t bytes) {
    if (buf.bytes >= bytes) return BN_OK;
    size_t want = std::max(bytes, buf.bytes + buf.bytes / 2);
    want = (want + 65535) & ~(size_t)65535;
    if (buf.ptr) {
        if (hipDeviceSynchronize() != hipSuccess) return BN_EHIP;
        // a captured graph may still address the old buffer: keep it until bn_destroy
        if (ctx->captured)
            ctx->retired.push_back(buf.ptr);
        else
            (void)hipFree(buf.ptr);
        buf.ptr = nullptr;
        buf.bytes = 0;
    }
    if (hipMalloc(&buf.ptr, want) != hipSuccess) {
        buf.ptr = nullptr;
        return BN_ENOMEM;
    }
    // status words must start below every epoch in use (epoch >= 1); the clear runs on
    // the null stream, so wait for it before a kernel on a non-blocking stream reads them
    if (hipMemset(buf.ptr, 0, want) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return BN_EHIP;
    buf.bytes = want;
    return BN_OK;
}

bn_status bn_ensure(bn_ctx *ctx, DevBuf &buf, size_t bytes, hipStream_t s) {
    if (buf.bytes >= bytes) return BN_OK;
    if (!ctx->tune.auto_grow && !ctx->grow_scope) return BN_ENOSPACE;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return BN_EHIP;
    if (cs != hipStreamCaptureStatusNone) return BN_ECAPTURE;
    return bn_grow(ctx, buf, bytes);
}

bn_status ws_reserve(bn_ctx *ctx, const WsNeed &need) {
    bn_status st;
    if ((st = bn_grow(ctx, ctx->status, need.status)) != BN_OK) return st;
    if ((st = bn_grow(ctx, ctx->work, need.work)) != BN_OK) return st;
    if ((st = bn_grow(ctx, ctx->kwork, need.kwork)) != BN_OK) return st;
    return bn_grow(ctx, ctx->mstage, need.mstage);
}

// Every buffer a call needs, checked (or grown, with auto_grow) before anything is
// enqueued: a short workspace fails the call with nothing launched.
static bn_status ws_acquire(bn_ctx *ctx, const WsNeed &need, hipStream_t s) {
    bn_status st;
    if ((st = bn_ensure(ctx, ctx->status, need.status, s)) != BN_OK) return st;
    if ((st = bn_ensure(ctx, ctx->work, need.work, s)) != BN_OK) return st;
    if ((st = bn_ensure(ctx, ctx->kwork, need.kwork, s)) != BN_OK) return st;
    return bn_ensure(ctx, ctx->mstage, need.mstage, s);
}

// ------------------------------------------------------------------ helpers ----
static bool overlaps(const void *x, size_t xbytes, const void *y, size_t ybytes) {
    const uintptr_t a0 = (uintptr_t)x, a1 = a0 + xbytes, b0 = (uintptr_t)y, b1 = b0 + ybytes;
    return xbytes && ybytes && a0 < b1 && b0 < a1;
}

static bool mul_overflow(size_t a, size_t b, size_t *out) { return __builtin_mul_overflow(a, b, out); }

static bn_status check_ptr(const void *p, size_t limbs) {
    if (limbs == 0) return BN_OK;
    if (!p) return BN_EINVAL;
    if ((uintptr_t)p & 7u) return BN_EINVAL;
    return BN_OK;
}

static inline hipStream_t S(bn_stream s) { return reinterpret_cast<hipStream_t>(s); }

// Workspace of one call (BN_OP_* of bn.h; in_place for multiplications whose output
// overlaps an operand).  The same quantities the launch code checks, taken at their
// largest over the operand alignments the call may see.
static WsNeed ws_need_for(const bn_ctx *ctx, int op, size_t na, size_t nb, size_t npairs, int form, int levels,
                          bool in_place) {
    WsNeed w;
    switch (op) {
        case BN_OP_ADDSUB:
            w.status = flat_scan_status_bytes(ctx, na, (u64)na * npairs);
            break;
        case BN_OP_ADDSUB_NC:
            w.status = flat_scan_ext_status_bytes(na, (u64)na * npairs);
            break;
        case BN_OP_ADDSUB_UNEQUAL:
            w = unequal_need(ctx, na, nb, npairs);
            break;
        case BN_OP_SUB_ABS:
            w.status = flat_scan_status_bytes(ctx, na, (u64)na * npairs);
            w.kwork = ((u64)na * npairs + npairs) * sizeof(u64);
            break;
        case BN_OP_MUL:
            w.work = mul_workspace_bytes(ctx, na, nb, npairs, form);
            w.status = mul_status_bytes(ctx, na, nb, npairs, form);
            if (in_place) w.mstage = (na + nb) * npairs * sizeof(u64);
            break;
        case BN_OP_MUL_KARATSUBA:
            if (levels == BN_KARATSUBA_AUTO) levels = karatsuba_auto_levels(ctx, na, nb);
            w = karatsuba_need(ctx, na, nb, npairs, levels, form);
            if (in_place) w.mstage = (na + nb) * npairs * sizeof(u64);
            break;
        default:
            break;
    }
    return w;
}

static bool op_valid(int op) { return op >= BN_OP_ADDSUB && op <= BN_OP_MUL_KARATSUBA; }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// ------------------------------------------------------------------ context ----
// Levels of BN_KARATSUBA_AUTO for na x nb products: none when one length is below half
// the other (both are zero-extended to the longer one, which would cost more than the
// recursion saves).
int karatsuba_auto_levels(const bn_ctx *ctx, u64 na, u64 nb) {
    const u64 lo = std::min(na, nb), hi = std::max(na, nb);
    if (2 * lo < hi) return 0;
    return bn_karatsuba_auto_levels(hi, (size_t)ctx->tune.karatsuba_limbs);
}

extern "C" {

const char *bn_version(void) { return BN_VERSION_STRING; }

const char *bn_strerror(bn_status s) {
    switch (s) {
        case BN_OK: return "ok";
        case BN_EINVAL: return "invalid argument";
        case BN_EALIAS: return "output overlaps an input";
        case BN_ERANGE: return "size out of range";
        case BN_ENOMEM: return "device allocation failed";
        case BN_EHIP: return "HIP runtime error";
        case BN_EUNSUPPORTED: return "unsupported device or feature";
        case BN_ECAPTURE: return "workspace must grow during stream capture (call bn_reserve_for first)";
        case BN_ENOSPACE: return "workspace too small for this call (call bn_reserve_for first)";
        default: return "unknown status";
    }
}

static bn_status load_tuning(bn_ctx *ctx, const char *path);

bn_status bn_create(bn_ctx **out, int device, const char *tuning_json) {
    if (!out) return BN_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return BN_EUNSUPPORTED;
    if (device < 0 || device >= ndev) return BN_EINVAL;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return BN_EHIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BN_EUNSUPPORTED;
    DeviceGuard g(device);
    bn_ctx *ctx = new bn_ctx();
    ctx->device = device;
    ctx->num_cu = prop.multiProcessorCount;
    if (hipMalloc(&ctx->ctl, sizeof(ScanCtl)) != hipSuccess) {
        delete ctx;
        return BN_ENOMEM;
    }
    ScanCtl init{};
    init.epoch = 1;
    if (hipMemcpy(ctx->ctl, &init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(ctx->ctl);
        delete ctx;
        return BN_EHIP;
    }
    if (scratch_setup(device) != BN_OK) {  // once per device: the no-allocation entry point's array
        (void)hipFree(ctx->ctl);
        delete ctx;
        return BN_EHIP;
    }
    if (tuning_json) {
        const bn_status st = load_tuning(ctx, tuning_json);
        if (st != BN_OK) {
            (void)hipFree(ctx->ctl);
            delete ctx;
            return st;
        }
    }
    *out = ctx;
    return BN_OK;
}

bn_status bn_destroy(bn_ctx *ctx) {
    if (!ctx) return BN_OK;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->status.ptr) (void)hipFree(ctx->status.ptr);
    if (ctx->work.ptr) (void)hipFree(ctx->work.ptr);
    if (ctx->kwork.ptr) (void)hipFree(ctx->kwork.ptr);
    if (ctx->mstage.ptr) (void)hipFree(ctx->mstage.ptr);
    if (ctx->ctl) (void)hipFree(ctx->ctl);
    for (void *p : ctx->retired) (void)hipFree(p);
    delete ctx;
    return BN_OK;
}

bn_status bn_reserve(bn_ctx *ctx, size_t bytes) {
    if (!ctx) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    return bn_grow(ctx, ctx->work, bytes);
}

bn_status bn_reserve_for(bn_ctx *ctx, int op, size_t na, size_t nb, size_t npairs, int form, int levels) {
    if (!ctx || !op_valid(op & ~BN_OP_IN_PLACE)) return BN_EINVAL;
    if (form != BN_MUL_AUTO && form != BN_MUL_MAD && form != BN_MUL_MFMA) return BN_EINVAL;
    if (levels != BN_KARATSUBA_AUTO && (levels < 0 || levels > BN_KARATSUBA_MAX_LEVELS)) return BN_EINVAL;
    size_t t;
    if (na > BN_MAX_LIMBS || nb > BN_MAX_LIMBS || mul_overflow(na + nb, npairs, &t) || t > 2 * BN_MAX_LIMBS)
        return BN_ERANGE;
    DeviceGuard g(ctx->device);
    return ws_reserve(ctx, ws_need_for(ctx, op & ~BN_OP_IN_PLACE, na, nb, npairs, form, levels,
                                       (op & BN_OP_IN_PLACE) != 0));
}

size_t bn_workspace_size(bn_ctx *ctx, int op, size_t na, size_t nb, size_t npairs, int form, int levels) {
    if (!ctx || !op_valid(op & ~BN_OP_IN_PLACE)) return 0;
    size_t t;
    if (na > BN_MAX_LIMBS || nb > BN_MAX_LIMBS || mul_overflow(na + nb, npairs, &t) || t > 2 * BN_MAX_LIMBS) return 0;
    const WsNeed w =
        ws_need_for(ctx, op & ~BN_OP_IN_PLACE, na, nb, npairs, form, levels, (op & BN_OP_IN_PLACE) != 0);
    return w.status + w.work + w.kwork + w.mstage;
}

bn_status bn_lookback_stats(bn_ctx *ctx, bn_stream stream, uint64_t *hist, size_t nbins) {
    if (!ctx || (!hist && nbins)) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    if (hipStreamSynchronize(S(stream)) != hipSuccess) return BN_EHIP;
    u64 h[LOOKBACK_BINS];
    if (hipMemcpy(h, ctx->ctl->hist, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return BN_EHIP;
    const u64 zero[LOOKBACK_BINS] = {};
    if (hipMemcpy(ctx->ctl->hist, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return BN_EHIP;
    for (size_t i = 0; i < nbins; ++i) hist[i] = i < (size_t)LOOKBACK_BINS ? h[i] : 0;
    return BN_OK;
}

bn_status bn_check(bn_ctx *ctx, bn_stream stream, uint32_t *flags) {
    if (!ctx) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    if (hipStreamSynchronize(S(stream)) != hipSuccess) return BN_EHIP;
    u64 err = 0;
    if (hipMemcpy(&err, &ctx->ctl->err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return BN_EHIP;
    const u64 zero = 0;
    if (hipMemcpy(&ctx->ctl->err, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return BN_EHIP;
    if (flags) *flags = (uint32_t)err;
    return BN_OK;
}

// --------------------------------------------------------------- add / sub ----
// fixed: look-back state in the per-GPU scratch array instead of the context's workspace
static bn_status addsub(bn_ctx *ctx, bool sub, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                        size_t npairs, uint64_t *carry, bn_stream stream, const ScanMem *fixed = nullptr) {
    if (!ctx) return BN_EINVAL;
    size_t N;
    if (mul_overflow(n, npairs, &N) || N > BN_MAX_LIMBS) return BN_ERANGE;
    bn_status st;
    if ((st = check_ptr(r, N)) || (st = check_ptr(a, N)) || (st = check_ptr(b, N))) return st;
    if (carry && ((uintptr_t)carry & 7u)) return BN_EINVAL;
    const size_t bytes = N * 8;
    if ((r != a && overlaps(r, bytes, a, bytes)) || (r != b && overlaps(r, bytes, b, bytes))) return BN_EALIAS;
    if (carry && (overlaps(carry, npairs * 8, r, bytes) || overlaps(carry, npairs * 8, a, bytes) ||
                  overlaps(carry, npairs * 8, b, bytes)))
        return BN_EALIAS;
    DeviceGuard g(ctx->device);
    if (fixed) {  // the status words of either operand alignment must fit the array
        if (flat_scan_status_bytes(ctx, n, N) > scan_state_bytes(fixed->max_tiles)) return BN_ERANGE;
        return launch_flat_scan_mem(ctx, sub, r, a, b, n, npairs, nullptr, false, 0, carry, S(stream), fixed);
    }
    if ((st = ws_acquire(ctx, ws_need_for(ctx, BN_OP_ADDSUB, n, n, npairs, 0, 0, false), S(stream))) != BN_OK)
        return st;
    return launch_flat_scan(ctx, sub, r, a, b, n, npairs, carry, S(stream));
}

static bn_status addsub_nc(bn_ctx *ctx, bool sub, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                           size_t npairs, const uint64_t *cin, uint64_t *carry, bn_stream stream) {
    if (!ctx) return BN_EINVAL;
    if (!cin && npairs) return BN_EINVAL;
    if (cin && ((uintptr_t)cin & 7u)) return BN_EINVAL;
    size_t N;
    if (mul_overflow(n, npairs, &N) || N > BN_MAX_LIMBS) return BN_ERANGE;
    bn_status st;
    if ((st = check_ptr(r, N)) || (st = check_ptr(a, N)) || (st = check_ptr(b, N))) return st;
    if (carry && ((uintptr_t)carry & 7u)) return BN_EINVAL;
    const size_t bytes = N * 8;
    if ((r != a && overlaps(r, bytes, a, bytes)) || (r != b && overlaps(r, bytes, b, bytes))) return BN_EALIAS;
    if (carry && (overlaps(carry, npairs * 8, r, bytes) || overlaps(carry, npairs * 8, a, bytes) ||
                  overlaps(carry, npairs * 8, b, bytes) || overlaps(carry, npairs * 8, cin, npairs * 8)))
        return BN_EALIAS;  // (a segment's carry-in and carry-out may be read and written by different workgroups)
    if (cin && overlaps(cin, npairs * 8, r, bytes)) return BN_EALIAS;
    DeviceGuard g(ctx->device);
    if (N == 0) {  // no limbs: the carry passes through
        if (!carry || npairs == 0) return BN_OK;
        return hipMemcpyAsync(carry, cin, npairs * 8, hipMemcpyDeviceToDevice, S(stream)) == hipSuccess ? BN_OK
                                                                                                : BN_EHIP;
    }
    if ((st = ws_acquire(ctx, ws_need_for(ctx, BN_OP_ADDSUB_NC, n, n, npairs, 0, 0, false), S(stream))) != BN_OK)
        return st;
    return launch_addsub_nc(ctx, sub, r, a, b, n, npairs, cin, carry, S(stream));
}

bn_status bn_add(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t *carry_out,
                 bn_stream stream) {
    return addsub(ctx, false, r, a, b, n, 1, carry_out, stream);
}

bn_status bn_sub(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t *borrow_out,
                 bn_stream stream) {
    return addsub(ctx, true, r, a, b, n, 1, borrow_out, stream);
}

bn_status bn_add_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs,
                         uint64_t *carry_out, bn_stream stream) {
    return addsub(ctx, false, r, a, b, n, npairs, carry_out, stream);
}

bn_status bn_sub_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs,
                         uint64_t *borrow_out, bn_stream stream) {
    return addsub(ctx, true, r, a, b, n, npairs, borrow_out, stream);
}

bn_status bn_addsub_n_batch_noalloc(bn_ctx *ctx, int sub, uint64_t *r, const uint64_t *a, const uint64_t *b,
                                     size_t n, size_t npairs, uint64_t *carry_out, bn_stream stream) {
    if (!ctx || (sub != 0 && sub != 1)) return BN_EINVAL;
    ScanMem m;
    if (!scratch_mem(ctx->device, &m)) return BN_EUNSUPPORTED;
    return addsub(ctx, sub != 0, r, a, b, n, npairs, carry_out, stream, &m);
}

bn_status bn_add_nc_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs,
                            const uint64_t *carry_in, uint64_t *carry_out, bn_stream stream) {
    return addsub_nc(ctx, false, r, a, b, n, npairs, carry_in, carry_out, stream);
}

bn_status bn_sub_nc_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs,
                            const uint64_t *borrow_in, uint64_t *borrow_out, bn_stream stream) {
    return addsub_nc(ctx, true, r, a, b, n, npairs, borrow_in, borrow_out, stream);
}

static bn_status addsub_unequal(bn_ctx *ctx, bool sub, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b,
                                size_t nb, size_t npairs, uint64_t *carry, bn_stream stream) {
    if (!ctx) return BN_EINVAL;
    if (na < nb) return BN_EINVAL;
    size_t NA, NB;
    if (mul_overflow(na, npairs, &NA) || NA > BN_MAX_LIMBS) return BN_ERANGE;
    NB = nb * npairs;  // nb <= na: cannot overflow
    bn_status st;
    if ((st = check_ptr(r, NA)) || (st = check_ptr(a, NA)) || (st = check_ptr(b, NB))) return st;
    if (carry && ((uintptr_t)carry & 7u)) return BN_EINVAL;
    // r may be a exactly, or b exactly when the lengths are equal
    if ((r != a && overlaps(r, NA * 8, a, NA * 8)) || (!(r == b && na == nb) && overlaps(r, NA * 8, b, NB * 8)))
        return BN_EALIAS;
    if (carry && (overlaps(carry, npairs * 8, r, NA * 8) || overlaps(carry, npairs * 8, a, NA * 8) ||
                  overlaps(carry, npairs * 8, b, NB * 8)))
        return BN_EALIAS;
    DeviceGuard g(ctx->device);
    if (NA == 0) return carry && npairs ? launch_fill_u64(carry, npairs, 0, S(stream)) : BN_OK;
    if ((st = ws_acquire(ctx, ws_need_for(ctx, BN_OP_ADDSUB_UNEQUAL, na, nb, npairs, 0, 0, false), S(stream))) !=
        BN_OK)
        return st;
    return launch_addsub_unequal(ctx, sub, r, a, na, b, nb, npairs, carry, S(stream));
}

bn_status bn_add_unequal(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b, size_t nb,
                         uint64_t *carry_out, bn_stream stream) {
    return addsub_unequal(ctx, false, r, a, na, b, nb, 1, carry_out, stream);
}

bn_status bn_sub_unequal(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b, size_t nb,
                         uint64_t *borrow_out, bn_stream stream) {
    return addsub_unequal(ctx, true, r, a, na, b, nb, 1, borrow_out, stream);
}

bn_status bn_add_unequal_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b,
                                 size_t nb, size_t npairs, uint64_t *carry_out, bn_stream stream) {
    return addsub_unequal(ctx, false, r, a, na, b, nb, npairs, carry_out, stream);
}

bn_status bn_sub_unequal_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b,
                                 size_t nb, size_t npairs, uint64_t *borrow_out, bn_stream stream) {
    return addsub_unequal(ctx, true, r, a, na, b, nb, npairs, borrow_out, stream);
}

bn_status bn_sub_abs_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                             size_t npairs, uint64_t *sign, bn_stream stream) {
    if (!ctx) return BN_EINVAL;
    size_t N;
    if (mul_overflow(n, npairs, &N) || N > BN_MAX_LIMBS) return BN_ERANGE;
    bn_status st;
    if ((st = check_ptr(r, N)) || (st = check_ptr(a, N)) || (st = check_ptr(b, N))) return st;
    if (sign && ((uintptr_t)sign & 7u)) return BN_EINVAL;
    const size_t bytes = N * 8;
    if ((r != a && overlaps(r, bytes, a, bytes)) || (r != b && overlaps(r, bytes, b, bytes))) return BN_EALIAS;
    if (sign && (overlaps(sign, npairs * 8, r, bytes) || overlaps(sign, npairs * 8, a, bytes) ||
                 overlaps(sign, npairs * 8, b, bytes)))
        return BN_EALIAS;
    DeviceGuard g(ctx->device);
    if ((st = ws_acquire(ctx, ws_need_for(ctx, BN_OP_SUB_ABS, n, n, npairs, 0, 0, false), S(stream))) != BN_OK)
        return st;
    return launch_sub_abs(ctx, r, a, b, n, npairs, sign, S(stream));
}

// ---------------------------------------------------------------- multiply ----
static bn_status mul_args(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t na, size_t nb,
                          size_t npairs, int form) {
    if (!ctx) return BN_EINVAL;
    if (form != BN_MUL_AUTO && form != BN_MUL_MAD && form != BN_MUL_MFMA) return BN_EINVAL;
    if (na > BN_MAX_LIMBS || nb > BN_MAX_LIMBS) return BN_ERANGE;
    size_t A, B, R;
    if (mul_overflow(na, npairs, &A) || mul_overflow(nb, npairs, &B) || mul_overflow(na + nb, npairs, &R) ||
        R > 2 * BN_MAX_LIMBS)
        return BN_ERANGE;
    bn_status st;
    if ((st = check_ptr(r, R)) || (st = check_ptr(a, A)) || (st = check_ptr(b, B))) return st;
    return BN_OK;
}

// A product whose output overlaps an operand is written to the context's staging
// buffer and copied into r after the last kernel that reads a or b.
static bool mul_in_place(const uint64_t *r, const uint64_t *a, const uint64_t *b, size_t na, size_t nb,
                         size_t npairs) {
    return overlaps(r, (na + nb) * npairs * 8, a, na * npairs * 8) || overlaps(r, (na + nb) * npairs * 8, b, nb * npairs * 8);
}

static bn_status mul_staged(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t na, size_t nb,
                            size_t npairs, hipStream_t s, const std::function<bn_status(u64 *)> &run) {
    if (!mul_in_place(r, a, b, na, nb, npairs)) return run(r);
    const size_t bytes = (na + nb) * npairs * 8;
    bn_status st = bn_ensure(ctx, ctx->mstage, bytes, s);
    if (st != BN_OK) return st;
    u64 *stage = static_cast<u64 *>(ctx->mstage.ptr);
    if ((st = run(stage)) != BN_OK) return st;
    return hipMemcpyAsync(r, stage, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess ? BN_OK : BN_EHIP;
}

bn_status bn_mul(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b, size_t nb, int form,
                 bn_stream stream) {
    bn_status st = mul_args(ctx, r, a, b, na, nb, 1, form);
    if (st != BN_OK) return st;
    DeviceGuard g(ctx->device);
    if ((st = ws_acquire(ctx, ws_need_for(ctx, BN_OP_MUL, na, nb, 1, form, 0, mul_in_place(r, a, b, na, nb, 1)),
                         S(stream))) != BN_OK)
        return st;
    return mul_staged(ctx, r, a, b, na, nb, 1, S(stream),
                      [&](u64 *out) { return launch_mul_batch(ctx, out, a, b, na, nb, 1, form, S(stream)); });
}

bn_status bn_mul_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t na, size_t nb,
                         size_t npairs, int form, bn_stream stream) {
    bn_status st = mul_args(ctx, r, a, b, na, nb, npairs, form);
    if (st != BN_OK) return st;
    DeviceGuard g(ctx->device);
    if ((st = ws_acquire(ctx,
                         ws_need_for(ctx, BN_OP_MUL, na, nb, npairs, form, 0, mul_in_place(r, a, b, na, nb, npairs)),
                         S(stream))) != BN_OK)
        return st;
    return mul_staged(ctx, r, a, b, na, nb, npairs, S(stream),
                      [&](u64 *out) { return launch_mul_batch(ctx, out, a, b, na, nb, npairs, form, S(stream)); });
}

int bn_karatsuba_auto_levels(size_t n, size_t min_half_limbs) {
    if (min_half_limbs == 0) min_half_limbs = 1;
    int levels = 0;
    size_t m = n;
    while (levels < BN_KARATSUBA_MAX_LEVELS && m >= 2 && (m + 1) / 2 >= min_half_limbs) {
        m = (m + 1) / 2;
        ++levels;
    }
    return levels;
}

bn_status bn_mul_karatsuba_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b,
                                 size_t nb, size_t npairs, int levels, int form, bn_stream stream) {
    bn_status st = mul_args(ctx, r, a, b, na, nb, npairs, form);
    if (st != BN_OK) return st;
    if (levels == BN_KARATSUBA_AUTO) levels = karatsuba_auto_levels(ctx, na, nb);
    if (levels < 0 || levels > BN_KARATSUBA_MAX_LEVELS) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    if ((st = ws_acquire(ctx,
                         ws_need_for(ctx, BN_OP_MUL_KARATSUBA, na, nb, npairs, form, levels,
                                     mul_in_place(r, a, b, na, nb, npairs)),
                         S(stream))) != BN_OK)
        return st;
    return mul_staged(ctx, r, a, b, na, nb, npairs, S(stream), [&](u64 *out) {
        return launch_mul_karatsuba(ctx, out, a, na, b, nb, npairs, levels, form, S(stream));
    });
}

bn_status bn_mul_karatsuba_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                                   size_t npairs, int levels, int form, bn_stream stream) {
    return bn_mul_karatsuba_batch(ctx, r, a, n, b, n, npairs, levels, form, stream);
}

// ------------------------------------------------------------------ ragged ----
bn_status bn_plan_mul_ragged(bn_ctx *ctx, const bn_pair *host_pairs, size_t npairs, int form, bn_plan **plan) {
    if (!ctx || !plan || (npairs && !host_pairs)) return BN_EINVAL;
    if (form != BN_MUL_AUTO && form != BN_MUL_MAD && form != BN_MUL_MFMA) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    bn_status st = plan_mul_ragged(ctx, host_pairs, npairs, form, plan);
    if (st != BN_OK) return st;
    // the plan's large items run through the batched path: its workspace, reserved now
    if ((st = ws_reserve(ctx, (*plan)->ws)) != BN_OK) {
        bn_plan_destroy(*plan);
        *plan = nullptr;
    }
    return st;
}

bn_status bn_plan_add_ragged(bn_ctx *ctx, const bn_pair *host_pairs, size_t npairs, bn_plan **plan) {
    if (!ctx || !plan || (npairs && !host_pairs)) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    return plan_add_ragged(ctx, host_pairs, npairs, plan);
}

bn_status bn_plan_destroy(bn_plan *plan) {
    if (!plan) return BN_OK;
    DeviceGuard g(plan->device);
    (void)hipDeviceSynchronize();
    if (plan->d_items) (void)hipFree(plan->d_items);
    if (plan->d_pairs) (void)hipFree(plan->d_pairs);
    delete plan;
    return BN_OK;
}

bn_status bn_mul_ragged(bn_ctx *ctx, const bn_plan *plan, uint64_t *r_pool, const uint64_t *a_pool,
                        const uint64_t *b_pool, bn_stream stream) {
    if (!ctx || !plan || plan->op != 0 || plan->device != ctx->device) return BN_EINVAL;
    if (plan->npairs && (!r_pool || !a_pool || !b_pool)) return BN_EINVAL;
    if (((uintptr_t)r_pool | (uintptr_t)a_pool | (uintptr_t)b_pool) & 7u) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    bn_status st = ws_acquire(ctx, plan->ws, S(stream));
    if (st != BN_OK) return st;
    return launch_mul_ragged(ctx, plan, r_pool, a_pool, b_pool, S(stream));
}

bn_status bn_add_ragged(bn_ctx *ctx, const bn_plan *plan, uint64_t *r_pool, const uint64_t *a_pool,
                        const uint64_t *b_pool, uint64_t *carry_out, bn_stream stream) {
    if (!ctx || !plan || plan->op != 1 || plan->device != ctx->device) return BN_EINVAL;
    if (plan->npairs && (!r_pool || !a_pool || !b_pool)) return BN_EINVAL;
    if (((uintptr_t)r_pool | (uintptr_t)a_pool | (uintptr_t)b_pool | (uintptr_t)carry_out) & 7u) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    return launch_add_ragged(ctx, plan, r_pool, a_pool, b_pool, carry_out, S(stream));
}

// ------------------------------------------------------------------ graphs ----
static bn_status capture(bn_stream stream, bn_graph **out, const std::function<bn_status()> &body);

bn_status bn_graph_capture_mul_ragged(bn_ctx *ctx, const bn_plan *plan, uint64_t *r_pool, const uint64_t *a_pool,
                                      const uint64_t *b_pool, bn_stream stream, bn_graph **graph) {
    if (!ctx || !plan || !graph || !stream || plan->op != 0 || plan->device != ctx->device) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    // large items use the batched pipeline: reserve its workspace before capture
    bn_status st;
    if ((st = ws_reserve(ctx, plan->ws)) != BN_OK) return st;
    ctx->captured = true;
    return capture(stream, graph, [&]() { return bn_mul_ragged(ctx, plan, r_pool, a_pool, b_pool, stream); });
}

bn_status bn_graph_capture_batch(bn_ctx *ctx, int op, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t na,
                                 size_t nb, size_t npairs, uint64_t *carry_out, int form, bn_stream stream,
                                 bn_graph **graph) {
    if (!ctx || !graph || !stream || op < 0 || op > 2) return BN_EINVAL;
    DeviceGuard g(ctx->device);
    bn_status st;
    if (op == 2) {
        if ((st = mul_args(ctx, r, a, b, na, nb, npairs, form)) != BN_OK) return st;
        if ((st = ws_reserve(ctx, ws_need_for(ctx, BN_OP_MUL, na, nb, npairs, form, 0,
                                              mul_in_place(r, a, b, na, nb, npairs)))) != BN_OK)
            return st;
        ctx->captured = true;
        return capture(stream, graph,
                       [&]() { return bn_mul_n_batch(ctx, r, a, b, na, nb, npairs, form, stream); });
    }
    if ((st = ws_reserve(ctx, ws_need_for(ctx, BN_OP_ADDSUB, na, na, npairs, 0, 0, false))) != BN_OK) return st;
    ctx->captured = true;
    return capture(stream, graph, [&]() {
        return op == 0 ? bn_add_n_batch(ctx, r, a, b, na, npairs, carry_out, stream)
                       : bn_sub_n_batch(ctx, r, a, b, na, npairs, carry_out, stream);
    });
}

bn_status bn_graph_launch(bn_graph *graph, bn_stream stream) {
    if (!graph || !graph->exec) return BN_EINVAL;
    return hipGraphLaunch(graph->exec, S(stream)) == hipSuccess ? BN_OK : BN_EHIP;
}

bn_status bn_graph_destroy(bn_graph *graph) {
    if (!graph) return BN_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return BN_OK;
}

// ------------------------------------------------------------------ params ----
static const char *kParamNames =
    "addsub.batch_waves,addsub.batch_rows,addsub.chain_waves,addsub.chain_rows,addsub.defer_tiles,"
    "mul.crossover_limbs,mul.small_crossover_limbs,mul.crossover_limbs_p64,mul.crossover_limbs_p128,mul.crossover_limbs_p256,mul.crossover_limbs_p512,mul.crossover_limbs_p1024,mul.mad_xchunk,mul.mfma_chunk,mul.mfma_rows,mul.karatsuba_limbs,"
    "ragged.pair_small,lookback.spin_limit,debug.flags,workspace.auto_grow";

const char *bn_param_names(void) { return kParamNames; }

bn_status bn_set_param(bn_ctx *ctx, const char *key, int64_t v) {
    if (!ctx || !key) return BN_EINVAL;
    Tuning &t = ctx->tune;
    const std::string k(key);
    if (k == "addsub.batch_waves" || k == "addsub.batch_rows") {
        const int w = k == "addsub.batch_waves" ? (int)v : t.batch_waves;
        const int r = k == "addsub.batch_rows" ? (int)v : t.batch_rows;
        if (!flat_scan_shape_ok(w, r)) return BN_EINVAL;
        t.batch_waves = w;
        t.batch_rows = r;
    } else if (k == "addsub.chain_waves" || k == "addsub.chain_rows") {
        const int w = k == "addsub.chain_waves" ? (int)v : t.chain_waves;
        const int r = k == "addsub.chain_rows" ? (int)v : t.chain_rows;
        if (!flat_scan_shape_ok(w, r)) return BN_EINVAL;
        t.chain_waves = w;
        t.chain_rows = r;
    } else if (k == "addsub.defer_tiles") {
        if (v < 0) return BN_EINVAL;
        t.defer_tiles = (u64)v;
    } else if (k == "mul.crossover_limbs") {
        if (v < 1) return BN_EINVAL;
        t.mul_crossover_limbs = v;
    } else if (k == "mul.small_crossover_limbs") {
        if (v < 1) return BN_EINVAL;
        t.mul_small_crossover_limbs = v;
    } else if (k == "mul.crossover_limbs_p64" || k == "mul.crossover_limbs_p128" || k == "mul.crossover_limbs_p256" ||
               k == "mul.crossover_limbs_p512" || k == "mul.crossover_limbs_p1024") {
        if (v < -1 || v == 0) return BN_EINVAL;
        (k == "mul.crossover_limbs_p64"    ? t.mul_crossover_p64
         : k == "mul.crossover_limbs_p128" ? t.mul_crossover_p128
         : k == "mul.crossover_limbs_p256" ? t.mul_crossover_p256
         : k == "mul.crossover_limbs_p512" ? t.mul_crossover_p512
                                           : t.mul_crossover_p1024) = v;
    } else if (k == "mul.mad_xchunk") {
        if (v < 64 || v > (1 << 20) || (v % 8)) return BN_EINVAL;
        t.mad_xchunk = (int)v;
    } else if (k == "mul.mfma_chunk") {
        if (v != 0 && (v < 16 || v > 256 || (v & 1))) return BN_EINVAL;  // even (steps run in pairs); staging registers
        t.mfma_chunk = (int)v;
    } else if (k == "mul.karatsuba_limbs") {
        if (v < 1) return BN_EINVAL;
        t.karatsuba_limbs = v;
    } else if (k == "mul.mfma_rows") {
        if (v != 1 && v != 2) return BN_EINVAL;
        t.mfma_rows = (int)v;
    } else if (k == "ragged.pair_small") {
        if (v != 0 && v != 1) return BN_EINVAL;
        t.ragged_pair = (int)v;
    } else if (k == "lookback.spin_limit") {
        if (v < 0 || v > 0xffffffffll) return BN_EINVAL;
        t.spin_limit = (u32)v;
    } else if (k == "debug.flags") {
        if (v < 0 || v > 3) return BN_EINVAL;
        t.debug_flags = (u32)v;
    } else if (k == "workspace.auto_grow") {
        if (v != 0 && v != 1) return BN_EINVAL;
        t.auto_grow = (int)v;
    } else {
        return BN_EINVAL;
    }
    return BN_OK;
}

bn_status bn_get_param(bn_ctx *ctx, const char *key, int64_t *v) {
    if (!ctx || !key || !v) return BN_EINVAL;
    const Tuning &t = ctx->tune;
    const std::string k(key);
    if (k == "addsub.batch_waves") *v = t.batch_waves;
    else if (k == "addsub.batch_rows") *v = t.batch_rows;
    else if (k == "addsub.chain_waves") *v = t.chain_waves;
    else if (k == "addsub.chain_rows") *v = t.chain_rows;
    else if (k == "addsub.defer_tiles") *v = (int64_t)t.defer_tiles;
    else if (k == "mul.crossover_limbs") *v = t.mul_crossover_limbs;
    else if (k == "mul.small_crossover_limbs") *v = t.mul_small_crossover_limbs;
    else if (k == "mul.crossover_limbs_p64") *v = t.mul_crossover_p64;
    else if (k == "mul.crossover_limbs_p128") *v = t.mul_crossover_p128;
    else if (k == "mul.crossover_limbs_p256") *v = t.mul_crossover_p256;
    else if (k == "mul.crossover_limbs_p512") *v = t.mul_crossover_p512;
    else if (k == "mul.crossover_limbs_p1024") *v = t.mul_crossover_p1024;
    else if (k == "mul.mad_xchunk") *v = t.mad_xchunk;
    else if (k == "mul.mfma_chunk") *v = t.mfma_chunk;
    else if (k == "mul.mfma_rows") *v = t.mfma_rows;
    else if (k == "mul.karatsuba_limbs") *v = t.karatsuba_limbs;
    else if (k == "ragged.pair_small") *v = t.ragged_pair;
    else if (k == "lookback.spin_limit") *v = t.spin_limit;
    else if (k == "debug.flags") *v = t.debug_flags;
    else if (k == "workspace.auto_grow") *v = t.auto_grow;
    else return BN_EINVAL;
    return BN_OK;
}

bn_status bn_load_tuning(bn_ctx *ctx, const char *path) {
    if (!ctx || !path) return BN_EINVAL;
    // all or nothing: a file with a bad entry leaves the settings as they were
    const Tuning saved = ctx->tune;
    const bn_status st = load_tuning(ctx, path);
    if (st != BN_OK) ctx->tune = saved;
    return st;
}

static bn_status load_tuning(bn_ctx *ctx, const char *path) {
    FILE *f = fopen(path, "rb");
    if (!f) return BN_EINVAL;
    std::string s;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, got);
    fclose(f);
    // flat object of "key": integer pairs
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) return BN_EINVAL;
        const std::string key = s.substr(i + 1, j - i - 1);
        size_t c = s.find(':', j);
        if (c == std::string::npos) return BN_EINVAL;
        ++c;
        while (c < s.size() && (s[c] == ' ' || s[c] == '\t' || s[c] == '\n' || s[c] == '\r')) ++c;
        char *end = nullptr;
        const long long v = strtoll(s.c_str() + c, &end, 10);
        if (end == s.c_str() + c) {
            // non-integer value (e.g. a string annotation): skip it, quoted text whole
            if (c < s.size() && s[c] == '"') {
                const size_t q = s.find('"', c + 1);
                if (q == std::string::npos) return BN_EINVAL;
                c = q + 1;
            }
            i = s.find_first_of(",}", c);
            if (i == std::string::npos) break;
            continue;
        }
        bn_status st = bn_set_param(ctx, key.c_str(), v);
        if (st != BN_OK && key.find('.') != std::string::npos) return st;
        i = (size_t)(end - s.c_str());
    }
    return BN_OK;
}

}  // extern "C"

static bn_status capture(bn_stream stream, bn_graph **out, const std::function<bn_status()> &body) {
    hipStream_t s = S(stream);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return BN_EHIP;
    bn_status st = body();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != BN_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess || !graph) return BN_EHIP;
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return BN_EHIP;
    }
    bn_graph *g = new bn_graph();
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return BN_OK;
}
