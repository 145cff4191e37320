// Internal declarations shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bn.h"

#include <atomic>
#include <vector>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

#define BN_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return BN_EHIP;          \
    } while (0)

// Device-side control block of the decoupled look-back (one per context).
//   epoch : tags status words; bumped by a one-thread kernel after every chained
//           scan, so status words of earlier launches never match
//   err   : sticky latch read and cleared by bn_check (bit 0: a look-back computed
//           a predecessor tile's aggregate itself instead of waiting for it)
constexpr int LOOKBACK_BINS = 32;
struct ScanCtl {
    u64 epoch;                // look-back epoch of launches recorded into graphs
    u64 err;                  // latched device events (bit 0: a look-back computed a predecessor itself)
    u64 pad[6];
    u64 hist[LOOKBACK_BINS];  // look-back distances, recorded when debug flag bit 1 is set
};

// Tile-shape selector for the flat scan kernel.
struct ScanShape {
    int waves;  // waves per workgroup (1, 2, 4 or 8)
    int rows;   // 128-limb rows per wave (1, 2, 4, 8 or 16)
};

struct Tuning {
    // add/sub tile shapes: "batch" is used when the tile length is a multiple of the
    // pair length (tiles never depend on each other), "chain" otherwise (look-back)
    int batch_waves = 1;
    int batch_rows = 1;
    int chain_waves = 4;
    int chain_rows = 8;
    i64 mul_crossover_limbs = 1;       // BN_MUL_AUTO, na + nb > 1024: MFMA when min(na, nb) >= this
    i64 mul_small_crossover_limbs = 28;  // BN_MUL_AUTO, na + nb <= 1024 (one-wave kernels): the same
    i64 mul_crossover_p64 = -1;        // the same for na + nb <= 64 (-1: mul_small_crossover_limbs)
    i64 mul_crossover_p128 = -1;       // the same for 64 < na + nb <= 128 (-1: mul_small_crossover_limbs)
    i64 mul_crossover_p256 = 2;        // the same for 128 < na + nb <= 256
    i64 mul_crossover_p512 = 2;        // the same for 256 < na + nb <= 512
    i64 mul_crossover_p1024 = 40;      // the same for 512 < na + nb <= 1024 (MFMA on the workspace path)
    int mad_cols = 8;                  // 32-bit columns per lane in the large mad kernel
    int mad_xchunk = 4096;             // x-range (32-bit digits) per mad work item
    int mfma_chunk = 0;                // Toeplitz steps staged in LDS per round (even, 16..256; three
                                       // workgroups of the large MFMA kernel fit a CU up to 234);
                                       // 0: by size (mfma_window in k_mul.hip)
    int mfma_rows = 2;                 // Toeplitz row groups of 64 per column block (1 or 2)
    int ragged_pair = 1;               // ragged multiplication plans: mad items of at most 32 product
                                       // limbs whose shorter operands have the same length run two
                                       // to a wave (1) or one each (0)
    i64 karatsuba_limbs = 2048;        // BN_KARATSUBA_AUTO: smallest half that is split again
    int auto_grow = 0;                 // 1: a compute call whose workspace is short grows it
                                       // (allocation + device synchronisation, never during a
                                       // capture); 0: it returns BN_ENOSPACE
    u32 spin_limit = 2048;             // look-back polls before computing a predecessor itself
    u64 defer_tiles = 8192;            // chained launches of at least this many tiles defer the
                                       // stores of all-propagate tiles to a fill pass (0: never)
    u32 debug_flags = 0;               // bit 0: tile 0 never publishes (exercises the self-help path)
                                       // bit 1: record look-back distances in ScanCtl::hist
};

// Workspace buffer of a context: sized by the reserve calls (or, with auto_grow, by the
// compute call that needs more; never while the stream is being captured).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Workspace a call needs, per buffer (bytes).
struct WsNeed {
    size_t status = 0;  // look-back status words of chained scans
    size_t work = 0;    // multiplication column sums / folded limbs / converted operands
    size_t kwork = 0;   // Karatsuba levels; |a - b| scratch
    size_t mstage = 0;  // products computed in place
};

struct bn_ctx {
    int device = 0;
    int num_cu = 256;           // compute units (sizes persistent grids)
    ScanCtl *ctl = nullptr;     // device control block
    DevBuf status;              // look-back status words
    DevBuf work;                // mul column accumulators / folded limbs
    DevBuf kwork;               // Karatsuba operand, product and combine arrays
    DevBuf mstage;              // products computed in place: staged here, then copied
    u64 host_epoch = 1ull << 61;  // epochs of chained scans launched outside a capture
    Tuning tune;
    bool captured = false;        // a graph has baked in buffer addresses of this context
    bool grow_scope = false;      // growth allowed inside the call (the autotuner's own calls)
    std::vector<void *> retired;  // buffers replaced after a capture, freed by bn_destroy
};

// One pair of a ragged batch as the device sees it.
struct RItem {
    u64 a_off, b_off, r_off;
    u32 na, nb;
    u32 form;   // BN_MUL_MAD / BN_MUL_MFMA (mul) or unused (add)
    u32 index;  // position in the caller's descriptor array
};

struct bn_plan {
    int op = 0;                    // 0 = mul ragged, 1 = add ragged
    int device = 0;
    size_t npairs = 0;
    u32 nsmall = 0;                // items run by the persistent kernels
    u32 nsmall_mad = 0;            // of which mad form (they come first in d_items)
    RItem *d_items = nullptr;      // device copy of the small items, each form sorted by work
    u32 npaired = 0;               // mad items that run two to a wave (d_pairs holds them as
    RItem *d_pairs = nullptr;      // consecutive couples; they are not among the nsmall)
    std::vector<RItem> large;      // mul items too big for one wave: one batched launch each
    u32 nmad = 0, nmfma = 0;       // items per form
    u64 work = 0;                  // sum of na * nb (mul) or n (add)
    WsNeed ws;                     // workspace of the large items (reserved when the plan is built)
};

struct bn_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// ---- internal helpers (bn_api.hip) ----
// `buf` holds at least `bytes`: BN_OK; else, when growth is allowed (auto_grow or the
// autotuner) and the stream is not being captured, grow it; else BN_ENOSPACE.
bn_status bn_ensure(bn_ctx *ctx, DevBuf &buf, size_t bytes, hipStream_t s);
// Grow `buf` to at least `bytes` now (host-synchronous; the reserve calls).
bn_status bn_grow(bn_ctx *ctx, DevBuf &buf, size_t bytes);
bn_status ws_reserve(bn_ctx *ctx, const WsNeed &need);
bn_status bn_launch_status();

// ---- add/sub (k_addsub.hip) ----
// Flat segmented add/sub over N = n * npairs limbs; a segment (pair) starts every n limbs.
bn_status launch_flat_scan(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs,
                           u64 *carry, hipStream_t s);
// The same with a per-segment carry-in (cin, device, bit 0; NULL for none) and/or every
// limb of b taken as bval (bconst; b unused): r = a +- b +- cin.  bconst without cin is
// built for addition only.
bn_status launch_flat_scan_ext(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs,
                               const u64 *cin, bool bconst, u64 bval, u64 *carry, hipStream_t s);
size_t flat_scan_status_bytes(const bn_ctx *ctx, u64 n, u64 N);
size_t scan_state_bytes(u64 tiles);  // status words + fill codes of a chained launch over `tiles` tiles
size_t flat_scan_ext_status_bytes(u64 n, u64 N);  // the same for launch_flat_scan_ext
bn_status launch_fill_u64(u64 *p, u64 count, u64 value, hipStream_t s);
// Where a chained launch keeps its look-back state: NULL for the context's control block
// and status array (grown by the reserve calls), or a fixed device array.
struct ScanMem {
    ScanCtl *ctl = nullptr;
    u64 *status = nullptr;                   // max_tiles status words, then max_tiles fill code bytes
    u64 max_tiles = 0;                       // status words available
    std::atomic<u64> *host_epoch = nullptr;  // epochs of launches outside a capture
    u32 dbg_mask = ~0u;                      // debug flags that apply
};
// The child products of a Karatsuba level of N products of out <= 4k limbs, for the
// scan that forms and adds the level's terms (launch_flat_scan_comb): per product q,
// P0, P1 and PD at 2k q (2k limbs each), the signs of its two differences in negA[q],
// negB[q].
struct ScanComb {
    const u64 *P0 = nullptr, *P1 = nullptr, *PD = nullptr;
    const u64 *negA = nullptr, *negB = nullptr;
    u64 k = 0;
};
bn_status launch_flat_scan_comb(bn_ctx *ctx, u64 *r, const ScanComb &comb, u64 out, u64 N, hipStream_t s);
// Subtraction with the operands swapped per pair: pair q computes b - a instead of
// a - b when its sign key says so (the largest of keys[q npieces .. q npieces +
// npieces - 1], bit 0), and the lane holding the pair's first limb stores that sign
// in neg[q].  Used by a Karatsuba split for |A_H - A_L|.
struct ScanSwap {
    const u64 *keys = nullptr;
    u64 npieces = 0;
    u64 *neg = nullptr;
};
// The second part of a two-part launch: npairs more pairs of the same length whose
// arrays lie elsewhere (b may be null with bconst); a carry array covers both parts,
// the first part's pairs first.  One launch when the first part ends on a tile
// boundary and no array overlaps another, else one launch per part.
struct ScanPart2 {
    u64 *r = nullptr;
    const u64 *a = nullptr, *b = nullptr;
    u64 npairs = 0;
};
// nbz >= 0: b holds nbz limbs per pair (its pair stride) and reads as zero past them.
bn_status launch_flat_scan_mem(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs,
                               const u64 *cin, bool bconst, u64 bval, u64 *carry, hipStream_t s,
                               const ScanMem *fixed, i64 nbz = -1, const ScanComb *comb = nullptr,
                               const ScanPart2 *part2 = nullptr, const ScanSwap *swap = nullptr);
// Unequal lengths, batched: pair p is a + p na, b + p nb (nb <= na), r + p na, and
// r_p = a_p +- b_p with b_p zero-extended to na limbs; one pass.
bn_status launch_flat_scan_bzx(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, u64 na, const u64 *b, u64 nb,
                               u64 npairs, u64 *carry, hipStream_t s);

// ---- the fixed per-GPU scratch array (scratch.hip) ----
// Once per device, with that device current (bn_create): take the array's device
// address and clear it.  Devices past the table are skipped (BN_OK).
bn_status scratch_setup(int device);
// The look-back state in that device's array; false if the device was never set up.
bool scratch_mem(int device, ScanMem *m);

// ---- add/sub extras (k_addsub_ext.hip) ----
bn_status launch_addsub_nc(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs,
                           const u64 *cin, u64 *carry, hipStream_t s);
bn_status launch_addsub_unequal(bn_ctx *ctx, bool sub, u64 *r, const u64 *a, u64 na, const u64 *b, u64 nb,
                                u64 npairs, u64 *carry, hipStream_t s);
WsNeed unequal_need(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs);
bn_status launch_sub_abs(bn_ctx *ctx, u64 *r, const u64 *a, const u64 *b, u64 n, u64 npairs, u64 *sign,
                         hipStream_t s);

// ---- mul (k_mul_*.hip) ----
bn_status launch_mul_batch(bn_ctx *ctx, u64 *r, const u64 *a, const u64 *b, u64 na, u64 nb, u64 npairs,
                           int form, hipStream_t s);
size_t mul_workspace_bytes(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs, int form);
size_t mul_status_bytes(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs, int form);  // chained-scan status words
int mul_pick_form(const bn_ctx *ctx, u64 na, u64 nb, int form);
bool mul_small_range(u64 P);  // products of P limbs that take mul.small_crossover_limbs

// ---- Karatsuba levels (k_karatsuba.hip) ----
// Products of na x nb limbs (pair p: a + p na, b + p nb, r + p (na + nb)) through
// `levels` Karatsuba levels on operands zero-extended to max(na, nb).
bn_status launch_mul_karatsuba(bn_ctx *ctx, u64 *r, const u64 *a, u64 na, const u64 *b, u64 nb, u64 npairs,
                               int levels, int form, hipStream_t s);
size_t karatsuba_workspace_bytes(u64 na, u64 nb, u64 npairs, int levels);
WsNeed karatsuba_need(const bn_ctx *ctx, u64 na, u64 nb, u64 npairs, int levels, int form);
// Levels that BN_KARATSUBA_AUTO takes for na x nb products (0 when the lengths differ by
// more than a factor of two: the zero-extension would cost more than it saves).
int karatsuba_auto_levels(const bn_ctx *ctx, u64 na, u64 nb);

// ---- ragged (k_ragged.hip) ----
bn_status plan_mul_ragged(bn_ctx *ctx, const bn_pair *pairs, size_t npairs, int form, bn_plan **plan);
bn_status plan_add_ragged(bn_ctx *ctx, const bn_pair *pairs, size_t npairs, bn_plan **plan);
bn_status launch_mul_ragged(bn_ctx *ctx, const bn_plan *plan, u64 *r, const u64 *a, const u64 *b, hipStream_t s);
bn_status launch_add_ragged(bn_ctx *ctx, const bn_plan *plan, u64 *r, const u64 *a, const u64 *b, u64 *carry,
                            hipStream_t s);
