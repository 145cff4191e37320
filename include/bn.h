/*
 * bn.h -- C ABI of the MI355X (gfx950) large-number arithmetic library.
 *
 * Operations follow the problem statements of "Leveraging SIMD for Accelerating
 * Large-number Arithmetic" (DigitsOnTurbo, DoT):
 *   - add/sub: DoT-Add-Words(A, B, m) -> (S, c_out) of Algorithm 1 / Theorem 1
 *     (Sec. 3.1), subtraction being its borrow mirror (Sec. 3.1, "Subtraction");
 *   - mul: DoT-Mul-Words(A, B, m, k) -> P = A x B of Algorithm 2 / Theorem 2
 *     (Sec. 3.2), with unequal operand lengths allowed (the proof of Theorem 2
 *     pads the shorter operand with zero limbs, Appendix B).
 *
 * Number format (Sec. 2.1, Theorem 1): little-endian arrays of 64-bit limbs,
 * limb 0 least significant, radix X = 2^64.
 *
 * Memory: every r/a/b/carry pointer is a DEVICE pointer owned by the caller.
 * Pointers must be 8-byte aligned; 16-byte alignment of r, a and b selects the
 * vector-load fast path.  The library owns a per-context device workspace
 * (look-back status words, column accumulators, Karatsuba and staging arrays).
 * Compute calls never allocate and never synchronise the host: size the workspace
 * beforehand with bn_reserve_for() (host-synchronous; ragged plans and graph captures
 * reserve their own), and a call whose workspace is short returns BN_ENOSPACE with
 * nothing enqueued.  Setting "workspace.auto_grow" to 1 lets such a call grow the
 * workspace itself instead (an allocation and a device synchronisation; refused with
 * BN_ECAPTURE while the stream is being captured).
 *
 * Streams: `bn_stream` is a hipStream_t (NULL = the legacy default stream).
 * Every compute call is asynchronous and stream-ordered: it validates its
 * arguments on the host, enqueues kernels and returns without synchronising.
 * Calls on one context must not overlap in time (they share the workspace):
 * issue them on one stream, or use one context per concurrently used stream.
 * A context is not thread-safe on the host either (its workspace, epoch counter
 * and settings change without a lock): one thread at a time per context; separate
 * contexts may be driven from separate threads.
 *
 * Errors: every entry point returns a bn_status.  Argument errors are detected
 * synchronously and nothing is enqueued.  HIP launch errors map to BN_EHIP.
 * Device-side events worth knowing about (see bn_check) are latched in the
 * context.  No C++ exception crosses the ABI.
 */
#ifndef BN_H_
#define BN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int bn_status;
#define BN_OK 0
#define BN_EINVAL (-1)        /* null pointer for a non-empty operand, misalignment, bad enum */
#define BN_EALIAS (-2)        /* output overlaps an input in a way the operation forbids */
#define BN_ERANGE (-3)        /* a size beyond the supported limits */
#define BN_ENOMEM (-4)        /* device workspace allocation failed */
#define BN_EHIP (-5)          /* a HIP runtime call or kernel launch failed */
#define BN_EUNSUPPORTED (-6)  /* no gfx950 device, or a feature not built */
#define BN_ECAPTURE (-7)      /* workspace would have to grow while the stream is being captured */
#define BN_ENOSPACE (-8)      /* the context's workspace is too small for the call (bn_reserve_for) */

typedef struct bn_ctx bn_ctx;
typedef void *bn_stream; /* hipStream_t */

/* Size limits (limbs).  A single operand may hold up to 2^34 limbs (128 GiB). */
#define BN_MAX_LIMBS (1ull << 34)

/* ---------------------------------------------------------------- context ---- */

/* Create a context on HIP device `device` (makes it current for the call).
 * Allocates the small control block; the workspace starts empty (bn_reserve_for).
 * tuning_json: a file written by bn_autotune to load into the context (as
 * bn_load_tuning does), or NULL for the built-in defaults.
 * Errors: BN_EINVAL (ctx NULL, or an unreadable / rejected tuning file), BN_EUNSUPPORTED
 * (device is not gfx950), BN_EHIP, BN_ENOMEM. */
bn_status bn_create(bn_ctx **ctx, int device, const char *tuning_json);

/* Synchronises the device and frees everything the context owns.  NULL is a no-op. */
bn_status bn_destroy(bn_ctx *ctx);

/* Human-readable text for a status code (static storage). */
const char *bn_strerror(bn_status s);

/* Grow the multiplication column workspace to at least `bytes` now (host-synchronous
 * allocation).  bn_reserve_for sizes every buffer of a call. */
bn_status bn_reserve(bn_ctx *ctx, size_t bytes);

/* The calls that take workspace, for bn_reserve_for / bn_workspace_size: */
#define BN_OP_ADDSUB 0          /* bn_add, bn_sub (npairs = 1), bn_add_n_batch, bn_sub_n_batch: na = n */
#define BN_OP_ADDSUB_NC 1       /* bn_add_nc_n_batch, bn_sub_nc_n_batch: na = n */
#define BN_OP_ADDSUB_UNEQUAL 2  /* bn_add_unequal, bn_sub_unequal (npairs = 1), bn_add_unequal_n_batch,
                                   bn_sub_unequal_n_batch: na, nb */
#define BN_OP_SUB_ABS 3         /* bn_sub_abs_n_batch: na = n */
#define BN_OP_MUL 4             /* bn_mul (npairs = 1), bn_mul_n_batch: na, nb, form */
#define BN_OP_MUL_KARATSUBA 5   /* bn_mul_karatsuba_batch: na, nb, form, levels (bn_mul_karatsuba_n_batch:
                                   na = nb = n) */
#define BN_OP_IN_PLACE 0x100    /* or'ed into a multiplication op: the output overlaps an operand
                                   (the staging buffer) */

/* Grow every workspace buffer now (host-synchronous: allocation and a device
 * synchronisation) so that a call of this shape runs without allocating -- eagerly or
 * inside a stream capture.  Needs are not monotone in the sizes (a single large product
 * splits its contraction and takes more than one of a batch): reserve each shape you
 * will call, or the largest per bn_workspace_size.
 * form and levels are used by the multiplication ops only (pass BN_MUL_AUTO, 0
 * otherwise).  Buffers only grow; once the context has captured a graph, replaced
 * buffers are kept until bn_destroy.  Errors: BN_EINVAL (NULL ctx, unknown op, form or
 * levels), BN_ERANGE, BN_ENOMEM, BN_EHIP. */
bn_status bn_reserve_for(bn_ctx *ctx, int op, size_t na, size_t nb, size_t npairs, int form, int levels);

/* Workspace bytes (all buffers together) a call of this shape needs; 0 for a NULL
 * ctx, an unknown op or sizes out of range.  Pure host computation. */
size_t bn_workspace_size(bn_ctx *ctx, int op, size_t na, size_t nb, size_t npairs, int form, int levels);

/* Synchronise `stream`, then read and clear the context's device-side latch.
 * *flags (may be NULL) receives it: bit 0 = since the last check, some add/sub tile
 * waited longer than "lookback.spin_limit" polls for a predecessor and computed
 * that predecessor's carry from the operands itself (results are exact either way).
 * Returns BN_OK, or BN_EHIP if the stream reported an error. */
bn_status bn_check(bn_ctx *ctx, bn_stream stream, uint32_t *flags);

/* Look-back distance histogram of the chained add/sub scans run since the last
 * call, recorded only while "debug.flags" bit 1 is set (one atomic per tile).
 * hist[k] (host array of nbins entries, nbins may be 0) receives the number of
 * workgroup tiles whose carry-in was decided by a predecessor 2^k <= d < 2^(k+1)
 * tiles back (d = 1: the nearest one had already published; reaching past the
 * first tile of the operand counts as that tile's distance + 1).  Bins past
 * BN_LOOKBACK_BINS read 0.  Deferred launches (see bn_add) record nothing.  Waits
 * for `stream`, then clears the histogram.
 * Returns BN_EINVAL for a NULL ctx, or hist NULL with nbins > 0; BN_EHIP on a
 * stream error. */
#define BN_LOOKBACK_BINS 32
bn_status bn_lookback_stats(bn_ctx *ctx, bn_stream stream, uint64_t *hist, size_t nbins);

/* ------------------------------------------------------- add / subtract ---- */

/* r = (a + b) mod 2^(64n); *carry_out = carry-out c_n in {0,1} (Theorem 1).
 * r may equal a or b exactly (in place); any other overlap is BN_EALIAS.
 * carry_out (device, one uint64) may be NULL.  n = 0 is valid (carry 0).
 * One pass over the operands: limb sums, generate/propagate flags, a wave64
 * ballot prefix scan, an LDS scan across waves and a decoupled look-back across
 * workgroups (Sec. 3.1 phases 1-4 restated as a parallel prefix computation).
 * Large launches (at least "addsub.defer_tiles" tiles) add two small kernels and no
 * tile waits for another tile's look-back: a tile whose every limb propagates stores
 * nothing and exits (its result is all ones or all zeros, fixed by its carry-in alone),
 * a tile whose 64-tile look-back window holds only such tiles keeps its sums for
 * carry-in 0, and after the launch a one-workgroup scan of the status words and a fill
 * pass write those constants and repairs -- at the same 24 bytes of traffic per limb.
 * Workspace: a launch whose workgroup tiles do not each start a pair (one long pair,
 * or pairs longer than a tile or not dividing it) keeps one look-back status word and
 * one fill code byte per tile: bn_reserve_for(BN_OP_ADDSUB); BN_ENOSPACE if short.  In place, a tile waiting
 * for an unpublished predecessor only waits (it never recomputes that tile from the
 * operands, which may already hold sums). */
bn_status bn_add(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                 uint64_t *carry_out, bn_stream stream);

/* r = (a - b) mod 2^(64n); *borrow_out = [a < b].  Same rules as bn_add. */
bn_status bn_sub(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                 uint64_t *borrow_out, bn_stream stream);

/* Uniform batch: pair p is limbs [p*n, (p+1)*n) of r, a and b; carry_out[p] (device,
 * npairs uint64, may be NULL) receives its carry/borrow.  Pairs are independent. */
bn_status bn_add_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b,
                         size_t n, size_t npairs, uint64_t *carry_out, bn_stream stream);
bn_status bn_sub_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b,
                         size_t n, size_t npairs, uint64_t *borrow_out, bn_stream stream);

/* For callers that cannot allocate device memory at call time (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc) and will not reserve a
 * workspace: bn_add_n_batch (sub = 0) or bn_sub_n_batch (sub = 1) with the look-back
 * status of chained launches kept in a fixed device array of the library, one per GPU,
 * instead of the context's workspace.  Arguments, results, in-place rules and errors
 * are those of bn_add_n_batch / bn_sub_n_batch (npairs = 1 is bn_add / bn_sub); the
 * context supplies the device and the tuned tile shapes only, and its workspace is
 * neither used nor grown.  The call allocates nothing and never synchronises.
 * Limit: the array holds BN_SCRATCH_MAX_TILES status words and as many fill code bytes
 * (about 1.1 MiB per GPU, held until the process ends), one each per workgroup tile of a
 * chained launch: with the default
 * shapes, one pair of up to 2^28 limbs (2 GiB per operand) -- batches whose pair length
 * divides 128 need no status words and have no such limit.  A launch that could need
 * more (at either operand alignment) returns BN_ERANGE with nothing enqueued.
 * The array is shared by every call on that GPU, from any context, and keeps the last
 * call's contents (each chained launch tags its words with an epoch of its own, so no
 * clearing is needed): calls that overlap in time on one GPU race and must be ordered
 * (one stream, or events).  BN_EINVAL if sub is not 0 or 1; BN_EUNSUPPORTED if the
 * context's device has no such array (device index 64 or above). */
#define BN_SCRATCH_MAX_TILES (1u << 17)
bn_status bn_addsub_n_batch_noalloc(bn_ctx *ctx, int sub, uint64_t *r, const uint64_t *a, const uint64_t *b,
                                    size_t n, size_t npairs, uint64_t *carry_out, bn_stream stream);

/* With a carry (borrow) into limb 0 of every pair: the c_in of Algorithm 1's W-limb
 * step (Sec. 3.1), which chains additions of more limbs than one call holds.
 * r_p = (a_p + b_p + cin_p) mod 2^(64n), carry_out[p] = the carry out; sub:
 * r_p = (a_p - b_p - bin_p) mod 2^(64n), borrow_out[p] = [a_p < b_p + bin_p].
 * carry_in (device, npairs uint64, bit 0 used) must be given (BN_EINVAL if NULL with
 * npairs > 0) and must not overlap carry_out or r (BN_EALIAS); r may equal a or b
 * exactly.  n = 0 copies carry_in to carry_out. */
bn_status bn_add_nc_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs,
                            const uint64_t *carry_in, uint64_t *carry_out, bn_stream stream);
bn_status bn_sub_nc_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs,
                            const uint64_t *borrow_in, uint64_t *borrow_out, bn_stream stream);

/* Unequal lengths (na >= nb, else BN_EINVAL): r[0, na) = a + b with b zero-extended
 * (the shorter operand padded with zero limbs, as in the proof of Theorem 2), carry
 * out in *carry_out; sub: r = (a - b) mod 2^(64 na) and the borrow.  One scan whose b
 * reads as zero past nb limbs (bn_add_unequal_n_batch with one pair).  r may equal a
 * exactly (or b when na == nb). */
bn_status bn_add_unequal(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b, size_t nb,
                         uint64_t *carry_out, bn_stream stream);
bn_status bn_sub_unequal(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b, size_t nb,
                         uint64_t *borrow_out, bn_stream stream);

/* Unequal lengths, batched: pair p is a + p*na, b + p*nb (na >= nb, else BN_EINVAL) and
 * r + p*na; r_p = (a_p + b_p) mod 2^(64 na) with b_p zero-extended to na limbs (the
 * shorter operand padded with zero limbs, as in the proof of Theorem 2) and
 * carry_out[p] its carry (device, npairs uint64, may be NULL); sub: r_p = (a_p - b_p)
 * mod 2^(64 na) and the borrow.  One pass of the scan: b's limbs are read by pair
 * position and count as zero past nb.  r may equal a exactly (or b when na == nb).
 * Workspace: bn_reserve_for(BN_OP_ADDSUB_UNEQUAL, na, nb, npairs) when pairs cross
 * workgroup tiles (na not dividing 128); BN_ENOSPACE if short. */
bn_status bn_add_unequal_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b,
                                 size_t nb, size_t npairs, uint64_t *carry_out, bn_stream stream);
bn_status bn_sub_unequal_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b,
                                 size_t nb, size_t npairs, uint64_t *borrow_out, bn_stream stream);

/* r_p = |a_p - b_p| and sign[p] = [a_p < b_p] (device, may be NULL): the signed
 * difference the Karatsuba step needs (App. A, Algorithm 4).  b - a goes to the
 * context's workspace (bn_reserve_for(BN_OP_SUB_ABS)), then a - b to r, then a select;
 * r may equal a or b exactly. */
bn_status bn_sub_abs_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                             size_t npairs, uint64_t *sign, bn_stream stream);

/* ------------------------------------------------------------ multiply ---- */

#define BN_MUL_AUTO 0 /* pick per size from the tuning table (mad below the crossover) */
#define BN_MUL_MAD 1  /* 32x32->64-bit v_mad_u64_u32 column products */
#define BN_MUL_MFMA 2 /* balanced signed 8-bit digit convolution on int8 MFMA, int32 accumulation */

/* r[0 .. na+nb) = a * b (Theorem 2), exactly na+nb limbs, leading zeros kept.
 * Column products (all independent), then one deferred carry-normalise pass
 * (Algorithm 2, phases 1-5).  na = 0 or nb = 0 gives r = 0 (na+nb limbs).
 * Workspace: bn_reserve_for(BN_OP_MUL) for products above one wave's size (na + nb >
 * 512 limbs on the MFMA form, > 1024 on the mad form); BN_ENOSPACE if short.
 * In place: r may overlap a or b, in whole or in part (e.g. r == a with room for
 * na+nb limbs).  The product then goes to a staging buffer the context owns (na+nb
 * limbs per pair, reserved with BN_OP_MUL | BN_OP_IN_PLACE) and one device-to-device
 * copy on `stream` moves it into r after every read of a and b. */
bn_status bn_mul(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b, size_t nb,
                 int form, bn_stream stream);

/* Uniform batch: a of pair p at a + p*na, b at b + p*nb, product at r + p*(na+nb). */
bn_status bn_mul_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t na,
                         size_t nb, size_t npairs, int form, bn_stream stream);

/* Uniform batch of products through `levels` Karatsuba levels above the schoolbook
 * kernels of `form` (the recursion the paper's libraries put above the base case,
 * App. A, Algorithm 4): with k = ceil(m/2), A = A_H X^k + A_L, B likewise,
 * P1 = A_H B_H, P0 = A_L B_L, P2 = sign(A_H-A_L) sign(B_H-B_L) |A_H-A_L| |B_H-B_L|,
 * A B = P1 X^(2k) + (P1 + P0 - P2) X^k + P0.  Each level turns N products of m limbs
 * into 3N of k limbs (for odd m the high halves, k - 1 limbs, are zero-extended to k);
 * the bottom level is one bn_mul_n_batch-style launch, the splits and combines are
 * batched add/sub passes.  Pair p: a + p*na, b + p*nb, product at r + p*(na+nb)
 * (exactly na + nb limbs).  Operands of unequal length are zero-extended to
 * m = max(na, nb) at the top level (the padding of Theorem 2's proof), so the work is
 * that of an m x m product: for lengths far apart bn_mul_n_batch does less.  Any sizes;
 * levels = 0 is bn_mul_n_batch; levels > BN_KARATSUBA_MAX_LEVELS is BN_EINVAL.
 * levels = BN_KARATSUBA_AUTO picks bn_karatsuba_auto_levels(max(na, nb),
 * "mul.karatsuba_limbs"), the libraries' size threshold for the recursion (App. A)
 * applied per level, or 0 when one length is below half the other.  r may overlap a or
 * b (in place, as for bn_mul).  Workspace: about 100 m npairs (3/2)^levels bytes,
 * reserved with bn_reserve_for(BN_OP_MUL_KARATSUBA, na, nb, ...); BN_ENOSPACE if
 * short. */
#define BN_KARATSUBA_MAX_LEVELS 8
#define BN_KARATSUBA_AUTO (-1)
bn_status bn_mul_karatsuba_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b,
                                 size_t nb, size_t npairs, int levels, int form, bn_stream stream);
/* Square products: bn_mul_karatsuba_batch with na = nb = n (product at r + 2*p*n). */
bn_status bn_mul_karatsuba_n_batch(bn_ctx *ctx, uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                                   size_t npairs, int levels, int form, bn_stream stream);

/* Karatsuba levels that BN_KARATSUBA_AUTO uses for n-limb operands: one more level
 * while the operand has at least 2 limbs, the halves (ceil(m/2) limbs) would keep at
 * least min_half_limbs limbs and the count stays within BN_KARATSUBA_MAX_LEVELS
 * (0 when n < 2 min_half_limbs - 1).  Pure host function (no device, no context). */
int bn_karatsuba_auto_levels(size_t n, size_t min_half_limbs);

/* ------------------------------------------------- ragged batches + plans ---- */

/* One pair of a ragged batch: offsets in limbs into pooled device arrays. */
typedef struct bn_pair {
    uint64_t a_off, b_off, r_off;
    uint32_t na, nb;
} bn_pair;

typedef struct bn_plan bn_plan;

/* Build a plan for a ragged multiply batch from a HOST copy of the descriptors:
 * validates sizes (1 <= na, nb <= 2^20), sorts the pairs by work (na*nb,
 * largest first), picks mad or MFMA per pair (form, or the tuned crossover for
 * BN_MUL_AUTO; automatic products of 129-256 limbs take MFMA), and uploads the work
 * list to device memory it owns.  Pairs that take the batched path (na + nb > 256) get
 * the context's workspace reserved here.
 * Offsets plus lengths must stay below 2^60 limbs (else BN_ERANGE).
 * Synchronous (allocates).  Product ranges must not overlap each other or the inputs. */
bn_status bn_plan_mul_ragged(bn_ctx *ctx, const bn_pair *host_pairs, size_t npairs, int form,
                             bn_plan **plan);
bn_status bn_plan_destroy(bn_plan *plan);

/* Run a planned ragged multiply: one persistent launch (both forms in one kernel when
 * the plan has both); wave k of W resident waves takes pairs k, k+W, ... of the
 * work-sorted list, after the couples of small mad items that run two to a wave
 * ("ragged.pair_small").  Pairs with
 * na + nb > 256 run through the batched path, one call each.  No allocation, no host
 * sync (the plan reserved the workspace; BN_ENOSPACE if it was given up since).
 * BN_EINVAL for a plan of another kind or one built on a context of another device. */
bn_status bn_mul_ragged(bn_ctx *ctx, const bn_plan *plan, uint64_t *r_pool, const uint64_t *a_pool,
                        const uint64_t *b_pool, bn_stream stream);

/* Ragged add: plan built with na == nb required (nb ignored); carry_out[p] in plan order
 * of the host descriptor array (NOT the sorted order).  May be NULL. */
bn_status bn_plan_add_ragged(bn_ctx *ctx, const bn_pair *host_pairs, size_t npairs, bn_plan **plan);
bn_status bn_add_ragged(bn_ctx *ctx, const bn_plan *plan, uint64_t *r_pool, const uint64_t *a_pool,
                        const uint64_t *b_pool, uint64_t *carry_out, bn_stream stream);

/* ------------------------------------------------------------ HIP graphs ---- */

typedef struct bn_graph bn_graph;

/* A graph addresses its context's workspace and, for ragged calls, the plan's work
 * list: destroy graphs before their context and plan.  Once a context has captured a
 * graph, a buffer that later calls outgrow is kept (not freed) until bn_destroy, so
 * replays stay valid after eager calls of any size; replays and eager calls on one
 * context share the workspace and must not overlap in time (one stream, or ordered). */

/* Capture one bn_mul_ragged call into an instantiated HIP graph (pointers are baked in).
 * The workspace must already be large enough (it is reserved here, before capture). */
bn_status bn_graph_capture_mul_ragged(bn_ctx *ctx, const bn_plan *plan, uint64_t *r_pool,
                                      const uint64_t *a_pool, const uint64_t *b_pool,
                                      bn_stream stream, bn_graph **graph);
/* Same for a uniform add/sub/mul batch (op: 0 add, 1 sub, 2 mul; na = nb = n for
 * add/sub).  Arguments and errors as for the eager call; for a multiplication whose
 * output overlaps an operand the staging buffer is reserved here too, and the graph
 * holds the device-to-device copy as a memcpy node.  The replays share the context's
 * workspace: replays and eager calls on one context must not overlap in time. */
bn_status bn_graph_capture_batch(bn_ctx *ctx, int op, uint64_t *r, const uint64_t *a, const uint64_t *b,
                                 size_t na, size_t nb, size_t npairs, uint64_t *carry_out, int form,
                                 bn_stream stream, bn_graph **graph);
bn_status bn_graph_launch(bn_graph *graph, bn_stream stream);
bn_status bn_graph_destroy(bn_graph *graph);

/* ------------------------------------------------------------ tuning ---- */

/* Named integer parameters of the context (see bn_param_names()):
 *   "addsub.batch_waves", "addsub.batch_rows"   add/sub tile shape when the tile length
 *                                      is a multiple of the pair length (independent tiles)
 *   "addsub.chain_waves", "addsub.chain_rows"   tile shape otherwise (look-back between tiles)
 *                                      waves in {1,2,4,8}, rows of 128 limbs in {1,2,4,8,16},
 *                                      except 8 waves x 16 rows
 *   "addsub.defer_tiles"               chained launches of at least this many tiles (default
 *                                      8192, 0 = never) defer the stores of tiles that
 *                                      propagate through every limb to a fill pass (bn_add)
 *   "mul.crossover_limbs"              BN_MUL_AUTO uses MFMA when min(na,nb) >= this
 *                                      (na + nb > 1024: the column-workspace kernels; default
 *                                      1, MFMA for every such product)
 *   "mul.small_crossover_limbs"        the same for na + nb <= 1024 (one wave per product) in
 *                                      each size class below whose own parameter is -1 (by
 *                                      default the classes of at most 128 limbs; default 28)
 *   "mul.crossover_limbs_p64",          the same for products of at most 64 limbs and of 65-128
 *   "mul.crossover_limbs_p128"         limbs (the mad form's lanes hold 1 or 2 limbs there, the
 *                                      MFMA form runs one column block); -1 (default): use
 *                                      "mul.small_crossover_limbs"
 *   "mul.crossover_limbs_p256",         the same for products of 129-256, 257-512 and 513-1024
 *   "mul.crossover_limbs_p512",         limbs (defaults 2, 2 and 40: the mad form's per-step work
 *   "mul.crossover_limbs_p1024"        grows with the product, the one-wave MFMA form's far
 *                                      less; above 512 limbs MFMA runs on the workspace path);
 *                                      -1: use "mul.small_crossover_limbs"
 *   "mul.mad_xchunk"                   32-bit digits of a per large mad work item
 *   "mul.mfma_chunk"                   Toeplitz steps staged in LDS per round by the large
 *                                      MFMA kernel: even, 16..256 (up to 234, three workgroups
 *                                      share a CU), or 0 (default): by size, 256 for unsplit
 *                                      launches whose shorter operand has >= 10240 limbs,
 *                                      224 otherwise
 *   "mul.karatsuba_limbs"              BN_KARATSUBA_AUTO splits while the halves keep at
 *                                      least this many limbs (default 2048, >= 1)
 *   "mul.mfma_rows"                    Toeplitz rows per column block of the large MFMA
 *                                      kernel, in groups of 64: 1 or 2 (default 2: the same
 *                                      LDS reads feed twice the MFMAs)
 *   "ragged.pair_small"                ragged multiplication plans built afterwards: mad
 *                                      items of at most 32 product limbs whose shorter
 *                                      operands have the same length run two to a wave, one
 *                                      per half (1, default), or one each (0)
 *   "lookback.spin_limit"              look-back polls before a tile computes an
 *                                      unpublished predecessor's carry itself
 *   "debug.flags"                      bit 0: tile 0 never publishes its status
 *                                      (test hook for the self-computed look-back; such
 *                                      launches do not defer);
 *                                      bit 1: record look-back distances
 *                                      (read with bn_lookback_stats)
 * Returns BN_EINVAL for an unknown key or an out-of-range value. */
bn_status bn_set_param(bn_ctx *ctx, const char *key, int64_t value);
bn_status bn_get_param(bn_ctx *ctx, const char *key, int64_t *value);
const char *bn_param_names(void);

/* Time the candidate add/sub tile shapes, the mad/MFMA crossovers (one for products of
 * at most 1024 limbs, one for larger ones) and the large MFMA kernel's staging window
 * on this device (scratch operands allocated internally), store the winners in the
 * context and, if out_json != NULL, write them as a JSON object.  Synchronous; takes
 * seconds. */
bn_status bn_autotune(bn_ctx *ctx, const char *out_json);

/* Measured device rates, the ceilings the rooflines are also stated against:
 * *mac96_per_s = 32x32-bit multiply-accumulates into a 96-bit sum per second
 * (v_mad_u64_u32 + v_addc_co_u32, the plain form's column step, Alg. 2 phase 2 on
 * random 32-bit digits); *mfma_i8_ops_per_s = int8 MFMA operations per second (2 per
 * multiply-add, v_mfma_i32_32x32x32_i8 with independent accumulators, on random
 * operand bytes: the rate depends on the data, and mostly-zero operands run about 25%
 * faster); and
 * *copy_bytes_per_s = bytes read plus written per second by a 512 MiB device copy
 * with 16-byte non-temporal loads and stores per lane (how the add/sub scan moves
 * its operands), the fastest of 2, 4 or 8 loads in flight per lane.  Each runs over every CU of the context's device.  Synchronises the
 * device; allocates and frees about 1 GiB.  Returns BN_EINVAL for NULL arguments,
 * BN_ENOMEM, or BN_EHIP. */
bn_status bn_probe_rates(bn_ctx *ctx, double *mac96_per_s, double *mfma_i8_ops_per_s, double *copy_bytes_per_s);

/* Load parameters written by bn_autotune (flat JSON object of "key": integer; keys
 * without a dot and non-integer values are skipped).  All or nothing: BN_EINVAL for an
 * unreadable file, a malformed entry or a rejected value, and then no setting changes. */
bn_status bn_load_tuning(bn_ctx *ctx, const char *json_path);

/* Library version string. */
const char *bn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BN_H_ */
