/* bn_host.h -- DoT addition and subtraction on the host CPU with x86-64 SIMD.
 *
 * The paper's own method (Sec. 3.1, Algorithm 1) as it runs on a CPU: limbs are
 * processed w at a time (w = 8 with AVX-512, w = 4 with AVX2); each step adds the w
 * limb pairs at once (phase 1), turns the lane-wise carries into a bit mask and shifts
 * it up one lane with the incoming carry at bit 0 (phase 2), adds the aligned carries
 * (phase 3), and only when that add wraps a lane resolves the rare cascade with the
 * integer-add trick on the mask of all-ones limbs (phase 4).  Steps are chained by the
 * carry out of the top lane.  Subtraction mirrors it (borrow = [a < b], cascade through
 * zero limbs).  A scalar add-with-carry chain is provided as the sequential reference
 * point.  This library is a host-side comparison point beside the GPU library (libbn);
 * it shares no code with it and the GPU path never calls it.
 *
 * Layout: little-endian arrays of uint64_t limbs (limb 0 least significant).  All
 * pointers are host pointers owned by the caller.  r may equal a or b exactly (in
 * place); any other overlap gives an unspecified result.  Every call is synchronous.
 */
#ifndef BN_HOST_H
#define BN_HOST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BNH_OK 0
#define BNH_EINVAL (-1)       /* NULL pointer with n > 0, bad ISA code, threads < 1 */
#define BNH_EUNSUPPORTED (-6) /* the requested ISA is not available on this CPU */

#define BNH_ISA_SCALAR 0 /* add-with-carry chain, one limb at a time */
#define BNH_ISA_AVX2 1   /* DoT, w = 4 limbs per step */
#define BNH_ISA_AVX512 2 /* DoT, w = 8 limbs per step (AVX-512F mask registers) */

/* The widest ISA code this CPU runs (checked with cpuid at run time). */
int bnh_isa_best(void);

/* r[0, n) = a + b + carry_in (carry_in in {0, 1}), *carry_out = carry out of limb
 * n-1 (may be NULL).  n = 0 passes the carry through.  isa: one of BNH_ISA_*. */
int bnh_add_n(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t carry_in, uint64_t *carry_out,
              int isa);

/* r[0, n) = a - b - borrow_in (mod 2^(64 n)), *borrow_out = 1 iff a < b + borrow_in. */
int bnh_sub_n(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t borrow_in, uint64_t *borrow_out,
              int isa);

/* Uniform batch: pair p at a + p n, b + p n, r + p n; carry_out[p] (may be NULL).
 * Pairs are split into `threads` contiguous ranges run on that many POSIX threads
 * (threads >= 1; 1 runs on the calling thread). */
int bnh_add_n_batch(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs, uint64_t *carry_out,
                    int isa, int threads);
int bnh_sub_n_batch(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs, uint64_t *carry_out,
                    int isa, int threads);

#ifdef __cplusplus
}
#endif

#endif /* BN_HOST_H */
