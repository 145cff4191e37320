/*
 * bn_oracle.c -- plain, slow, obviously correct CPU oracle for large-number
 * add / sub / mul over little-endian 64-bit limbs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it (through oracle/__init__.py).  It shares no code,
 * header, table or helper with the GPU path.
 *
 * Number format (paper, Sec. 2.1 "Large numbers and their representation", and
 * the statement of Theorem 1): an m-limb operand is A = sum_{i<m} A_i X^i with
 * X = 2^64 (saturated radix), limb 0 least significant, 0 <= A_i < X.
 *
 * Every routine is the plain definition the paper proves DoT equal to; no
 * blocking, no vectorisation, no reordering beyond that definition.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>

typedef unsigned __int128 u128;

/*
 * Addition: Theorem 1 (Sec. 3.1, "Correctness of DoT-Addition") defines the
 * result as r_i = (A_i + B_i + c_i) mod X, c_0 = 0, c_{i+1} = floor((A_i + B_i +
 * c_i) / X), carry-out c_m.  This is also the sequential carry chain of the
 * GMP-style MPN-ADD-M (Appendix A, Algorithm 3).  Written out with a 128-bit
 * intermediate so the floor/mod are literal.  r may alias a or b exactly.
 */
uint64_t bnref_add_n(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n)
{
    uint64_t c = 0;
    for (size_t i = 0; i < n; ++i) {
        u128 t = (u128)a[i] + (u128)b[i] + (u128)c;
        r[i] = (uint64_t)t;            /* (A_i + B_i + c_i) mod X   */
        c = (uint64_t)(t >> 64);       /* floor((A_i + B_i + c_i)/X) */
    }
    return c;
}

/*
 * Subtraction: the paper states that DoT subtraction mirrors addition with
 * borrows in place of carries (Sec. 3.1, "Subtraction").  Plain definition:
 * r_i = (A_i - B_i - br_i) mod X, br_0 = 0, br_{i+1} = [A_i < B_i + br_i].
 * For A < B the result is (A - B) mod X^m with final borrow 1 (the convention of
 * the mpn-level primitive the paper replaces).  r may alias a or b exactly.
 */
uint64_t bnref_sub_n(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n)
{
    uint64_t br = 0;
    for (size_t i = 0; i < n; ++i) {
        u128 need = (u128)b[i] + (u128)br;      /* B_i + br_i, up to 2^64 */
        u128 t = (u128)a[i] - need;             /* wraps mod 2^128 when negative */
        r[i] = (uint64_t)t;
        br = ((u128)a[i] < need) ? 1u : 0u;
    }
    return br;
}

/*
 * Multiplication: Theorem 2 (Sec. 3.2, vertical-and-crosswise correctness and
 * its proof in Appendix B) fixes A x B = sum_i sum_j A_i B_j X^{i+j}.  The plain
 * definition is written here as textbook row-by-row schoolbook accumulation
 * (Appendix A, "base-case multiplication routines"): for every i, add A_i * B
 * shifted by i limbs into r.  Each step t = A_i*B_j + r_{i+j} + c is at most
 * (X-1)^2 + 2(X-1) = X^2 - 1, so the 128-bit intermediate never overflows.
 * The product has exactly na+nb limbs (leading zero limbs kept).
 * r must not overlap a or b.
 */
void bnref_mul(uint64_t *r, const uint64_t *a, size_t na, const uint64_t *b, size_t nb)
{
    memset(r, 0, (na + nb) * sizeof(uint64_t));
    for (size_t i = 0; i < na; ++i) {
        uint64_t c = 0;
        for (size_t j = 0; j < nb; ++j) {
            u128 t = (u128)a[i] * (u128)b[j] + (u128)r[i + j] + (u128)c;
            r[i + j] = (uint64_t)t;
            c = (uint64_t)(t >> 64);
        }
        r[i + nb] = c;
    }
}

/* ---- batch forms: a plain loop over independent pairs, nothing more ---- */

/* pair p occupies limbs [p*n, (p+1)*n) of r, a, b; carry[p] in {0,1} (carry may be NULL) */
void bnref_add_n_batch(uint64_t *r, const uint64_t *a, const uint64_t *b,
                       size_t n, size_t npairs, uint64_t *carry)
{
    for (size_t p = 0; p < npairs; ++p) {
        uint64_t c = bnref_add_n(r + p * n, a + p * n, b + p * n, n);
        if (carry) carry[p] = c;
    }
}

void bnref_sub_n_batch(uint64_t *r, const uint64_t *a, const uint64_t *b,
                       size_t n, size_t npairs, uint64_t *borrow)
{
    for (size_t p = 0; p < npairs; ++p) {
        uint64_t c = bnref_sub_n(r + p * n, a + p * n, b + p * n, n);
        if (borrow) borrow[p] = c;
    }
}

/*
 * With a carry (borrow) into limb 0: the W-limb addition step of Alg. 1 takes a
 * carry-in c_in (Sec. 3.1); the recurrences above with c_0 = cin (resp. br_0 = bin)
 * instead of 0.  cin, bin in {0, 1}.
 */
uint64_t bnref_add_nc(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t cin)
{
    uint64_t c = cin;
    for (size_t i = 0; i < n; ++i) {
        u128 t = (u128)a[i] + (u128)b[i] + (u128)c;
        r[i] = (uint64_t)t;
        c = (uint64_t)(t >> 64);
    }
    return c;
}

uint64_t bnref_sub_nc(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t bin)
{
    uint64_t br = bin;
    for (size_t i = 0; i < n; ++i) {
        u128 need = (u128)b[i] + (u128)br;
        u128 t = (u128)a[i] - need;
        r[i] = (uint64_t)t;
        br = ((u128)a[i] < need) ? 1u : 0u;
    }
    return br;
}

void bnref_add_nc_batch(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs,
                        const uint64_t *cin, uint64_t *carry)
{
    for (size_t p = 0; p < npairs; ++p) {
        uint64_t c = bnref_add_nc(r + p * n, a + p * n, b + p * n, n, cin[p] & 1u);
        if (carry) carry[p] = c;
    }
}

void bnref_sub_nc_batch(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, size_t npairs,
                        const uint64_t *bin, uint64_t *borrow)
{
    for (size_t p = 0; p < npairs; ++p) {
        uint64_t c = bnref_sub_nc(r + p * n, a + p * n, b + p * n, n, bin[p] & 1u);
        if (borrow) borrow[p] = c;
    }
}

/* pair p: a at p*na, b at p*nb, product at p*(na+nb) */
void bnref_mul_n_batch(uint64_t *r, const uint64_t *a, const uint64_t *b,
                       size_t na, size_t nb, size_t npairs)
{
    for (size_t p = 0; p < npairs; ++p)
        bnref_mul(r + p * (na + nb), a + p * na, na, b + p * nb, nb);
}

/*
 * Ragged batch: desc holds 5 uint64 per pair {a_off, b_off, r_off, na, nb},
 * offsets in limbs into the pooled arrays; the product of pair p is written to
 * r_pool[r_off .. r_off + na + nb).
 */
void bnref_mul_ragged(uint64_t *r_pool, const uint64_t *a_pool, const uint64_t *b_pool,
                      const uint64_t *desc, size_t npairs)
{
    for (size_t p = 0; p < npairs; ++p) {
        const uint64_t *d = desc + 5 * p;
        bnref_mul(r_pool + d[2], a_pool + d[0], (size_t)d[3], b_pool + d[1], (size_t)d[4]);
    }
}

/* same descriptor layout; na must equal nb; carry[p] (may be NULL) */
void bnref_add_ragged(uint64_t *r_pool, const uint64_t *a_pool, const uint64_t *b_pool,
                      const uint64_t *desc, size_t npairs, uint64_t *carry)
{
    for (size_t p = 0; p < npairs; ++p) {
        const uint64_t *d = desc + 5 * p;
        uint64_t c = bnref_add_n(r_pool + d[2], a_pool + d[0], b_pool + d[1], (size_t)d[3]);
        if (carry) carry[p] = c;
    }
}
