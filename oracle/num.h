/*
 * Oracle arithmetic: error-free transformations, double-double (DD) and
 * quad-double (QD) numbers, and exact floating-point expansions.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle is a plain, slow CPU model of what
 * the GPU library computes; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header or
 * constant with the GPU library.
 *
 * The paper (Kouya, "Performance evaluation of multiple precision matrix
 * multiplications using parallelized Strassen and Winograd algorithms",
 * Sec. 1 and Sec. 3) uses DD numbers (two doubles, about 106 bits) and QD
 * numbers (four doubles, about 212 bits) from Bailey's QD library.  The paper
 * prints none of that library's algorithms, so this file re-derives them
 * from published mathematics:
 *   - TwoSum (Knuth, TAOCP vol. 2, Sec. 4.2.2), FastTwoSum (Dekker 1971),
 *     TwoProd through one fused multiply-add (exact for finite results).
 *   - DD addition: the accurate double-word sum of Joldes, Muller and
 *     Popescu (ACM TOMS 2017): two TwoSums, then two FastTwoSum
 *     renormalisations; relative error about 3u^2.
 *   - DD multiplication: the FMA-based double-word product of the same
 *     paper; relative error below 5u^2.
 *   - DD division: classical long division with two correction steps.
 *   - QD: a QD value is a non-overlapping expansion truncated to its four
 *     largest terms.  Sums and products are formed exactly as expansions
 *     (Shewchuk 1997, "Adaptive precision floating-point arithmetic and
 *     fast robust geometric predicates": Grow-Expansion with zero
 *     elimination, Compress) and then rounded to four terms by repeated
 *     extraction of the compressed expansion's leading term.  This is
 *     slower than the usual QD kernels but provably accurate (relative
 *     error about 2^-208 per operation) and independent of them.
 *
 * Build with -ffp-contract=off and without -ffast-math: the EFTs rely on
 * every + - * being rounded separately.
 */
#ifndef ORACLE_NUM_H
#define ORACLE_NUM_H

#include <math.h>
#include <stdint.h>

/* ---- error-free transformations --------------------------------------- */

/* s + e == a + b exactly, s = fl(a + b).  Knuth's branch-free TwoSum. */
static inline void or_two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *e = (a - av) + (b - bv);
    *s = x;
}

/* s + e == a + b exactly, provided a == 0 or |a| >= |b| (Dekker). */
static inline void or_fast_two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    *e = b - (x - a);
    *s = x;
}

/* p + e == a * b exactly (barring underflow), p = fl(a * b). */
static inline void or_two_prod(double a, double b, double *p, double *e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* ---- exact expansions (Shewchuk 1997) ---------------------------------- */
/* An expansion is an array of doubles, non-overlapping, sorted by increasing
 * magnitude, whose exact sum is the value.  Zero components are removed.   */

/* e := e + b exactly (Grow-Expansion, zero elimination); returns new length.
 * e must have room for n + 1 entries. */
int or_exp_grow(double *e, int n, double b);

/* Rewrites e[0..n) in place as an equal-valued non-overlapping expansion
 * whose largest component approximates the sum to within one ulp
 * (Compress).  Returns the new length (0 if the sum is zero). */
int or_exp_compress(double *e, int n);

/* out[0..k) := the k leading terms of the value of e, each the leading
 * term of the compressed remainder; destroys e.  Terms beyond the value's
 * support are zero. */
void or_exp_round(double *e, int n, double *out, int k);

/* ---- DD ----------------------------------------------------------------- */
/* A DD number is (hi, lo) with value hi + lo and |lo| <= ulp(hi)/2.        */

void or_dd_add(const double *x, const double *y, double *z);
void or_dd_sub(const double *x, const double *y, double *z);
void or_dd_mul(const double *x, const double *y, double *z);
void or_dd_div(const double *x, const double *y, double *z);

/* ---- QD ----------------------------------------------------------------- */
/* A QD number is c[0..3], a non-overlapping expansion with c[0] largest.   */

void or_qd_add(const double *x, const double *y, double *z);
void or_qd_sub(const double *x, const double *y, double *z);
void or_qd_mul(const double *x, const double *y, double *z);
void or_qd_div(const double *x, const double *y, double *z);

#endif
