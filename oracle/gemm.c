/*
 * Oracle matrix products C := A B in DD or QD arithmetic
 * (TEST INFRASTRUCTURE ONLY).
 *
 * The four algorithms the paper times (Sec. 2 and Sec. 3, Tables 1-2):
 *   Simple   c_ij := sum_k a_ik b_kj with k ascending (Sec. 2, Eq. 1);
 *   Block    C_ij := sum_K A_iK B_Kj over square blocks of side bs, each
 *            block product formed on its own and then added (Sec. 2);
 *   Strassen Strassen's 1969 seven-product recursion, `levels` deep;
 *   Winograd the Strassen-Winograd variant (seven products, fifteen
 *            additions), `levels` deep.
 * The paper's figures of the parallel Strassen and Winograd schemes are not
 * available, so the formulas are the textbook ones, written out below.
 * A Strassen or Winograd product is equilibrated first (exact power-of-two
 * row scaling of A and column scaling of B, undone on C; see product_top).
 * Below the recursion (levels == 0, or a dimension below 2) the product is
 * Block.  A dimension that is odd at some level is peeled: the even leading
 * part recurses, and the odd last column of A / row of B (a rank-one
 * update), the last column of C and the last row of C are Block products.
 *
 * Arithmetic is the oracle's DD (P = 2) or QD (P = 4) from num.c.  Inside,
 * a matrix is an array of P-double numbers: element (i, j) of M starts at
 * M.p + (i*M.ld + j)*P.  Row blocks run in parallel with OpenMP, which
 * does not change any result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#include <string.h>

#include "num.h"

typedef void (*binop)(const double *, const double *, double *);

typedef struct {
    int P;
    binop add, sub, mul;
} arith;

typedef struct {
    double *p;
    int64_t ld;
} mat;

static inline double *at(const arith *ar, mat M, int64_t i, int64_t j) {
    return M.p + (i * M.ld + j) * ar->P;
}

static mat sub(const arith *ar, mat M, int64_t i, int64_t j) {
    mat r = {at(ar, M, i, j), M.ld};
    return r;
}

static mat mat_new(const arith *ar, int64_t r, int64_t c) {
    mat M;
    M.ld = c > 0 ? c : 1;
    M.p = (double *)calloc((size_t)(r > 0 ? r : 1) * (size_t)M.ld * ar->P, sizeof(double));
    return M;
}

/* Z := X op Y elementwise over r x c. */
static void ew(const arith *ar, binop op, int64_t r, int64_t c, mat X, mat Y, mat Z) {
#pragma omp parallel for schedule(static) if (r * c > 4096)
    for (int64_t i = 0; i < r; i++)
        for (int64_t j = 0; j < c; j++) op(at(ar, X, i, j), at(ar, Y, i, j), at(ar, Z, i, j));
}

static void simple(const arith *ar, int64_t m, int64_t n, int64_t l, mat A, mat B, mat C) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; i++) {
        double acc[4], t[4];
        for (int64_t j = 0; j < n; j++) {
            memset(acc, 0, sizeof acc);
            for (int64_t k = 0; k < l; k++) {
                ar->mul(at(ar, A, i, k), at(ar, B, k, j), t);
                ar->add(acc, t, acc);
            }
            memcpy(at(ar, C, i, j), acc, sizeof(double) * ar->P);
        }
    }
}

static void block(const arith *ar, int bs, int64_t m, int64_t n, int64_t l, mat A, mat B,
                  mat C) {
    int64_t mb = (m + bs - 1) / bs, nb = (n + bs - 1) / bs;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int64_t bi = 0; bi < mb; bi++)
        for (int64_t bj = 0; bj < nb; bj++) {
            int64_t i0 = bi * bs, j0 = bj * bs;
            int64_t i1 = i0 + bs < m ? i0 + bs : m, j1 = j0 + bs < n ? j0 + bs : n;
            double acc[4], t[4];
            for (int64_t i = i0; i < i1; i++)
                for (int64_t j = j0; j < j1; j++) memset(at(ar, C, i, j), 0, sizeof(double) * ar->P);
            for (int64_t k0 = 0; k0 < l; k0 += bs) {
                int64_t k1 = k0 + bs < l ? k0 + bs : l;
                /* block product A_iK B_Kj, then C_ij += it */
                for (int64_t i = i0; i < i1; i++)
                    for (int64_t j = j0; j < j1; j++) {
                        memset(acc, 0, sizeof acc);
                        for (int64_t k = k0; k < k1; k++) {
                            ar->mul(at(ar, A, i, k), at(ar, B, k, j), t);
                            ar->add(acc, t, acc);
                        }
                        ar->add(at(ar, C, i, j), acc, at(ar, C, i, j));
                    }
            }
        }
}

static void product(const arith *ar, int algo, int levels, int bs, int64_t m, int64_t n,
                    int64_t l, mat A, mat B, mat C);

/* C := A B for even m, n, l by one Strassen (algo 2) or Winograd (algo 3)
 * step; the seven products recurse with levels - 1. */
static void seven(const arith *ar, int algo, int levels, int bs, int64_t m, int64_t n, int64_t l,
                  mat A, mat B, mat C) {
    int64_t h = m / 2, q = l / 2, w = n / 2;
    mat A11 = sub(ar, A, 0, 0), A12 = sub(ar, A, 0, q), A21 = sub(ar, A, h, 0), A22 = sub(ar, A, h, q);
    mat B11 = sub(ar, B, 0, 0), B12 = sub(ar, B, 0, w), B21 = sub(ar, B, q, 0), B22 = sub(ar, B, q, w);
    mat C11 = sub(ar, C, 0, 0), C12 = sub(ar, C, 0, w), C21 = sub(ar, C, h, 0), C22 = sub(ar, C, h, w);
    mat M[7];
    for (int t = 0; t < 7; t++) M[t] = mat_new(ar, h, w);
    mat S1 = mat_new(ar, h, q), S2 = mat_new(ar, h, q), T1 = mat_new(ar, q, w), T2 = mat_new(ar, q, w);
    int nl = levels - 1;
    if (algo == 2) {
        /* Strassen 1969:
         * M1=(A11+A22)(B11+B22) M2=(A21+A22)B11 M3=A11(B12-B22) M4=A22(B21-B11)
         * M5=(A11+A12)B22 M6=(A21-A11)(B11+B12) M7=(A12-A22)(B21+B22)
         * C11=M1+M4-M5+M7 C12=M3+M5 C21=M2+M4 C22=M1-M2+M3+M6 */
        ew(ar, ar->add, h, q, A11, A22, S1);
        ew(ar, ar->add, q, w, B11, B22, T1);
        product(ar, algo, nl, bs, h, w, q, S1, T1, M[0]);
        ew(ar, ar->add, h, q, A21, A22, S1);
        product(ar, algo, nl, bs, h, w, q, S1, B11, M[1]);
        ew(ar, ar->sub, q, w, B12, B22, T1);
        product(ar, algo, nl, bs, h, w, q, A11, T1, M[2]);
        ew(ar, ar->sub, q, w, B21, B11, T1);
        product(ar, algo, nl, bs, h, w, q, A22, T1, M[3]);
        ew(ar, ar->add, h, q, A11, A12, S1);
        product(ar, algo, nl, bs, h, w, q, S1, B22, M[4]);
        ew(ar, ar->sub, h, q, A21, A11, S1);
        ew(ar, ar->add, q, w, B11, B12, T1);
        product(ar, algo, nl, bs, h, w, q, S1, T1, M[5]);
        ew(ar, ar->sub, h, q, A12, A22, S1);
        ew(ar, ar->add, q, w, B21, B22, T1);
        product(ar, algo, nl, bs, h, w, q, S1, T1, M[6]);
        ew(ar, ar->add, h, w, M[0], M[3], C11);
        ew(ar, ar->sub, h, w, C11, M[4], C11);
        ew(ar, ar->add, h, w, C11, M[6], C11);
        ew(ar, ar->add, h, w, M[2], M[4], C12);
        ew(ar, ar->add, h, w, M[1], M[3], C21);
        ew(ar, ar->sub, h, w, M[0], M[1], C22);
        ew(ar, ar->add, h, w, C22, M[2], C22);
        ew(ar, ar->add, h, w, C22, M[5], C22);
    } else {
        /* Strassen-Winograd:
         * S1=A21+A22 S2=S1-A11 S3=A11-A21 S4=A12-S2
         * T1=B12-B11 T2=B22-T1 T3=B22-B12 T4=T2-B21
         * P1=A11B11 P2=A12B21 P3=S4B22 P4=A22T4 P5=S1T1 P6=S2T2 P7=S3T3
         * U2=P1+P6 U3=U2+P7 U4=U2+P5
         * C11=P1+P2 C12=U4+P3 C21=U3-P4 C22=U3+P5 */
        mat S3 = mat_new(ar, h, q), T3 = mat_new(ar, q, w);
        ew(ar, ar->add, h, q, A21, A22, S1);
        ew(ar, ar->sub, h, q, S1, A11, S2);
        ew(ar, ar->sub, h, q, A11, A21, S3);
        ew(ar, ar->sub, q, w, B12, B11, T1);
        ew(ar, ar->sub, q, w, B22, T1, T2);
        ew(ar, ar->sub, q, w, B22, B12, T3);
        product(ar, algo, nl, bs, h, w, q, A11, B11, M[0]);
        product(ar, algo, nl, bs, h, w, q, A12, B21, M[1]);
        product(ar, algo, nl, bs, h, w, q, S1, T1, M[4]);
        product(ar, algo, nl, bs, h, w, q, S2, T2, M[5]);
        product(ar, algo, nl, bs, h, w, q, S3, T3, M[6]);
        /* S4 and T4 reuse S3 and T3 */
        ew(ar, ar->sub, h, q, A12, S2, S3);
        ew(ar, ar->sub, q, w, T2, B21, T3);
        product(ar, algo, nl, bs, h, w, q, S3, B22, M[2]);
        product(ar, algo, nl, bs, h, w, q, A22, T3, M[3]);
        ew(ar, ar->add, h, w, M[0], M[1], C11);
        ew(ar, ar->add, h, w, M[0], M[5], C21);          /* U2 */
        ew(ar, ar->add, h, w, C21, M[4], C12);           /* U4 = U2 + P5 */
        ew(ar, ar->add, h, w, C12, M[2], C12);           /* C12 = U4 + P3 */
        ew(ar, ar->add, h, w, C21, M[6], C21);           /* U3 = U2 + P7 */
        ew(ar, ar->add, h, w, C21, M[4], C22);           /* C22 = U3 + P5 */
        ew(ar, ar->sub, h, w, C21, M[3], C21);           /* C21 = U3 - P4 */
        free(S3.p);
        free(T3.p);
    }
    for (int t = 0; t < 7; t++) free(M[t].p);
    free(S1.p);
    free(S2.p);
    free(T1.p);
    free(T2.p);
}

static void product(const arith *ar, int algo, int levels, int bs, int64_t m, int64_t n,
                    int64_t l, mat A, mat B, mat C) {
    if (m <= 0 || n <= 0) return;
    if (l <= 0) {
        for (int64_t i = 0; i < m; i++)
            for (int64_t j = 0; j < n; j++) memset(at(ar, C, i, j), 0, sizeof(double) * ar->P);
        return;
    }
    if (algo == 0) {
        simple(ar, m, n, l, A, B, C);
        return;
    }
    if (algo == 1 || levels <= 0 || m < 2 || n < 2 || l < 2) {
        block(ar, bs, m, n, l, A, B, C);
        return;
    }
    int64_t me = m & ~(int64_t)1, ne = n & ~(int64_t)1, le = l & ~(int64_t)1;
    seven(ar, algo, levels, bs, me, ne, le, A, B, C);
    if (l != le) { /* rank-one update with the last column of A, last row of B */
        mat T = mat_new(ar, me, ne);
        block(ar, bs, me, ne, 1, sub(ar, A, 0, le), sub(ar, B, le, 0), T);
        ew(ar, ar->add, me, ne, C, T, C);
        free(T.p);
    }
    if (n != ne) block(ar, bs, me, 1, l, A, sub(ar, B, 0, ne), sub(ar, C, 0, ne));
    if (m != me) block(ar, bs, 1, n, l, sub(ar, A, me, 0), B, sub(ar, C, me, 0));
}

/* Exact power-of-two equilibration around a Strassen / Winograd product:
 * row i of A is scaled by 2^-e_i and column j of B by 2^-f_j, where 2^e_i and
 * 2^f_j bound the row's / column's largest leading component, the product of
 * the scaled matrices is formed, and entry (i, j) is scaled back by
 * 2^(e_i + f_j).  The recursion's sums then mix rows (and columns) of equal
 * scale, so the row-normwise error does not depend on the rows' magnitudes.
 * Conventional products need no scaling and get none. */
static void product_top(const arith *ar, int algo, int levels, int bs, int64_t m, int64_t n,
                        int64_t l, mat A, mat B, mat C) {
    if (!(algo == 2 || algo == 3) || levels <= 0 || m < 2 || n < 2 || l < 2) {
        product(ar, algo, levels, bs, m, n, l, A, B, C);
        return;
    }
    int P = ar->P;
    int *ea = (int *)calloc((size_t)m, sizeof(int)), *fb = (int *)calloc((size_t)n, sizeof(int));
    for (int64_t i = 0; i < m; i++) {
        double mx = 0.0;
        for (int64_t k = 0; k < l; k++) mx = fmax(mx, fabs(at(ar, A, i, k)[0]));
        if (mx > 0.0) frexp(mx, &ea[i]);
    }
    for (int64_t j = 0; j < n; j++) {
        double mx = 0.0;
        for (int64_t k = 0; k < l; k++) mx = fmax(mx, fabs(at(ar, B, k, j)[0]));
        if (mx > 0.0) frexp(mx, &fb[j]);
    }
    mat As = mat_new(ar, m, l), Bs = mat_new(ar, l, n);
    for (int64_t i = 0; i < m; i++)
        for (int64_t k = 0; k < l; k++)
            for (int c = 0; c < P; c++) at(ar, As, i, k)[c] = ldexp(at(ar, A, i, k)[c], -ea[i]);
    for (int64_t k = 0; k < l; k++)
        for (int64_t j = 0; j < n; j++)
            for (int c = 0; c < P; c++) at(ar, Bs, k, j)[c] = ldexp(at(ar, B, k, j)[c], -fb[j]);
    product(ar, algo, levels, bs, m, n, l, As, Bs, C);
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++)
            for (int c = 0; c < P; c++)
                at(ar, C, i, j)[c] = ldexp(at(ar, C, i, j)[c], ea[i] + fb[j]);
    free(As.p);
    free(Bs.p);
    free(ea);
    free(fb);
}

/* planes <-> numbers */
static void from_planes(int P, int64_t r, int64_t c, const double *src, double *dst) {
    for (int64_t i = 0; i < r * c; i++)
        for (int k = 0; k < P; k++) dst[i * P + k] = src[k * r * c + i];
}
static void to_planes(int P, int64_t r, int64_t c, const double *src, double *dst) {
    for (int64_t i = 0; i < r * c; i++)
        for (int k = 0; k < P; k++) dst[k * r * c + i] = src[i * P + k];
}

static void arith_of(int P, arith *ar) {
    ar->P = P;
    if (P == 2) {
        ar->add = or_dd_add;
        ar->sub = or_dd_sub;
        ar->mul = or_dd_mul;
    } else {
        ar->add = or_qd_add;
        ar->sub = or_qd_sub;
        ar->mul = or_qd_mul;
    }
}

/* C := A B.  P = 2 (DD) or 4 (QD); algo 0 Simple, 1 Block, 2 Strassen,
 * 3 Winograd; bs is the Block side (the paper uses 32).  A (m x l), B
 * (l x n) and C (m x n) are in plane layout.  Returns 0, or -1 on bad
 * arguments. */
int or_gemm(int P, int algo, int levels, int bs, int64_t m, int64_t n, int64_t l,
            const double *A, const double *B, double *C) {
    if ((P != 2 && P != 4) || algo < 0 || algo > 3 || bs < 1 || m < 0 || n < 0 || l < 0)
        return -1;
    arith ar;
    arith_of(P, &ar);
    mat a = mat_new(&ar, m, l), b = mat_new(&ar, l, n), c = mat_new(&ar, m, n);
    from_planes(P, m, l, A, a.p);
    from_planes(P, l, n, B, b.p);
    product_top(&ar, algo, levels, bs, m, n, l, a, b, c);
    to_planes(P, m, n, c.p, C);
    free(a.p);
    free(b.p);
    free(c.p);
    return 0;
}

/* Used by the LU oracle: C := A B on number-layout matrices. */
void or_product_numbers(int P, int algo, int levels, int bs, int64_t m, int64_t n, int64_t l,
                        double *A, int64_t lda, double *B, int64_t ldb, double *C, int64_t ldc) {
    arith ar;
    arith_of(P, &ar);
    mat a = {A, lda}, b = {B, ldb}, c = {C, ldc};
    product_top(&ar, algo, levels, bs, m, n, l, a, b, c);
}

/* Host thread control for timing the oracle (no arithmetic). */
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }
