/*
 * Oracle LU factorisation and solve in DD or QD arithmetic
 * (TEST INFRASTRUCTURE ONLY).
 *
 * Blocked right-looking LU as the paper states it (Sec. 4, steps 1-3):
 * split A into A11 (K x K), A12, A21, A22; factor A11 = L11 U11; turn A12
 * into U12 = L11^-1 A12 and A21 into L21; update A22 := A22 - L21 U12 with
 * a matrix product; repeat on the updated A22.  The paper factors without
 * pivoting; this oracle also offers partial pivoting (row interchanges chosen
 * by the largest |a_ic| in the current column, first index on ties), in
 * which case the whole (n-j) x K panel is factored column by column and each
 * interchange is applied to full rows, as LAPACK's getrf does.  The last
 * block may be narrower than K.  The product in step 3 is any of the four
 * algorithms of gemm.c; the paper uses Winograd there (Sec. 4).
 *
 * Solving A x = b (Sec. 4, Eq. 2) applies the interchanges to b, then a
 * forward substitution with the unit lower factor and a back substitution
 * with the upper factor.
 *
 * Matrices are in plane layout (P planes of components, row-major); the
 * working copies interleave the P components of each element.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "num.h"

void or_product_numbers(int P, int algo, int levels, int bs, int64_t m, int64_t n, int64_t l,
                        double *A, int64_t lda, double *B, int64_t ldb, double *C, int64_t ldc);

/* Arithmetic of one precision: DD (P = 2) or QD (P = 4). */
typedef struct {
    int P;
    void (*sub)(const double *, const double *, double *);
    void (*mul)(const double *, const double *, double *);
    void (*div)(const double *, const double *, double *);
} lu_arith;

static lu_arith lu_arith_for(int P) {
    lu_arith a;
    a.P = P;
    a.sub = P == 2 ? or_dd_sub : or_qd_sub;
    a.mul = P == 2 ? or_dd_mul : or_qd_mul;
    a.div = P == 2 ? or_dd_div : or_qd_div;
    return a;
}

/* element (i, j) of an interleaved copy: P consecutive components */
#define E(M, ld, i, j) ((M) + ((i) * (ld) + (j)) * P)

/* sign of |x| - |y|, decided in the working precision */
static int abs_cmp(const lu_arith *ar, const double *x, const double *y) {
    const int P = ar->P;
    double ax[4], ay[4], d[4];
    for (int c = 0; c < P; c++) {
        ax[c] = x[0] < 0 ? -x[c] : x[c];
        ay[c] = y[0] < 0 ? -y[c] : y[c];
    }
    ar->sub(ax, ay, d);
    return (d[0] > 0) - (d[0] < 0);
}

static void swap_rows(double *A, int P, int64_t n, int64_t r1, int64_t r2) {
    if (r1 == r2) return;
    for (int64_t j = 0; j < n * P; j++) {
        double t = A[r1 * n * P + j];
        A[r1 * n * P + j] = A[r2 * n * P + j];
        A[r2 * n * P + j] = t;
    }
}

/* In-place factorisation in precision P; returns info (0, or 1 + the first
 * column whose pivot is exactly zero; the factorisation continues past it),
 * or -1 for bad arguments. */
int or_getrf_p(int P, int64_t n, double *Ap, int32_t *ipiv, int panel, int pivot, int algo,
               int levels, int bs) {
    if ((P != 2 && P != 4) || n < 0 || panel < 1) return -1;
    const lu_arith ar = lu_arith_for(P);
    double *A = (double *)malloc(sizeof(double) * P * (size_t)(n * n + 1));
    for (int64_t i = 0; i < n * n; i++)
        for (int c = 0; c < P; c++) A[P * i + c] = Ap[c * n * n + i];
    int info = 0;
    double t[4];
    for (int64_t j0 = 0; j0 < n; j0 += panel) {
        int64_t kb = n - j0 < panel ? n - j0 : panel;
        int64_t j1 = j0 + kb;
        /* step 2 (panel): factor columns j0..j1-1 of rows j0..n-1 */
        for (int64_t c = j0; c < j1; c++) {
            int64_t p = c;
            if (pivot)
                for (int64_t r = c + 1; r < n; r++)
                    if (abs_cmp(&ar, E(A, n, r, c), E(A, n, p, c)) > 0) p = r;
            ipiv[c] = (int32_t)p;
            swap_rows(A, P, n, c, p);
            double *piv = E(A, n, c, c);
            int zero = 1;
            for (int k = 0; k < P; k++) zero &= piv[k] == 0.0;
            if (zero) {
                if (!info) info = (int)(c + 1);
                continue;
            }
            for (int64_t r = c + 1; r < n; r++) {
                ar.div(E(A, n, r, c), piv, E(A, n, r, c));
                for (int64_t cc = c + 1; cc < j1; cc++) {
                    ar.mul(E(A, n, r, c), E(A, n, c, cc), t);
                    ar.sub(E(A, n, r, cc), t, E(A, n, r, cc));
                }
            }
        }
        if (j1 >= n) break;
        /* step 2 (row block): U12 := L11^-1 A12 by forward substitution */
        for (int64_t c = j0; c < j1; c++)
            for (int64_t r = c + 1; r < j1; r++)
                for (int64_t jj = j1; jj < n; jj++) {
                    ar.mul(E(A, n, r, c), E(A, n, c, jj), t);
                    ar.sub(E(A, n, r, jj), t, E(A, n, r, jj));
                }
        /* step 3: A22 := A22 - L21 U12 */
        int64_t r2 = n - j1;
        double *T = (double *)calloc((size_t)(r2 * r2) * P, sizeof(double));
        or_product_numbers(P, algo, levels, bs, r2, r2, kb, E(A, n, j1, j0), n, E(A, n, j0, j1), n,
                           T, r2);
        for (int64_t r = 0; r < r2; r++)
            for (int64_t c = 0; c < r2; c++)
                ar.sub(E(A, n, j1 + r, j1 + c), E(T, r2, r, c), E(A, n, j1 + r, j1 + c));
        free(T);
    }
    for (int64_t i = 0; i < n * n; i++)
        for (int c = 0; c < P; c++) Ap[c * n * n + i] = A[P * i + c];
    free(A);
    return info;
}

/* Solves A X = B with the factors of or_getrf_p; B (n x nrhs, plane layout,
 * P planes) is overwritten with X. */
int or_getrs_p(int P, int64_t n, int64_t nrhs, const double *LUp, const int32_t *ipiv,
               double *Bp) {
    if ((P != 2 && P != 4) || n < 0 || nrhs < 0) return -1;
    const lu_arith ar = lu_arith_for(P);
    double t[4], a[4];
    for (int64_t j = 0; j < nrhs; j++) {
        double *x = (double *)malloc(sizeof(double) * P * (size_t)(n + 1));
        for (int64_t i = 0; i < n; i++)
            for (int c = 0; c < P; c++) x[P * i + c] = Bp[c * n * nrhs + i * nrhs + j];
        for (int64_t i = 0; i < n; i++) {
            int64_t p = ipiv[i];
            if (p != i)
                for (int c = 0; c < P; c++) {
                    double h = x[P * i + c];
                    x[P * i + c] = x[P * p + c];
                    x[P * p + c] = h;
                }
        }
        for (int64_t i = 0; i < n; i++)
            for (int64_t k = 0; k < i; k++) {
                for (int c = 0; c < P; c++) a[c] = LUp[c * n * n + i * n + k];
                ar.mul(a, x + P * k, t);
                ar.sub(x + P * i, t, x + P * i);
            }
        for (int64_t i = n - 1; i >= 0; i--) {
            for (int64_t k = i + 1; k < n; k++) {
                for (int c = 0; c < P; c++) a[c] = LUp[c * n * n + i * n + k];
                ar.mul(a, x + P * k, t);
                ar.sub(x + P * i, t, x + P * i);
            }
            for (int c = 0; c < P; c++) a[c] = LUp[c * n * n + i * n + i];
            ar.div(x + P * i, a, x + P * i);
        }
        for (int64_t i = 0; i < n; i++)
            for (int c = 0; c < P; c++) Bp[c * n * nrhs + i * nrhs + j] = x[P * i + c];
        free(x);
    }
    return 0;
}

int or_getrf(int64_t n, double *Ap, int32_t *ipiv, int panel, int pivot, int algo, int levels,
             int bs) {
    return or_getrf_p(2, n, Ap, ipiv, panel, pivot, algo, levels, bs);
}

int or_getrs(int64_t n, int64_t nrhs, const double *LUp, const int32_t *ipiv, double *Bp) {
    return or_getrs_p(2, n, nrhs, LUp, ipiv, Bp);
}
