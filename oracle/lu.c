/*
 * Oracle LU factorisation and solve in DD arithmetic
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
 * Matrices are in plane layout (hi plane, then lo plane, row-major).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "num.h"

void or_product_numbers(int P, int algo, int levels, int bs, int64_t m, int64_t n, int64_t l,
                        double *A, int64_t lda, double *B, int64_t ldb, double *C, int64_t ldc);

#define E(M, ld, i, j) ((M) + ((i) * (ld) + (j)) * 2)

/* sign of |x| - |y| for DD numbers, decided in DD arithmetic */
static int dd_abs_cmp(const double *x, const double *y) {
    double ax[2] = {x[0], x[1]}, ay[2] = {y[0], y[1]}, d[2];
    if (ax[0] < 0) { ax[0] = -ax[0]; ax[1] = -ax[1]; }
    if (ay[0] < 0) { ay[0] = -ay[0]; ay[1] = -ay[1]; }
    or_dd_sub(ax, ay, d);
    return (d[0] > 0) - (d[0] < 0);
}

static void swap_rows(double *A, int64_t n, int64_t r1, int64_t r2) {
    if (r1 == r2) return;
    for (int64_t j = 0; j < n * 2; j++) {
        double t = A[r1 * n * 2 + j];
        A[r1 * n * 2 + j] = A[r2 * n * 2 + j];
        A[r2 * n * 2 + j] = t;
    }
}

/* In-place factorisation; returns info (0, or 1 + the first column whose
 * pivot is exactly zero; the factorisation continues past it). */
int or_getrf(int64_t n, double *Ap, int32_t *ipiv, int panel, int pivot, int algo, int levels,
             int bs) {
    if (n < 0 || panel < 1) return -1;
    double *A = (double *)malloc(sizeof(double) * 2 * (size_t)(n * n + 1));
    for (int64_t i = 0; i < n * n; i++) {
        A[2 * i] = Ap[i];
        A[2 * i + 1] = Ap[n * n + i];
    }
    int info = 0;
    double t[2];
    for (int64_t j0 = 0; j0 < n; j0 += panel) {
        int64_t kb = n - j0 < panel ? n - j0 : panel;
        int64_t j1 = j0 + kb;
        /* step 2 (panel): factor columns j0..j1-1 of rows j0..n-1 */
        for (int64_t c = j0; c < j1; c++) {
            int64_t p = c;
            if (pivot)
                for (int64_t r = c + 1; r < n; r++)
                    if (dd_abs_cmp(E(A, n, r, c), E(A, n, p, c)) > 0) p = r;
            ipiv[c] = (int32_t)p;
            swap_rows(A, n, c, p);
            double *piv = E(A, n, c, c);
            if (piv[0] == 0.0 && piv[1] == 0.0) {
                if (!info) info = (int)(c + 1);
                continue;
            }
            for (int64_t r = c + 1; r < n; r++) {
                or_dd_div(E(A, n, r, c), piv, E(A, n, r, c));
                for (int64_t cc = c + 1; cc < j1; cc++) {
                    or_dd_mul(E(A, n, r, c), E(A, n, c, cc), t);
                    or_dd_sub(E(A, n, r, cc), t, E(A, n, r, cc));
                }
            }
        }
        if (j1 >= n) break;
        /* step 2 (row block): U12 := L11^-1 A12 by forward substitution */
        for (int64_t c = j0; c < j1; c++)
            for (int64_t r = c + 1; r < j1; r++)
                for (int64_t jj = j1; jj < n; jj++) {
                    or_dd_mul(E(A, n, r, c), E(A, n, c, jj), t);
                    or_dd_sub(E(A, n, r, jj), t, E(A, n, r, jj));
                }
        /* step 3: A22 := A22 - L21 U12 */
        int64_t r2 = n - j1;
        double *T = (double *)calloc((size_t)(r2 * r2) * 2, sizeof(double));
        or_product_numbers(2, algo, levels, bs, r2, r2, kb, E(A, n, j1, j0), n, E(A, n, j0, j1), n,
                           T, r2);
        for (int64_t r = 0; r < r2; r++)
            for (int64_t c = 0; c < r2; c++)
                or_dd_sub(E(A, n, j1 + r, j1 + c), E(T, r2, r, c), E(A, n, j1 + r, j1 + c));
        free(T);
    }
    for (int64_t i = 0; i < n * n; i++) {
        Ap[i] = A[2 * i];
        Ap[n * n + i] = A[2 * i + 1];
    }
    free(A);
    return info;
}

/* Solves A X = B with the factors of or_getrf; B (n x nrhs, plane layout)
 * is overwritten with X. */
int or_getrs(int64_t n, int64_t nrhs, const double *LUp, const int32_t *ipiv, double *Bp) {
    if (n < 0 || nrhs < 0) return -1;
    double t[2];
    for (int64_t j = 0; j < nrhs; j++) {
        double *x = (double *)malloc(sizeof(double) * 2 * (size_t)(n + 1));
        for (int64_t i = 0; i < n; i++) {
            x[2 * i] = Bp[i * nrhs + j];
            x[2 * i + 1] = Bp[n * nrhs + i * nrhs + j];
        }
        for (int64_t i = 0; i < n; i++) {
            int64_t p = ipiv[i];
            if (p != i) {
                double h = x[2 * i], lo = x[2 * i + 1];
                x[2 * i] = x[2 * p];
                x[2 * i + 1] = x[2 * p + 1];
                x[2 * p] = h;
                x[2 * p + 1] = lo;
            }
        }
        for (int64_t i = 0; i < n; i++)
            for (int64_t k = 0; k < i; k++) {
                double lik[2] = {LUp[i * n + k], LUp[n * n + i * n + k]};
                or_dd_mul(lik, x + 2 * k, t);
                or_dd_sub(x + 2 * i, t, x + 2 * i);
            }
        for (int64_t i = n - 1; i >= 0; i--) {
            for (int64_t k = i + 1; k < n; k++) {
                double uik[2] = {LUp[i * n + k], LUp[n * n + i * n + k]};
                or_dd_mul(uik, x + 2 * k, t);
                or_dd_sub(x + 2 * i, t, x + 2 * i);
            }
            double uii[2] = {LUp[i * n + i], LUp[n * n + i * n + i]};
            or_dd_div(x + 2 * i, uii, x + 2 * i);
        }
        for (int64_t i = 0; i < n; i++) {
            Bp[i * nrhs + j] = x[2 * i];
            Bp[n * nrhs + i * nrhs + j] = x[2 * i + 1];
        }
        free(x);
    }
    return 0;
}
