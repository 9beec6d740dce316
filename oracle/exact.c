/*
 * Exact matrix-product entries (TEST INFRASTRUCTURE ONLY).
 *
 * The paper defines the product entry by entry, c_ij = sum_k a_ik b_kj
 * (Sec. 2, Eq. 1), over real numbers.  Here every input number is an
 * unevaluated sum of P doubles, so each term a_ik * b_kj is the exact sum
 * of P*P TwoProd pairs; all of them are accumulated without rounding into
 * one expansion (Grow-Expansion, compressed whenever it gets long) and the
 * expansion is rounded once at the end.  The result does not depend on any
 * summation order, so it is the reference every algorithm is measured
 * against.
 *
 * Matrices are in plane layout: component c of element (i, j) of an r x s
 * matrix X is X[c*r*s + i*s + j].
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "num.h"

typedef struct {
    double *e;
    int n, cap, soft;
} expn;

static void expn_init(expn *x) {
    x->cap = 256;
    x->soft = 32;
    x->n = 0;
    x->e = (double *)malloc(sizeof(double) * (size_t)x->cap);
}

/* x := x + b exactly.  The expansion is compressed whenever it reaches a
 * soft length, which keeps each Grow-Expansion short. */
static void expn_add(expn *x, double b) {
    if (b == 0.0) return;
    if (x->n >= x->soft) {
        x->n = or_exp_compress(x->e, x->n);
        if (x->n >= x->soft / 2) x->soft *= 2;
        if (x->soft + 2 > x->cap) {
            x->cap = 2 * x->soft + 2;
            x->e = (double *)realloc(x->e, sizeof(double) * (size_t)x->cap);
        }
    }
    x->n = or_exp_grow(x->e, x->n, b);
}

/* Adds the exact product (sum of P doubles) * (sum of P doubles) * sgn. */
static void expn_add_prod(expn *x, int P, const double *a, int64_t as, const double *b,
                          int64_t bs, double sgn) {
    for (int u = 0; u < P; u++)
        for (int v = 0; v < P; v++) {
            double p, q;
            or_two_prod(a[u * as], b[v * bs], &p, &q);
            expn_add(x, sgn * q);
            expn_add(x, sgn * p);
        }
}

/* Exact value of alpha*sum_k a_ik b_kj + beta*c0_ij for the sampled (i, j),
 * with alpha in {+1,-1} and beta in {0, 1}.  c0 (may be NULL when beta is
 * 0) holds P numbers per sample, component-major: c0[c*nidx + t].
 * On return out[c*nidx + t], c < kout, holds the leading kout terms. */
void or_exact_entries(int P, int64_t m, int64_t n, int64_t l, int alpha, int beta,
                      const double *A, const double *B, const double *c0, int64_t nidx,
                      const int64_t *ii, const int64_t *jj, int kout, double *out) {
    int64_t psa = m * l, psb = l * n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nidx; t++) {
        expn x;
        expn_init(&x);
        int64_t i = ii[t], j = jj[t];
        for (int64_t k = 0; k < l; k++)
            expn_add_prod(&x, P, A + i * l + k, psa, B + k * n + j, psb, (double)alpha);
        if (beta)
            for (int c = P - 1; c >= 0; c--) expn_add(&x, c0[c * nidx + t]);
        double r[8];
        or_exp_round(x.e, x.n, r, kout);
        for (int c = 0; c < kout; c++) out[c * nidx + t] = r[c];
        free(x.e);
    }
}

/* As or_exact_entries, but returns for each sample the leading term of the
 * exact difference (exact value) - (sum of the Pc doubles chat[c*nidx+t]).
 * This measures a computed entry's error without rounding the reference. */
void or_exact_error(int P, int64_t m, int64_t n, int64_t l, int alpha, int beta,
                    const double *A, const double *B, const double *c0, int64_t nidx,
                    const int64_t *ii, const int64_t *jj, int Pc, const double *chat,
                    double *err) {
    int64_t psa = m * l, psb = l * n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nidx; t++) {
        expn x;
        expn_init(&x);
        int64_t i = ii[t], j = jj[t];
        for (int64_t k = 0; k < l; k++)
            expn_add_prod(&x, P, A + i * l + k, psa, B + k * n + j, psb, (double)alpha);
        if (beta)
            for (int c = P - 1; c >= 0; c--) expn_add(&x, c0[c * nidx + t]);
        for (int c = Pc - 1; c >= 0; c--) expn_add(&x, -chat[c * nidx + t]);
        double r[1];
        or_exp_round(x.e, x.n, r, 1);
        err[t] = r[0];
        free(x.e);
    }
}

/* The raw expansion of sum_k x_k y_k for two length-l vectors of P-double
 * numbers (component stride ps).  Writes at most cap components,
 * increasing magnitude, and returns the count (-1 if cap is too small). */
int or_exact_dot_expansion(int P, int64_t l, const double *x, int64_t psx, const double *y,
                           int64_t psy, double *out, int cap) {
    expn e;
    expn_init(&e);
    for (int64_t k = 0; k < l; k++) expn_add_prod(&e, P, x + k, psx, y + k, psy, 1.0);
    e.n = or_exp_compress(e.e, e.n);
    int n = e.n;
    if (n > cap) {
        free(e.e);
        return -1;
    }
    memcpy(out, e.e, sizeof(double) * (size_t)n);
    free(e.e);
    return n;
}

/* Expansion helpers exported for the tests' exactness pins. */
int or_expansion_sum(const double *in, int nin, double *out) {
    int n = 0;
    for (int i = 0; i < nin; i++) n = or_exp_grow(out, n, in[i]);
    return or_exp_compress(out, n);
}

void or_expansion_round(const double *in, int nin, int k, double *out) {
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(nin + 1));
    int n = 0;
    for (int i = 0; i < nin; i++) n = or_exp_grow(tmp, n, in[i]);
    or_exp_round(tmp, n, out, k);
    free(tmp);
}

/* Elementwise arithmetic exported for pins: op 0 add, 1 sub, 2 mul, 3 div
 * (div for DD only).  x, y, z hold cnt numbers of P doubles each, AoS. */
void or_elementwise(int P, int op, int64_t cnt, const double *x, const double *y, double *z) {
    for (int64_t t = 0; t < cnt; t++) {
        const double *a = x + t * P, *b = y + t * P;
        double *c = z + t * P;
        if (P == 2) {
            if (op == 0) or_dd_add(a, b, c);
            else if (op == 1) or_dd_sub(a, b, c);
            else if (op == 2) or_dd_mul(a, b, c);
            else or_dd_div(a, b, c);
        } else {
            if (op == 0) or_qd_add(a, b, c);
            else if (op == 1) or_qd_sub(a, b, c);
            else if (op == 2) or_qd_mul(a, b, c);
            else or_qd_div(a, b, c);
        }
    }
}

/* Error-free transformations exported for pins: op 0 TwoSum, 1 FastTwoSum,
 * 2 TwoProd on cnt pairs; writes s[t], e[t]. */
void or_eft(int op, int64_t cnt, const double *a, const double *b, double *s, double *e) {
    for (int64_t t = 0; t < cnt; t++) {
        if (op == 0) or_two_sum(a[t], b[t], &s[t], &e[t]);
        else if (op == 1) or_fast_two_sum(a[t], b[t], &s[t], &e[t]);
        else or_two_prod(a[t], b[t], &s[t], &e[t]);
    }
}
