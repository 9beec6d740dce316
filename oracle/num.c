/*
 * Oracle arithmetic (TEST INFRASTRUCTURE ONLY): exact expansions, DD and QD
 * operations.  See num.h for the published algorithms each routine follows.
 */
#include "num.h"

#include <stdlib.h>
#include <string.h>

/* ---- expansions --------------------------------------------------------- */

int or_exp_grow(double *e, int n, double b) {
    /* Grow-Expansion: carry Q through the components from the smallest up;
     * every rounding error h is kept as a component (zeros dropped).  The
     * output index never passes the input index, so it runs in place. */
    double q = b;
    int k = 0;
    for (int i = 0; i < n; i++) {
        double h;
        or_two_sum(q, e[i], &q, &h);
        if (h != 0.0) e[k++] = h;
    }
    if (q != 0.0) e[k++] = q;
    return k;
}

int or_exp_compress(double *e, int n) {
    /* Compress: a top-down pass that merges components into larger ones,
     * then a bottom-up pass that pushes the carries to the top.  TwoSum is
     * used where the published form uses FastTwoSum; it returns the same
     * pair whenever FastTwoSum's precondition holds and is exact always. */
    if (n <= 0) return 0;
    double stackbuf[64];
    double *g = n <= 64 ? stackbuf : (double *)malloc(sizeof(double) * (size_t)n);
    double Q = e[n - 1];
    int bottom = n - 1;
    for (int i = n - 2; i >= 0; i--) {
        double q;
        or_two_sum(Q, e[i], &Q, &q);
        if (q != 0.0) {
            g[bottom--] = Q;
            Q = q;
        }
    }
    g[bottom] = Q;
    int top = 0;
    for (int i = bottom + 1; i < n; i++) {
        double q;
        or_two_sum(g[i], Q, &Q, &q);
        if (q != 0.0) e[top++] = q;
    }
    e[top++] = Q;
    if (g != stackbuf) free(g);
    if (top == 1 && e[0] == 0.0) return 0;
    return top;
}

void or_exp_round(double *e, int n, double *out, int k) {
    /* After Compress the leading component is within one ulp of the whole
     * sum and the other components are exactly the remainder, so taking
     * the leading term k times yields k terms whose error is below about
     * 2^(-52 k) times the value. */
    for (int t = 0; t < k; t++) {
        n = or_exp_compress(e, n);
        if (n == 0) {
            out[t] = 0.0;
            continue;
        }
        out[t] = e[n - 1];
        n -= 1;
    }
}

/* ---- DD ----------------------------------------------------------------- */

void or_dd_add(const double *x, const double *y, double *z) {
    /* Accurate double-word + double-word (Joldes, Muller, Popescu 2017). */
    double sh, sl, th, tl, c, vh, vl, w;
    or_two_sum(x[0], y[0], &sh, &sl);
    or_two_sum(x[1], y[1], &th, &tl);
    c = sl + th;
    or_fast_two_sum(sh, c, &vh, &vl);
    w = tl + vl;
    or_fast_two_sum(vh, w, &z[0], &z[1]);
}

void or_dd_sub(const double *x, const double *y, double *z) {
    double ny[2] = {-y[0], -y[1]};
    or_dd_add(x, ny, z);
}

void or_dd_mul(const double *x, const double *y, double *z) {
    /* FMA-based double-word product (Joldes, Muller, Popescu 2017): the
     * exact product of the high parts plus the three cross terms. */
    double ch, cl1, tl0, tl1, cl2, cl3;
    or_two_prod(x[0], y[0], &ch, &cl1);
    tl0 = x[1] * y[1];
    tl1 = fma(x[0], y[1], tl0);
    cl2 = fma(x[1], y[0], tl1);
    cl3 = cl1 + cl2;
    or_fast_two_sum(ch, cl3, &z[0], &z[1]);
}

/* DD times a double, as a DD. */
static void dd_mul_d(const double *x, double b, double *z) {
    double ph, pl;
    or_two_prod(x[0], b, &ph, &pl);
    pl = fma(x[1], b, pl);
    or_fast_two_sum(ph, pl, &z[0], &z[1]);
}

void or_dd_div(const double *x, const double *y, double *z) {
    /* Long division: a quotient digit from the high parts, the remainder
     * formed in DD, and two more digits from the remainders. */
    double p[2], r[2], t[2], q3dd[2];
    double q1 = x[0] / y[0];
    dd_mul_d(y, q1, p);
    or_dd_sub(x, p, r);
    double q2 = r[0] / y[0];
    dd_mul_d(y, q2, p);
    or_dd_sub(r, p, r);
    double q3 = r[0] / y[0];
    or_fast_two_sum(q1, q2, &t[0], &t[1]);
    q3dd[0] = q3;
    q3dd[1] = 0.0;
    or_dd_add(t, q3dd, z);
}

/* ---- QD ----------------------------------------------------------------- */

void or_qd_add(const double *x, const double *y, double *z) {
    double e[9];
    int n = 0;
    for (int i = 3; i >= 0; i--) n = or_exp_grow(e, n, x[i]);
    for (int i = 3; i >= 0; i--) n = or_exp_grow(e, n, y[i]);
    or_exp_round(e, n, z, 4);
}

void or_qd_sub(const double *x, const double *y, double *z) {
    double ny[4] = {-y[0], -y[1], -y[2], -y[3]};
    or_qd_add(x, ny, z);
}

void or_qd_mul(const double *x, const double *y, double *z) {
    /* All sixteen partial products, each split exactly by TwoProd, summed
     * exactly as an expansion, then rounded to four terms. */
    double e[33];
    int n = 0;
    for (int i = 3; i >= 0; i--)
        for (int j = 3; j >= 0; j--) {
            double p, q;
            or_two_prod(x[i], y[j], &p, &q);
            n = or_exp_grow(e, n, q);
            n = or_exp_grow(e, n, p);
        }
    or_exp_round(e, n, z, 4);
}

void or_qd_div(const double *x, const double *y, double *z) {
    /* Long division: each quotient digit is the leading term of the current
     * remainder divided by y's leading term; the remainder r - q y is formed
     * exactly (the product q y as an expansion, the difference rounded to
     * four terms) and five digits are summed exactly, then rounded to four
     * terms. */
    double r[4] = {x[0], x[1], x[2], x[3]}, q[5], qy[4], qq[4];
    for (int t = 0; t < 5; t++) {
        q[t] = r[0] / y[0];
        qq[0] = q[t];
        qq[1] = qq[2] = qq[3] = 0.0;
        or_qd_mul(y, qq, qy);
        or_qd_sub(r, qy, r);
    }
    double e[6];
    int n = 0;
    for (int t = 4; t >= 0; t--) n = or_exp_grow(e, n, q[t]);
    or_exp_round(e, n, z, 4);
}
