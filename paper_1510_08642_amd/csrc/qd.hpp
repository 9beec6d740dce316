// Device-side quad-double (QD) arithmetic and the number-type traits the
// templated kernels use (DDNum: 2 planes, QDNum: 4 planes).
//
// A QD value is c0 + c1 + c2 + c3 with each term below about half an ulp of
// the one before.  Two building blocks:
//
//  * qd_add: the eight input terms are summed error-free by repeated
//    bottom-up TwoSum passes ("VecSum", Ogita, Rump and Oishi 2005); each
//    pass leaves an approximation of what remains in its first slot and the
//    exact rounding errors behind it, so four passes extract four terms; the
//    small leftover is added to the last one and the result renormalised.
//    The error is about 2^-200 (|a| + |b|) in the worst case and far smaller
//    in practice.
//
//  * qd_mac: a multiply-accumulate into four "order buckets" s0..s3, bucket k
//    holding quantities of relative size about u^k (u = 2^-53).  The product
//    terms a_i b_j with i + j <= 2 are split exactly by TwoProd and added into
//    their bucket by TwoSum, whose rounding errors move one bucket down; order
//    3 terms (and the errors that reach it) are plain FMA/adds.  Terms of
//    order >= 4 are dropped (below 2^-212 relative).  113 FP64 operations per
//    multiply-add; qd_renorm restores the bucket ordering.
#pragma once
#include "eft.hpp"

#pragma clang fp contract(off)

namespace ddqd {

struct qd_t {
  double c[4];
};

struct qd_acc {
  double s0, s1, s2, s3;
};

__device__ __forceinline__ void qd_renorm(double& c0, double& c1, double& c2, double& c3) {
  two_sum(c2, c3, c2, c3);
  two_sum(c1, c2, c1, c2);
  two_sum(c0, c1, c0, c1);
  two_sum(c1, c2, c1, c2);
  two_sum(c2, c3, c2, c3);
}

__device__ __forceinline__ qd_t qd_neg(qd_t a) {
  return qd_t{{-a.c[0], -a.c[1], -a.c[2], -a.c[3]}};
}

__device__ __forceinline__ qd_t qd_add(qd_t a, qd_t b) {
  double v[8] = {a.c[0], b.c[0], a.c[1], b.c[1], a.c[2], b.c[2], a.c[3], b.c[3]};
#pragma unroll
  for (int k = 0; k < 4; k++) {
#pragma unroll
    for (int i = 7; i > k; i--) two_sum(v[i - 1], v[i], v[i - 1], v[i]);
  }
  double tail = (v[4] + v[5]) + (v[6] + v[7]);
  qd_t z{{v[0], v[1], v[2], v[3] + tail}};
  qd_renorm(z.c[0], z.c[1], z.c[2], z.c[3]);
  return z;
}

__device__ __forceinline__ qd_t qd_sub(qd_t a, qd_t b) { return qd_add(a, qd_neg(b)); }

__device__ __forceinline__ void qd_mac(qd_acc& s, const double a[4], const double b[4]) {
  double p00, e00, p01, e01, p10, e10, p02, e02, p11, e11, p20, e20;
  two_prod(a[0], b[0], p00, e00);
  two_prod(a[0], b[1], p01, e01);
  two_prod(a[1], b[0], p10, e10);
  two_prod(a[0], b[2], p02, e02);
  two_prod(a[1], b[1], p11, e11);
  two_prod(a[2], b[0], p20, e20);
  double o3 = a[0] * b[3];
  o3 = __builtin_fma(a[1], b[2], o3);
  o3 = __builtin_fma(a[2], b[1], o3);
  o3 = __builtin_fma(a[3], b[0], o3);
  // order 0
  double r0;
  two_sum(s.s0, p00, s.s0, r0);
  // order 1: r0, e00, p01, p10
  double r1, r2, r3, r4;
  two_sum(s.s1, r0, s.s1, r1);
  two_sum(s.s1, e00, s.s1, r2);
  two_sum(s.s1, p01, s.s1, r3);
  two_sum(s.s1, p10, s.s1, r4);
  // order 2: r1..r4, e01, e10, p02, p11, p20
  double q[9];
  two_sum(s.s2, r1, s.s2, q[0]);
  two_sum(s.s2, r2, s.s2, q[1]);
  two_sum(s.s2, r3, s.s2, q[2]);
  two_sum(s.s2, r4, s.s2, q[3]);
  two_sum(s.s2, e01, s.s2, q[4]);
  two_sum(s.s2, e10, s.s2, q[5]);
  two_sum(s.s2, p02, s.s2, q[6]);
  two_sum(s.s2, p11, s.s2, q[7]);
  two_sum(s.s2, p20, s.s2, q[8]);
  // order 3
  double t3 = ((e02 + e11) + (e20 + o3)) + (((q[0] + q[1]) + (q[2] + q[3])) +
                                             ((q[4] + q[5]) + (q[6] + q[7]) + q[8]));
  s.s3 = s.s3 + t3;
}

__device__ __forceinline__ qd_t qd_mul(qd_t a, qd_t b) {
  qd_acc s{0.0, 0.0, 0.0, 0.0};
  qd_mac(s, a.c, b.c);
  qd_renorm(s.s0, s.s1, s.s2, s.s3);
  return qd_t{{s.s0, s.s1, s.s2, s.s3}};
}

// ---- number-type traits for templated kernels ------------------------------

struct DDNum {
  static constexpr int P = 2;
  using T = dd_t;
  __device__ static T load(const double* p, int64_t ps, int64_t idx) {
    return T{p[idx], p[ps + idx]};
  }
  __device__ static void store(double* p, int64_t ps, int64_t idx, T v) {
    p[idx] = v.hi;
    p[ps + idx] = v.lo;
  }
  __device__ static T add(T a, T b) { return dd_add(a, b); }
  __device__ static T sub(T a, T b) { return dd_sub(a, b); }
  __device__ static T neg(T a) { return dd_neg(a); }
  __device__ static T scale(T a, int e) { return T{ldexp(a.hi, e), ldexp(a.lo, e)}; }
};

struct QDNum {
  static constexpr int P = 4;
  using T = qd_t;
  __device__ static T load(const double* p, int64_t ps, int64_t idx) {
    return T{{p[idx], p[ps + idx], p[2 * ps + idx], p[3 * ps + idx]}};
  }
  __device__ static void store(double* p, int64_t ps, int64_t idx, T v) {
    p[idx] = v.c[0];
    p[ps + idx] = v.c[1];
    p[2 * ps + idx] = v.c[2];
    p[3 * ps + idx] = v.c[3];
  }
  __device__ static T add(T a, T b) { return qd_add(a, b); }
  __device__ static T sub(T a, T b) { return qd_sub(a, b); }
  __device__ static T neg(T a) { return qd_neg(a); }
  __device__ static T scale(T a, int e) {
    return T{{ldexp(a.c[0], e), ldexp(a.c[1], e), ldexp(a.c[2], e), ldexp(a.c[3], e)}};
  }
};

}  // namespace ddqd
