// Device-side error-free transformations and double-double (DD) arithmetic
// for gfx950.  Everything is built from IEEE binary64 add, multiply and
// fused multiply-add with round-to-nearest; the library is compiled with
// -ffp-contract=off and this header forbids contraction as well, because a
// contracted a*b+c inside TwoSum or TwoProd silently destroys exactness.
//
// Published algorithms used:
//   TwoSum (Knuth, TAOCP vol. 2), FastTwoSum (Dekker 1971), TwoProd with one
//   FMA; the accurate double-word sum and the FMA double-word product of
//   Joldes, Muller and Popescu (ACM TOMS 2017); DD division by long
//   division with a DD remainder.
#pragma once
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace ddqd {

struct dd_t {
  double hi, lo;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  double x = a + b;
  double bv = x - a;
  double av = x - bv;
  e = (a - av) + (b - bv);
  s = x;
}

// requires a == 0 or |a| >= |b|
__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
  double x = a + b;
  e = b - (x - a);
  s = x;
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  double x = a * b;
  e = __builtin_fma(a, b, -x);
  p = x;
}

// Lazy DD multiply-add into a running pair (s, e): the product's leading
// part p = fl(a_h b_h) joins s by TwoSum; its tail err(a_h b_h) + a_h b_l +
// a_l b_h (three FMAs; a_l b_l is below 2^-106 relative and dropped) and the
// TwoSum error join e.  12 FP64 operations; callers renormalise (s, e) with
// TwoSum every few steps so that e's own rounding stays near u^2 sum |a||b|.
__device__ __forceinline__ void dd_mac(double& s, double& e, double ah, double al, double bh,
                                       double bl) {
  double p = ah * bh;
  double q = __builtin_fma(ah, bh, -p);
  q = __builtin_fma(ah, bl, q);
  q = __builtin_fma(al, bh, q);
  double t = s + p;
  double z = t - s;
  double err = (s - (t - z)) + (p - z);
  s = t;
  e = e + (err + q);
}

// accurate DD + DD, relative error about 3u^2
__device__ __forceinline__ dd_t dd_add(dd_t x, dd_t y) {
  double sh, sl, th, tl, vh, vl;
  two_sum(x.hi, y.hi, sh, sl);
  two_sum(x.lo, y.lo, th, tl);
  double c = sl + th;
  fast_two_sum(sh, c, vh, vl);
  double w = tl + vl;
  dd_t z;
  fast_two_sum(vh, w, z.hi, z.lo);
  return z;
}

__device__ __forceinline__ dd_t dd_neg(dd_t x) { return dd_t{-x.hi, -x.lo}; }

__device__ __forceinline__ dd_t dd_sub(dd_t x, dd_t y) { return dd_add(x, dd_neg(y)); }

// FMA-based DD * DD, relative error below 5u^2
__device__ __forceinline__ dd_t dd_mul(dd_t x, dd_t y) {
  double ch, cl;
  two_prod(x.hi, y.hi, ch, cl);
  double t = x.lo * y.lo;
  t = __builtin_fma(x.hi, y.lo, t);
  t = __builtin_fma(x.lo, y.hi, t);
  cl = cl + t;
  dd_t z;
  fast_two_sum(ch, cl, z.hi, z.lo);
  return z;
}

__device__ __forceinline__ dd_t dd_mul_d(dd_t x, double b) {
  double ph, pl;
  two_prod(x.hi, b, ph, pl);
  pl = __builtin_fma(x.lo, b, pl);
  dd_t z;
  fast_two_sum(ph, pl, z.hi, z.lo);
  return z;
}

// DD / DD by long division: three quotient digits from DD remainders.
__device__ __forceinline__ dd_t dd_div(dd_t x, dd_t y) {
  double q1 = x.hi / y.hi;
  dd_t r = dd_sub(x, dd_mul_d(y, q1));
  double q2 = r.hi / y.hi;
  r = dd_sub(r, dd_mul_d(y, q2));
  double q3 = r.hi / y.hi;
  dd_t q;
  fast_two_sum(q1, q2, q.hi, q.lo);
  return dd_add(q, dd_t{q3, 0.0});
}

// sign of |x| - |y|, decided in DD
__device__ __forceinline__ int dd_abs_cmp(dd_t x, dd_t y) {
  if (x.hi < 0.0) x = dd_neg(x);
  if (y.hi < 0.0) y = dd_neg(y);
  dd_t d = dd_sub(x, y);
  return (d.hi > 0.0) - (d.hi < 0.0);
}

}  // namespace ddqd
