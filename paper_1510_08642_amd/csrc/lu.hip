// LU kernels in DD and QD: the narrow-panel factorisation (getf2), row
// interchanges (laswp), small triangular solves, thin panel products, and the
// blocked triangular solves of getrs.  The blocked right-looking driver that
// strings them together with the matrix product lives in lu_driver.hip.
//
// Paper: Sec. 4, steps 1-3 (factor A11, form U12 and L21, update A22 with a
// matrix product) and Eq. 2 (solve Ax = b); the paper runs the LU in DD and
// in QD.  Partial pivoting (largest |a_ic|, first index on ties, decided in
// the working precision) is an option the paper, which factors without
// pivoting, does not use.
//
// Every kernel is written once over LuArith<P> (P = 2 for DD, 4 for QD): the
// value type, its operations, and an accumulator for x - sum_k a_k b_k.  DD
// accumulates lazily (TwoSum of the high product into one word, the low
// parts and the TwoSum errors into a second, one rounding at the end); QD
// uses the order-bucket multiply-add of qd.hpp.
#include "common.hpp"
#include "ddqd.h"
#include "eft.hpp"
#include "qd.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

template <int P>
struct LuArith;

template <>
struct LuArith<2> {
  using T = dd_t;
  static constexpr int P = 2;
  struct Acc {
    double w[2];
  };
  __device__ static double get(const T& x, int c) { return c == 0 ? x.hi : x.lo; }
  __device__ static void put(T& x, int c, double v) {
    if (c == 0)
      x.hi = v;
    else
      x.lo = v;
  }
  __device__ static T zero() { return T{0.0, 0.0}; }
  __device__ static T one() { return T{1.0, 0.0}; }
  __device__ static bool is_zero(const T& x) { return x.hi == 0.0 && x.lo == 0.0; }
  __device__ static T abs(T x) { return x.hi < 0.0 ? dd_neg(x) : x; }
  // bound on |x - leading term|
  __device__ static double tail(const T& x) { return fabs(x.lo); }
  __device__ static int abs_cmp(T x, T y) { return dd_abs_cmp(x, y); }
  __device__ static T add(T a, T b) { return dd_add(a, b); }
  __device__ static T sub(T a, T b) { return dd_sub(a, b); }
  __device__ static T mul(T a, T b) { return dd_mul(a, b); }
  __device__ static T div(T a, T b) { return dd_div(a, b); }
  // x / y by three long-division digits, each the leading remainder times an
  // FP64 reciprocal of y.hi shared by the whole column (a digit may be off by
  // an ulp; the next remainder, formed in DD, absorbs it).
  __device__ static T div_digits(T x, T y, double yinv) {
    const double q1 = x.hi * yinv;
    dd_t r = dd_sub(x, dd_mul_d(y, q1));
    const double q2 = r.hi * yinv;
    r = dd_sub(r, dd_mul_d(y, q2));
    const double q3 = r.hi * yinv;
    dd_t q;
    fast_two_sum(q1, q2, q.hi, q.lo);
    return dd_add(q, dd_t{q3, 0.0});
  }
  // 1 / y: the FP64 reciprocal x0 of y.hi refined by one Newton step,
  // x0 + x0 (1 - y x0), the residual 1 - y x0 formed by two FMAs (relative
  // error about 2^-104)
  __device__ static T recip(T y) {
    const double x0 = 1.0 / y.hi;
    double e = fma(-y.hi, x0, 1.0);
    e = fma(-y.lo, x0, e);
    T x;
    fast_two_sum(x0, x0 * e, x.hi, x.lo);
    return x;
  }
  __device__ static Acc acc(T x) { return Acc{{x.hi, x.lo}}; }
  // a -= p q
  __device__ static void acc_sub(Acc& a, T p, T q) {
    const double h = p.hi * q.hi;
    const double e = fma(p.hi, q.lo, fma(p.lo, q.hi, fma(p.hi, q.hi, -h)));
    double t;
    two_sum(a.w[0], -h, a.w[0], t);
    a.w[1] += t - e;
  }
  __device__ static T value(const Acc& a) {
    T v;
    two_sum(a.w[0], a.w[1], v.hi, v.lo);
    return v;
  }
  // the same accumulation kept in a number's registers: x -= p q leaves x
  // as an unnormalised pair (sum, error); norm() restores a DD
  __device__ static void lazy_sub(T& x, T p, T q) {
    Acc a{{x.hi, x.lo}};
    acc_sub(a, p, q);
    x.hi = a.w[0];
    x.lo = a.w[1];
  }
  __device__ static T norm(T x) { return value(Acc{{x.hi, x.lo}}); }
};

template <>
struct LuArith<4> {
  using T = qd_t;
  static constexpr int P = 4;
  struct Acc {
    double w[4];
  };
  __device__ static double get(const T& x, int c) { return x.c[c]; }
  __device__ static void put(T& x, int c, double v) { x.c[c] = v; }
  __device__ static T zero() { return T{{0.0, 0.0, 0.0, 0.0}}; }
  __device__ static T one() { return T{{1.0, 0.0, 0.0, 0.0}}; }
  __device__ static bool is_zero(const T& x) {
    return x.c[0] == 0.0 && x.c[1] == 0.0 && x.c[2] == 0.0 && x.c[3] == 0.0;
  }
  __device__ static T abs(T x) { return x.c[0] < 0.0 ? qd_neg(x) : x; }
  __device__ static double tail(const T& x) {
    return fabs(x.c[1]) + fabs(x.c[2]) + fabs(x.c[3]);
  }
  __device__ static int abs_cmp(T x, T y) {
    const qd_t d = qd_sub(abs(x), abs(y));
    return (d.c[0] > 0.0) - (d.c[0] < 0.0);
  }
  __device__ static T add(T a, T b) { return qd_add(a, b); }
  __device__ static T sub(T a, T b) { return qd_sub(a, b); }
  __device__ static T mul(T a, T b) { return qd_mul(a, b); }
  __device__ static T mul_d(T a, double q) { return qd_mul(a, T{{q, 0.0, 0.0, 0.0}}); }
  // x / y by five long-division digits, each the leading term of the
  // remainder times a reciprocal of y's leading term; the remainders and the
  // sum of the digits are formed in QD.
  __device__ static T div_digits(T x, T y, double yinv) {
    qd_t r = x, q = zero();
#pragma unroll
    for (int t = 0; t < 5; t++) {
      const double d = r.c[0] * yinv;
      r = qd_sub(r, mul_d(y, d));
      q = qd_add(q, T{{d, 0.0, 0.0, 0.0}});
    }
    return q;
  }
  __device__ static T div(T a, T b) { return div_digits(a, b, 1.0 / b.c[0]); }
  // 1 / y: the DD reciprocal of y's two leading terms (as LuArith<2>),
  // then one Newton step x + x (1 - y x) in QD (relative error about 2^-207)
  __device__ static T recip(T y) {
    const double x0 = 1.0 / y.c[0];
    double e = fma(-y.c[0], x0, 1.0);
    e = fma(-y.c[1], x0, e);
    T x{{0.0, 0.0, 0.0, 0.0}};
    fast_two_sum(x0, x0 * e, x.c[0], x.c[1]);
    const T r = qd_sub(one(), qd_mul(y, x));
    return qd_add(x, qd_mul(x, r));
  }
  __device__ static Acc acc(T x) { return Acc{{x.c[0], x.c[1], x.c[2], x.c[3]}}; }
  // a -= p q
  __device__ static void acc_sub(Acc& a, T p, T q) {
    qd_acc s{a.w[0], a.w[1], a.w[2], a.w[3]};
    const double np[4] = {-p.c[0], -p.c[1], -p.c[2], -p.c[3]};
    qd_mac(s, np, q.c);
    a.w[0] = s.s0;
    a.w[1] = s.s1;
    a.w[2] = s.s2;
    a.w[3] = s.s3;
  }
  __device__ static T value(const Acc& a) {
    T v{{a.w[0], a.w[1], a.w[2], a.w[3]}};
    qd_renorm(v.c[0], v.c[1], v.c[2], v.c[3]);
    return v;
  }
  // the same accumulation kept in a number's registers (order buckets);
  // norm() restores a QD
  __device__ static void lazy_sub(T& x, T p, T q) {
    Acc a{{x.c[0], x.c[1], x.c[2], x.c[3]}};
    acc_sub(a, p, q);
#pragma unroll
    for (int c = 0; c < 4; c++) x.c[c] = a.w[c];
  }
  __device__ static T norm(T x) { return value(Acc{{x.c[0], x.c[1], x.c[2], x.c[3]}}); }
};

template <int P>
__device__ __forceinline__ typename LuArith<P>::T ld_num(const double* A, int64_t ps,
                                                         int64_t idx) {
  typename LuArith<P>::T v;
#pragma unroll
  for (int c = 0; c < P; c++) LuArith<P>::put(v, c, A[c * ps + idx]);
  return v;
}
template <int P>
__device__ __forceinline__ void st_num(double* A, int64_t ps, int64_t idx,
                                       const typename LuArith<P>::T& v) {
#pragma unroll
  for (int c = 0; c < P; c++) A[c * ps + idx] = LuArith<P>::get(v, c);
}

// (x, i) beats (y, j): larger |value|; on equal values the smaller row index.
// i < 0 marks "no candidate".  The leading terms decide when they differ by
// more than the trailing terms can make up (their difference is exact when
// they are within a factor 2, and far larger than the tails otherwise); only
// near-ties take the full comparison in the working precision.
template <int P>
__device__ __forceinline__ bool better(const typename LuArith<P>::T& x, int i,
                                       const typename LuArith<P>::T& y, int j) {
  using N = LuArith<P>;
  if (i < 0) return false;
  if (j < 0) return true;
  const double dh = fabs(N::get(x, 0)) - fabs(N::get(y, 0));
  const double lim = 2.0 * (N::tail(x) + N::tail(y));
  if (dh > lim) return true;
  if (-dh > lim) return false;
  const int c = N::abs_cmp(x, y);
  return c > 0 || (c == 0 && i < j);
}

// DPP lane exchange of a 64-bit value inside rows of 16 lanes.
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, kCtrl, 0xF, 0xF,
                                                            false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), kCtrl,
                                                            0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
template <int kCtrl>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xF, 0xF, false);
}
// lane i <- lane i^1, i^2 (quad permutes), 7-i and 15-i within the row
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int P, int kCtrl>
__device__ __forceinline__ void argmax_step_dpp(typename LuArith<P>::T& b, int& bi, int& tag) {
  using N = LuArith<P>;
  typename N::T o;
#pragma unroll
  for (int c = 0; c < P; c++) N::put(o, c, dpp_f64<kCtrl>(N::get(b, c)));
  const int oi = dpp_i32<kCtrl>(bi), ot = dpp_i32<kCtrl>(tag);
  if (better<P>(o, oi, b, bi)) {
    b = o;
    bi = oi;
    tag = ot;
  }
}
template <int P>
__device__ __forceinline__ void argmax_step_shfl(typename LuArith<P>::T& b, int& bi, int& tag,
                                                 int off) {
  using N = LuArith<P>;
  typename N::T o;
#pragma unroll
  for (int c = 0; c < P; c++) N::put(o, c, __shfl_xor(N::get(b, c), off, 64));
  const int oi = __shfl_xor(bi, off, 64), ot = __shfl_xor(tag, off, 64);
  if (better<P>(o, oi, b, bi)) {
    b = o;
    bi = oi;
    tag = ot;
  }
}
// after the four steps every lane of a 16-lane row holds the row's best
template <int P>
__device__ __forceinline__ void argmax_row16(typename LuArith<P>::T& b, int& bi, int& tag) {
  argmax_step_dpp<P, kDppXor1>(b, bi, tag);
  argmax_step_dpp<P, kDppXor2>(b, bi, tag);
  argmax_step_dpp<P, kDppHalfMirror>(b, bi, tag);
  argmax_step_dpp<P, kDppMirror>(b, bi, tag);
}
__device__ __forceinline__ double row16_max(double x) {
  x = fmax(x, dpp_f64<kDppXor1>(x));
  x = fmax(x, dpp_f64<kDppXor2>(x));
  x = fmax(x, dpp_f64<kDppHalfMirror>(x));
  return fmax(x, dpp_f64<kDppMirror>(x));
}

__device__ __forceinline__ double readlane_f64(double v, int k) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), k);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int P>
__device__ __forceinline__ typename LuArith<P>::T readlane_num(const typename LuArith<P>::T& v,
                                                               int k) {
  typename LuArith<P>::T r;
#pragma unroll
  for (int c = 0; c < P; c++) LuArith<P>::put(r, c, readlane_f64(LuArith<P>::get(v, c), k));
  return r;
}
// lane k's accumulator as a number, in every lane, for a triangular solve's
// next step.  DD: the pair (w0, w1) as it is, unnormalised (its sum is the
// value; a product with it drops only the low word's cross term with the
// other factor's low part, which leaves it accurate relative to the partial
// sums), keeping the normalisation off the step-to-step chain.  QD: the
// normalised value (a product reads the components as terms of decreasing
// order).
template <int P>
__device__ __forceinline__ typename LuArith<P>::T readlane_words(const typename LuArith<P>::Acc& a,
                                                                 int k);
template <int P>
__device__ __forceinline__ typename LuArith<P>::T readlane_acc(const typename LuArith<P>::Acc& a,
                                                               int k);
template <>
__device__ __forceinline__ dd_t readlane_words<2>(const LuArith<2>::Acc& a, int k) {
  return dd_t{readlane_f64(a.w[0], k), readlane_f64(a.w[1], k)};
}
template <>
__device__ __forceinline__ qd_t readlane_words<4>(const LuArith<4>::Acc& a, int k) {
  return readlane_acc<4>(a, k);
}
// the value held by lane k's accumulator, in every lane
template <int P>
__device__ __forceinline__ typename LuArith<P>::T readlane_acc(const typename LuArith<P>::Acc& a,
                                                               int k) {
  typename LuArith<P>::Acc r;
#pragma unroll
  for (int c = 0; c < P; c++) r.w[c] = readlane_f64(a.w[c], k);
  return LuArith<P>::value(r);
}

// The lane holding the best candidate of a wave (largest |x|, then the
// smallest index; idx < 0 marks "no candidate"), the same in every lane, or
// -1 if no lane has one.  The FP64 maximum M of the leading terms finds the
// leader.  Candidates are normalized, so the trailing terms of each add at
// most about 2^-52 of its leading term (or a few units of the smallest
// subnormal): a lane can equal or beat the leader only if its leading term is
// within 2^-48 M + 2^-1060 of M, and when that holds for one lane alone it is
// the winner.  Otherwise the comparison in the working precision decides
// among those lanes.  kRow0: candidates only in lanes 0..15.
template <int P, bool kRow0>
__device__ __forceinline__ int wave_argmax(const typename LuArith<P>::T& x, int idx) {
  using N = LuArith<P>;
  const int lane = threadIdx.x % 64;
  const bool valid = idx >= 0;
  const double h = valid ? fabs(N::get(x, 0)) : -1.0;
  double M = row16_max(h);
  if (kRow0) {
    M = readlane_f64(M, 0);
  } else {
    M = fmax(fmax(readlane_f64(M, 0), readlane_f64(M, 16)),
             fmax(readlane_f64(M, 32), readlane_f64(M, 48)));
  }
  if (!(M >= 0.0)) return -1;
  const bool close = valid && (M - h) <= 0x1p-48 * M + 0x1p-1060;
  const uint64_t mask = __ballot(close);
  if (__popcll(mask) == 1) return __ffsll((unsigned long long)mask) - 1;
  typename N::T b = close ? x : N::zero();
  int bi = close ? idx : -1, tag = lane;
  argmax_row16<P>(b, bi, tag);
  if (!kRow0) {
    argmax_step_shfl<P>(b, bi, tag, 16);
    argmax_step_shfl<P>(b, bi, tag, 32);
  }
  return __builtin_amdgcn_readlane(tag, 0);
}

typedef double f64x2 __attribute__((ext_vector_type(2)));  // one 16-byte access

// ---- getf2: factor an m x w strip (w <= W) held in registers ---------------
// One workgroup of T threads; thread t owns local rows t + T q, q < RPT.
// The strip moves between HBM and registers through an LDS tile, so that
// global accesses run along the rows (coalesced); a full-width strip moves in
// 16-byte chunks with all of a thread's loads in flight before the first is
// used.
// Column c, with one barrier:
//   1. every wave finds its best candidate |a_ic| (rows i >= c; compared in
//      the working precision, ties to the smaller row; see wave_argmax); it publishes the value, the
//      row index and the winning row's W values, and the owner of row c
//      publishes row c;
//   2. after the barrier every wave reduces the wave winners itself and reads
//      the pivot row p from the winning wave's slot; the owners of rows c and
//      p exchange them in registers;
//   3. the column below the pivot is multiplied by the pivot's reciprocal
//      (formed once per column by a Newton step) and the remaining strip
//      columns get the rank-1 update, accumulated lazily in the numbers'
//      own registers (as the products' accumulators: at most W - 1 updates
//      before a column is normalised at the start of its own step; rows
//      are normalised when published).
// The published slots are double-buffered by the parity of c: a slot is
// rewritten two columns later, after a barrier that every reader of its old
// contents has passed.
// ipiv[c0 + c] receives the global (0-based) pivot row; info the first
// 1-based global column whose pivot is exactly zero, if none was recorded
// before.  Other columns of the matrix are interchanged later by laswp.

template <int P, int T, int RPT, int W>
__global__ __launch_bounds__(T) void getf2_kernel(double* A, int64_t lda, int64_t ps,
                                                   int64_t r0, int64_t m, int64_t c0, int w,
                                                   int32_t* ipiv, int32_t* info, int pivot) {
  constexpr int kLd = W + 2;  // padded LDS row of the staging tile (16-byte rows)
  constexpr int kH = W >= 2 ? W / 2 : 1;  // 16-byte chunks in a full strip row
  constexpr int kWaves = T / 64;
  static_assert(kWaves == 4 || kWaves == 8 || kWaves == 16, "T must be 256, 512 or 1024");
  __shared__ __align__(16) double tile[T * kLd];
  using N = LuArith<P>;
  using V = typename N::T;
  __shared__ double s_val[2][kWaves][P];
  __shared__ int s_idx[2][kWaves];
  __shared__ double s_row[2][kWaves][P][W];
  __shared__ double s_rowc[2][P][W];
  const int t = threadIdx.x, lane = t % 64, wave = t / 64;
  V v[RPT][W];
  // Full-width strips whose rows start on 16 bytes move in 16-byte chunks,
  // with the loads of every row block and plane in flight at once; other
  // strips (the last, narrower one of a panel; odd offsets) by 8-byte words,
  // one row block at a time.
  const bool vec = W % 2 == 0 && w == W && ((lda | ps | c0) & 1) == 0 &&
                   ((uintptr_t)A & 15) == 0;
  if (vec) {
    f64x2 xs[RPT][P][kH];
#pragma unroll
    for (int q = 0; q < RPT; q++) {
#pragma unroll
      for (int j = 0; j < kH; j++) {
        // rows past the strip re-read its last row (the values are not used)
        const int e = t + T * j, k2 = e % kH;
        const int64_t row = min((int64_t)T * q + e / kH, m - 1);
        const double* src = A + (r0 + row) * lda + c0 + 2 * k2;
#pragma unroll
        for (int c = 0; c < P; c++) xs[q][c][j] = *(const f64x2*)(src + c * ps);
      }
    }
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int64_t rows = min((int64_t)T, m - (int64_t)T * q);
      if (rows <= 0) {
#pragma unroll
        for (int k = 0; k < W; k++) v[q][k] = N::zero();
        continue;
      }
#pragma unroll
      for (int plane = 0; plane < P; plane++) {
#pragma unroll
        for (int j = 0; j < kH; j++) {
          const int e = t + T * j, r = e / kH, k2 = e % kH;
          if (r < rows) *(f64x2*)&tile[r * kLd + 2 * k2] = xs[q][plane][j];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < W; k++) N::put(v[q][k], plane, t < rows ? tile[t * kLd + k] : 0.0);
        __syncthreads();
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int64_t rows = min((int64_t)T, m - (int64_t)T * q);
      if (rows <= 0) {
#pragma unroll
        for (int k = 0; k < W; k++) v[q][k] = N::zero();
        continue;
      }
      const int n = (int)rows * w;
      const double* src = A + (r0 + (int64_t)T * q) * lda + c0;
      double xs[P][W];
#pragma unroll
      for (int j = 0; j < W; j++) {  // every load in flight before the first use
        const int e = min(t + T * j, n - 1), r = e / w, k = e - r * w;
#pragma unroll
        for (int c = 0; c < P; c++) xs[c][j] = src[c * ps + (int64_t)r * lda + k];
      }
#pragma unroll
      for (int plane = 0; plane < P; plane++) {
#pragma unroll
        for (int j = 0; j < W; j++) {
          const int e = t + T * j, r = e / w, k = e - r * w;
          if (e < n) tile[r * kLd + k] = xs[plane][j];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < W; k++)
          N::put(v[q][k], plane, (t < rows && k < w) ? tile[t * kLd + k] : 0.0);
        __syncthreads();
      }
    }
  }
  // The column loop is unrolled so that every register index is a constant.
#pragma unroll
  for (int c = 0; c < W; c++) {
    if (c >= w) break;
    const int buf = c & 1;
    // column c has received all its updates (kept unnormalised, see 3.)
#pragma unroll
    for (int q = 0; q < RPT; q++) v[q][c] = N::norm(v[q][c]);
    // 1. wave-local pivot search among local rows >= c
    V best = N::zero();
    int bi = -1;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int i = t + T * q;
      if (i >= c && i < m) {
        const V x = N::abs(v[q][c]);
        if (better<P>(x, i, best, bi)) {
          best = x;
          bi = i;
        }
      }
    }
    const int wl = wave_argmax<P, false>(best, bi);
    // the winning lane publishes its own candidate (lane 0 "none" if no lane
    // has one)
    if (lane == (wl >= 0 ? wl : 0)) {
#pragma unroll
      for (int cc = 0; cc < P; cc++) s_val[buf][wave][cc] = wl >= 0 ? N::get(best, cc) : 0.0;
      s_idx[buf][wave] = wl >= 0 ? bi : -1;
    }
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int i = t + T * q;
      // columns before c hold multipliers and column c was normalized at the
      // start of this step; only the lazily updated columns after c need it
      if (lane == wl && i == bi)
#pragma unroll
        for (int k = 0; k < W; k++) {
          const V x = k > c ? N::norm(v[q][k]) : v[q][k];
#pragma unroll
          for (int cc = 0; cc < P; cc++) s_row[buf][wave][cc][k] = N::get(x, cc);
        }
      if (i == c)
#pragma unroll
        for (int k = 0; k < W; k++) {
          const V x = k > c ? N::norm(v[q][k]) : v[q][k];
#pragma unroll
          for (int cc = 0; cc < P; cc++) s_rowc[buf][cc][k] = N::get(x, cc);
        }
    }
    __syncthreads();
    // 2. the winners of all waves, reduced by every wave
    V b = N::zero();
    int pi = -1;
    if (lane < kWaves) {
#pragma unroll
      for (int cc = 0; cc < P; cc++) N::put(b, cc, s_val[buf][lane][cc]);
      pi = s_idx[buf][lane];
    }
    const int wv = wave_argmax<P, true>(b, pi);
    int p = wv >= 0 ? __builtin_amdgcn_readlane(pi, wv) : -1;
    const bool use_c = !pivot || p < 0;
    if (use_c) p = c;
    // the pivot row's values (P planes of W) and row c's
    const double* rp = use_c ? &s_rowc[buf][0][0] : &s_row[buf][wv][0][0];
    auto rpv = [&](int k) {
      V r;
#pragma unroll
      for (int cc = 0; cc < P; cc++) N::put(r, cc, rp[cc * W + k]);
      return r;
    };
    auto rcv = [&](int k) {
      V r;
#pragma unroll
      for (int cc = 0; cc < P; cc++) N::put(r, cc, s_rowc[buf][cc][k]);
      return r;
    };
    if (t == 0) ipiv[c0 + c] = (int32_t)(r0 + p);
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int i = t + T * q;
      if (i == c) {
#pragma unroll
        for (int k = 0; k < W; k++) v[q][k] = rpv(k);
      } else if (i == p) {
#pragma unroll
        for (int k = 0; k < W; k++) v[q][k] = rcv(k);
      }
    }
    // 3. division by the pivot and rank-1 update of the strip
    const V u = rpv(c);
    if (t == 0 && N::is_zero(u) && *info == 0) *info = (int32_t)(c0 + c + 1);
    if (!N::is_zero(u)) {
      // multipliers by the pivot's reciprocal (one reciprocal per column, as
      // LAPACK scales the column); long division where 1 / u.hi would leave
      // the normal range
      const bool by_recip = fabs(N::get(u, 0)) >= 0x1p-1000;
      const V uinv = by_recip ? N::recip(u) : N::zero();
      const double uinv0 = 1.0 / N::get(u, 0);
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const int i = t + T * q;
        if (i > c && i < m) {
          const V l = by_recip ? N::mul(v[q][c], uinv) : N::div_digits(v[q][c], u, uinv0);
          v[q][c] = l;
#pragma unroll
          for (int k = c + 1; k < W; k++)
            if (k < w) N::lazy_sub(v[q][k], l, rpv(k));
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RPT; q++) {
    const int64_t rows = min((int64_t)T, m - (int64_t)T * q);
    if (rows <= 0) continue;
    const int n = (int)rows * w;
    double* dst = A + (r0 + (int64_t)T * q) * lda + c0;
#pragma unroll
    for (int plane = 0; plane < P; plane++) {
      __syncthreads();  // the tile's previous readers are done
      if (t < rows)
#pragma unroll
        for (int k = 0; k < W; k++) tile[t * kLd + k] = N::get(v[q][k], plane);
      __syncthreads();
      if (vec) {
#pragma unroll
        for (int j = 0; j < kH; j++) {
          const int e = t + T * j, r = e / kH, k2 = e % kH;
          if (r < rows)
            *(f64x2*)(dst + plane * ps + (int64_t)r * lda + 2 * k2) =
                *(const f64x2*)&tile[r * kLd + 2 * k2];
        }
      } else {
#pragma unroll
        for (int j = 0; j < W; j++) {
          const int e = t + T * j, r = e / w, k = e - r * w;
          if (e < n) dst[plane * ps + (int64_t)r * lda + k] = tile[r * kLd + k];
        }
      }
    }
  }
}

// ---- laswp: rows k <-> ipiv[k] for k in [k0, k1), in order ------------------
// One thread per column (coalesced across threads), all P planes, columns
// [skip0, skip1) excluded; thread n_cols applies the same interchanges to
// perm (if given).
__global__ __launch_bounds__(256) void laswp_kernel(double* A, int64_t lda, int64_t ps, int P,
                                                    int64_t n_cols, int64_t skip0, int64_t skip1,
                                                    int64_t k0, int64_t k1, const int32_t* ipiv,
                                                    int32_t* perm) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j > n_cols || (j >= skip0 && j < skip1)) return;
  if (j == n_cols) {
    if (!perm) return;
    for (int64_t k = k0; k < k1; k++) {
      const int64_t p = ipiv[k];
      if (p != k) {
        const int32_t x = perm[k];
        perm[k] = perm[p];
        perm[p] = x;
      }
    }
    return;
  }
  for (int64_t k = k0; k < k1; k++) {
    const int64_t p = ipiv[k];
    if (p != k) {
      const int64_t a = k * lda + j, b = p * lda + j;
      for (int c = 0; c < P; c++) {
        const double h = A[c * ps + a];
        A[c * ps + a] = A[c * ps + b];
        A[c * ps + b] = h;
      }
    }
  }
}

// ---- C -= A B for the thin products inside the panel ------------------------
// A (m x l), B (l x n), C (m x n) are blocks of one plane-layout matrix (same
// ld and plane stride).  One thread per entry of C, accumulated from C's
// value down (LuArith<P>::Acc).
template <int P>
__global__ __launch_bounds__(256) void lu_update_kernel(const double* A, const double* B,
                                                        double* C, int64_t ld, int64_t ps,
                                                        int64_t m, int64_t n, int64_t l) {
  using N = LuArith<P>;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e / n, j = e - i * n;
  typename N::Acc acc = N::acc(ld_num<P>(C, ps, i * ld + j));
  int64_t k = 0;
  // U k at a time with every load in flight before the first product
  constexpr int U = P == 2 ? 8 : 4;
  for (; k + U <= l; k += U) {
    typename N::T a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      a[u] = ld_num<P>(A, ps, i * ld + k + u);
      b[u] = ld_num<P>(B, ps, (k + u) * ld + j);
    }
#pragma unroll
    for (int u = 0; u < U; u++) N::acc_sub(acc, a[u], b[u]);
  }
  for (; k < l; k++) N::acc_sub(acc, ld_num<P>(A, ps, i * ld + k), ld_num<P>(B, ps, k * ld + j));
  st_num<P>(C, ps, i * ld + j, N::value(acc));
}

// ---- unit-lower triangular solve with one wave per column: X := L^-1 X -----
// L = A[r0 .. r0+nb, c0 .. c0+nb) (unit diagonal, nb <= R), X = the nb rows
// r0.. of columns [x0, x0 + ncols).  Lane i of a wave holds x_i of one column
// as an accumulator; step k finishes x_k, broadcasts it with readlane, and
// the lanes below subtract L_ik x_k (forward substitution, one rounding per
// unknown).  A workgroup takes up to 16 adjacent columns, staging L
// (transposed, so a step reads one LDS row) and its X tile through LDS so
// that global accesses run along the rows.  R = 64 for DD, 32 for QD (LDS).
constexpr int kTrsmCols = 16;
template <int P>
constexpr int trsm_rows() {
  return P == 2 ? 64 : 32;
}

// Stages L and the X tile of columns [x0 + j0, x0 + j0 + nc) in LDS and solves
// (waves < nc, one column each); Xs then holds X = L^-1 X.
template <int P>
__device__ __forceinline__ void trsm_tile(const double* A, int64_t lda, int64_t ps, int64_t r0,
                                          int64_t c0, int nb, int64_t x0, int64_t j0, int nc,
                                          double (&Ls)[P][trsm_rows<P>()][trsm_rows<P>() + 1],
                                          double (&Xs)[P][trsm_rows<P>()][kTrsmCols + 1]) {
  using N = LuArith<P>;
  const int t = threadIdx.x, lane = t % 64, wave = t / 64, nt = blockDim.x;
  // L and X tiles, eight elements per thread in flight at a time
  for (int e0 = t; e0 < nb * nb; e0 += 8 * nt) {
    double x[8][P];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int e = min(e0 + u * nt, nb * nb - 1), i = e / nb, k = e - i * nb;
#pragma unroll
      for (int c = 0; c < P; c++) x[u][c] = A[c * ps + (r0 + i) * lda + c0 + k];
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int e = e0 + u * nt, i = e / nb, k = e - i * nb;
      if (e < nb * nb)
#pragma unroll
        for (int c = 0; c < P; c++) Ls[c][k][i] = x[u][c];
    }
  }
  for (int e0 = t; e0 < nb * nc; e0 += 8 * nt) {
    double x[8][P];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int e = min(e0 + u * nt, nb * nc - 1), i = e / nc, cc = e - i * nc;
#pragma unroll
      for (int c = 0; c < P; c++) x[u][c] = A[c * ps + (r0 + i) * lda + x0 + j0 + cc];
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int e = e0 + u * nt, i = e / nc, cc = e - i * nc;
      if (e < nb * nc)
#pragma unroll
        for (int c = 0; c < P; c++) Xs[c][i][cc] = x[u][c];
    }
  }
  __syncthreads();
  if (wave < nc) {
    typename N::T xin = N::zero();
    if (lane < nb)
#pragma unroll
      for (int c = 0; c < P; c++) N::put(xin, c, Xs[c][lane][wave]);
    typename N::Acc acc = N::acc(xin);
    for (int k = 0; k < nb - 1; k++) {
      const typename N::T xk = readlane_acc<P>(acc, k);
      if (lane > k && lane < nb) {
        typename N::T lk;
#pragma unroll
        for (int c = 0; c < P; c++) N::put(lk, c, Ls[c][k][lane]);
        N::acc_sub(acc, lk, xk);
      }
    }
    if (lane < nb) {
      const typename N::T x = N::value(acc);
#pragma unroll
      for (int c = 0; c < P; c++) Xs[c][lane][wave] = N::get(x, c);
    }
  }
  __syncthreads();
}

template <int P>
__device__ __forceinline__ void store_x_tile(double* A, int64_t lda, int64_t ps, int64_t r0,
                                             int nb, int64_t x0, int64_t j0, int nc,
                                             const double (&Xs)[P][trsm_rows<P>()]
                                                                [kTrsmCols + 1]) {
  for (int e = threadIdx.x; e < nb * nc; e += blockDim.x) {
    const int i = e / nc, cc = e - i * nc;
#pragma unroll
    for (int c = 0; c < P; c++) A[c * ps + (r0 + i) * lda + x0 + j0 + cc] = Xs[c][i][cc];
  }
}

template <int P>
__global__ __launch_bounds__(1024) void trsm_wave_kernel(double* A, int64_t lda, int64_t ps,
                                                         int64_t r0, int64_t c0, int nb,
                                                         int64_t x0, int64_t ncols) {
  constexpr int R = trsm_rows<P>();
  __shared__ double Ls[P][R][R + 1];
  __shared__ double Xs[P][R][kTrsmCols + 1];
  const int cpb = blockDim.x / 64;  // columns per workgroup
  const int64_t j0 = (int64_t)blockIdx.x * cpb;
  const int nc = (int)min((int64_t)cpb, ncols - j0);
  trsm_tile<P>(A, lda, ps, r0, c0, nb, x0, j0, nc, Ls, Xs);
  store_x_tile<P>(A, lda, ps, r0, nb, x0, j0, nc, Xs);
}

// ---- the solve and the thin product of one panel step in one launch --------
// X := L^-1 X as trsm_wave_kernel (L at (r0, r0), nb <= R rows, columns
// [x0, x0 + ncols)), then rows [r0 + nb, r0 + nb + mb) of the same columns
// -= A[those rows, r0 .. r0 + nb) X, each entry accumulated from its value
// down with k ascending, as lu_update_kernel does (the same values as the
// two launches, bit for bit).  Workgroup (g, h) takes column group g and the
// kTrsmUpdRows rows of block h; every row block solves its group's X itself in
// LDS from the unsolved values in A (the solve is small and saves a launch and
// the trip of X through memory).  X is not stored here: a row block could
// still be reading the unsolved values.  Inside a panel nothing else reads
// those rows of those columns (later interchanges only move rows below them),
// so trsm_nodes_kernel solves and stores the X of all such steps of a panel
// once the panel is factored.
constexpr int kTrsmUpdRows = 32;

template <int P>
__global__ __launch_bounds__(1024) void trsm_update_kernel(double* A, int64_t lda, int64_t ps,
                                                           int64_t r0, int nb, int64_t x0,
                                                           int64_t ncols, int64_t mb) {
  using N = LuArith<P>;
  constexpr int R = trsm_rows<P>();
  __shared__ double Ls[P][R][R + 1];
  __shared__ double Xs[P][R][kTrsmCols + 1];
  const int cpb = blockDim.x / 64;
  const int64_t j0 = (int64_t)blockIdx.x * cpb;
  const int nc = (int)min((int64_t)cpb, ncols - j0);
  trsm_tile<P>(A, lda, ps, r0, r0, nb, x0, j0, nc, Ls, Xs);
  const int64_t i0 = r0 + nb + (int64_t)blockIdx.y * kTrsmUpdRows;
  const int64_t rows = min((int64_t)kTrsmUpdRows, r0 + nb + mb - i0);
  constexpr int U = P == 2 ? 8 : 4;
  for (int e = threadIdx.x; e < rows * nc; e += blockDim.x) {
    const int il = e / nc, cc = e - il * nc;
    const int64_t i = i0 + il, j = x0 + j0 + cc;
    typename N::Acc acc = N::acc(ld_num<P>(A, ps, i * lda + j));
    const double* arow = A + i * lda + r0;
    int k = 0;
    for (; k + U <= nb; k += U) {
      typename N::T a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        a[u] = ld_num<P>(arow, ps, k + u);
#pragma unroll
        for (int c = 0; c < P; c++) N::put(b[u], c, Xs[c][k + u][cc]);
      }
#pragma unroll
      for (int u = 0; u < U; u++) N::acc_sub(acc, a[u], b[u]);
    }
    for (; k < nb; k++) {
      typename N::T b;
#pragma unroll
      for (int c = 0; c < P; c++) N::put(b, c, Xs[c][k][cc]);
      N::acc_sub(acc, ld_num<P>(arow, ps, k), b);
    }
    st_num<P>(A, ps, i * lda + j, N::value(acc));
  }
}

// X := L^-1 X for the steps recorded by the panel (their tiles are disjoint
// and lie above the diagonal, where no L is read): workgroup (g, q) solves
// column group g of step q and stores it.
template <int P>
__global__ __launch_bounds__(1024) void trsm_nodes_kernel(double* A, int64_t lda, int64_t ps,
                                                          TrsmNodes nodes) {
  constexpr int R = trsm_rows<P>();
  __shared__ double Ls[P][R][R + 1];
  __shared__ double Xs[P][R][kTrsmCols + 1];
  const int q = blockIdx.y;
  const int cpb = blockDim.x / 64;
  const int64_t j0 = (int64_t)blockIdx.x * cpb;
  if (j0 >= nodes.nc[q]) return;  // uniform per workgroup
  const int nc = (int)min((int64_t)cpb, nodes.nc[q] - j0);
  trsm_tile<P>(A, lda, ps, nodes.r0[q], nodes.r0[q], nodes.nb[q], nodes.x0[q], j0, nc, Ls, Xs);
  store_x_tile<P>(A, lda, ps, nodes.r0[q], nodes.nb[q], nodes.x0[q], j0, nc, Xs);
}

__global__ void lu_init_kernel(int32_t* info, int32_t* perm, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0) *info = 0;
  if (perm && i < n) perm[i] = (int32_t)i;
}

// ---- getrs pieces ----------------------------------------------------------

// perm from ipiv: the interchanges applied in order to the identity (one
// thread; the row permutation is inherently sequential in ipiv).
__global__ void perm_from_ipiv_kernel(const int32_t* ipiv, int64_t n, int32_t* perm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
  for (int64_t k = 0; k < n; k++) {
    const int64_t p = ipiv[k];
    if (p != k) {
      const int32_t x = perm[k];
      perm[k] = perm[p];
      perm[p] = x;
    }
  }
}

// X[i][:] = B[perm[i]][:] (X tight, n x nrhs, P planes); also clears the
// nflags block flags of the two triangular solves that follow.
__global__ __launch_bounds__(256) void gather_rows_kernel(const double* B, int64_t ldb,
                                                          int64_t psb, int P, const int32_t* perm,
                                                          int64_t n, int64_t nrhs, double* X,
                                                          int* flags, int nflags) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < nflags) flags[e] = 0;
  if (e >= n * nrhs) return;
  const int64_t i = e / nrhs, c = e % nrhs;
  const int64_t src = (int64_t)perm[i] * ldb + c;
  for (int q = 0; q < P; q++) X[q * n * nrhs + e] = B[q * psb + src];
}

__global__ __launch_bounds__(256) void scatter_rows_kernel(const double* X, int64_t n,
                                                           int64_t nrhs, int P, double* B,
                                                           int64_t ldb, int64_t psb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t i = e / nrhs, c = e % nrhs;
  for (int q = 0; q < P; q++) B[q * psb + i * ldb + c] = X[q * n * nrhs + e];
}

// block size of the blocked triangular solves
template <int P>
constexpr int trsv_block() {
  return P == 2 ? kTrsvBlockDD : kTrsvBlockQD;
}

// Longest wait for a block another workgroup solves (100 MHz ticks: 2 s).
// Reached only if that workgroup never runs; the solve then finishes with
// wrong values instead of hanging, and records it in the flag word after the
// block flags.
constexpr uint64_t kTrsvWaitTicks = 200000000ull;
constexpr int kTrsvWgs = 32;  // workgroups of one triangular solve launch
// The first blocks of a triangle are solved by substitution: the chain
// reaches them before an inverse could be formed.
constexpr int kTrsvDirect = 3;

// One triangle of X := T^-1 X (unit lower, or upper with its diagonal; X is
// n x nrhs, nrhs <= 16, tight) in one launch of G <= kTrsvWgs workgroups:
// workgroup w solves the block rows of TB rows in steps s = w, w + G, ...,
// step s being block row I = s (lower) or nb - 1 - s (upper).
//   1. It first forms Z = D^-1 of its diagonal block D = T_II, while it has
//      nothing else to do (the chain reaches block I only after the blocks
//      before it): wave v computes the columns v, v + 16, ... of Z, lane =
//      row, by substitution on the unit vectors (the upper solve multiplies
//      by reciprocals of the diagonal formed by all lanes at once), the
//      columns of one wave interleaved so that their dependent chains
//      overlap.
//   2. It applies, in the order they are solved, every block J it depends
//      on (J < I lower, J > I upper): it stages T_IJ while it waits for J's
//      flag, then forms sum_k T_IJ[i][k] X_J[k][c] with tpe threads per
//      entry (each a slice of k accumulated lazily, the slices summed in a
//      fixed butterfly) and subtracts it from its entry r_I.
//   3. X_I = Z r_I, by the same sliced products, is stored with
//      device-coherent stores and published: flag[I] := tag (1 lower,
//      2 upper) with release semantics at device scope; readers acquire the
//      flag and load the values device-coherently.
// So the chain's step from one block to the next is two small parallel
// products and a flag, not a row-by-row substitution.  Step s waits only
// for earlier steps, so the chain progresses once every workgroup of the
// launch has been dispatched (a few dozen workgroups: a handful of
// concurrent solves cannot fill the device with waiting ones).  The
// accumulation order is fixed: the result does not depend on timing.
template <int P>
__global__ __launch_bounds__(1024) void trsv_chain_kernel(const double* T, int64_t ldt,
                                                          int64_t pst, double* X, int64_t n,
                                                          int64_t nrhs, int upper, int* flags) {
  using N = LuArith<P>;
  using V = typename N::T;
  constexpr int TB = trsv_block<P>();
  constexpr int kPer = (TB * TB + 1023) / 1024;  // tile elements per thread
  constexpr int kZc = TB / 16;                   // columns of Z per wave
  __shared__ double Ws[P][TB][TB + 1];            // T_IJ
  __shared__ double Zs[P][TB][TB + 1];            // D = T_II, then Z = D^-1
  __shared__ double Ys[P][TB][17];                // X_J, then r_I, then X_I
  const int64_t nb = (n + TB - 1) / TB;
  for (int64_t s = blockIdx.x; s < nb; s += gridDim.x) {
    const int64_t I = upper ? nb - 1 - s : s;
    const int tag = upper ? 2 : 1;
    const int64_t i0 = I * TB;
    const int rows = (int)(n - i0 < TB ? n - i0 : TB);
    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    const int nr = (int)nrhs;
    const int64_t psx = n * nrhs;
    // threads per entry of X_I in the products: a power of two <= 16 (lanes
    // of one wave) with rows * nr * tpe <= 1024
    int tpe = 1;
    while (tpe < 16 && rows * nr * tpe * 2 <= 1024) tpe *= 2;
    const int ent = t / tpe, slice = t % tpe;
    const int ui = nr > 0 ? ent / nr : 0, uc = nr > 0 ? ent % nr : 0;
    const bool uin = ent < rows * nr;
    V x = N::zero();
    if (uin)
#pragma unroll
      for (int c = 0; c < P; c++) N::put(x, c, X[c * psx + (i0 + ui) * nrhs + uc]);

    auto stage = [&](int64_t J, double (&v)[kPer][P]) {
      const int64_t j0 = J * TB;
      const int cols = (int)(n - j0 < TB ? n - j0 : TB);
#pragma unroll
      for (int q = 0; q < kPer; q++) {
        const int e = t + 1024 * q, i = e / TB, k = e % TB;
        const bool in = e < TB * TB && i < rows && k < cols;
        const int64_t o = (i0 + (in ? i : 0)) * ldt + j0 + (in ? k : 0);
#pragma unroll
        for (int c = 0; c < P; c++)
          v[q][c] = in ? T[c * pst + o] : ((J == I && c == 0 && i == k) ? 1.0 : 0.0);
      }
    };
    auto to_lds = [&](const double (&v)[kPer][P], double (&W)[P][TB][TB + 1]) {
#pragma unroll
      for (int q = 0; q < kPer; q++) {
        const int e = t + 1024 * q, i = e / TB, k = e % TB;
        if (e < TB * TB)
#pragma unroll
          for (int c = 0; c < P; c++) W[c][i][k] = v[q][c];
      }
    };
    // -(sum over this thread's slice of k of W[ui][k] Ys[k][uc]), the slices
    // of an entry then summed by a butterfly inside the wave (every thread
    // of the entry ends with the same value)
    auto product = [&](const double (&W)[P][TB][TB + 1], int cols) {
      typename N::Acc a = N::acc(N::zero());
      if (uin)
        for (int k = slice; k < cols; k += tpe) {
          V tv, yv;
#pragma unroll
          for (int c = 0; c < P; c++) {
            N::put(tv, c, W[c][ui][k]);
            N::put(yv, c, Ys[c][k][uc]);
          }
          N::acc_sub(a, tv, yv);
        }
      V part = N::value(a);
      for (int off = 1; off < tpe; off <<= 1) {
        V o;
#pragma unroll
        for (int c = 0; c < P; c++) N::put(o, c, __shfl_xor(N::get(part, c), off, 64));
        part = (slice & off) ? N::add(o, part) : N::add(part, o);
      }
      return part;
    };
    const bool by_inverse = s >= kTrsvDirect;  // uniform
    {
      // 1. Z = D^-1 (the first blocks keep D)
      double vd[kPer][P];
      stage(I, vd);
      __syncthreads();  // the previous step's readers of Zs are done
      to_lds(vd, Zs);
      __syncthreads();
    }
    if (by_inverse) {
      auto dval = [&](int i, int k) {
        V r;
#pragma unroll
        for (int c = 0; c < P; c++) N::put(r, c, Zs[c][i][k]);
        return r;
      };
      typename N::Acc za[kZc];
#pragma unroll
      for (int q = 0; q < kZc; q++) za[q] = N::acc(lane == wave + 16 * q ? N::one() : N::zero());
      if (!upper) {
        for (int k = 0; k < TB - 1; k++) {
#pragma unroll
          for (int q = 0; q < kZc; q++) {
            if (k < wave + 16 * q) continue;  // uniform: column j starts at row j
            const V zk = readlane_words<P>(za[q], k);
            if (lane > k && lane < TB) N::acc_sub(za[q], dval(lane, k), zk);
          }
        }
      } else {
        const V inv = lane < TB ? N::div(N::one(), dval(lane, lane)) : N::zero();
        for (int k = TB - 1; k >= 0; k--) {
#pragma unroll
          for (int q = 0; q < kZc; q++) {
            if (k > wave + 16 * q) continue;  // uniform: column j has rows <= j
            const V zk = N::mul(readlane_words<P>(za[q], k), readlane_num<P>(inv, k));
            if (lane == k)
              za[q] = N::acc(zk);
            else if (lane < k)
              N::acc_sub(za[q], dval(lane, k), zk);
          }
        }
      }
      __syncthreads();  // every wave has read D
      if (lane < TB)
#pragma unroll
        for (int q = 0; q < kZc; q++) {
          const V z = N::value(za[q]);
#pragma unroll
          for (int c = 0; c < P; c++) Zs[c][lane][wave + 16 * q] = N::get(z, c);
        }
    }
    // 2. the blocks this one depends on
    double v[kPer][P];
    for (int64_t d = 0; d < s; d++) {
      const int64_t J = upper ? nb - 1 - d : d;
      stage(J, v);  // the tile's loads fly while this workgroup waits for J
      if (t == 0) {
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(flags + J, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != tag) {
          __builtin_amdgcn_s_sleep(2);
          if (__builtin_amdgcn_s_memrealtime() - t0 > kTrsvWaitTicks) {
            __hip_atomic_fetch_or(flags + nb, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
      __syncthreads();  // J is published (and every reader of Ws / Ys of the last step is done)
      const int64_t j0 = J * TB;
      const int cols = (int)(n - j0 < TB ? n - j0 : TB);
      {
        const int yi = t / 16, yc = t % 16;
        if (yi < cols && yc < nr)
#pragma unroll
          for (int c = 0; c < P; c++)
            Ys[c][yi][yc] = __hip_atomic_load(X + c * psx + (j0 + yi) * nrhs + yc,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      to_lds(v, Ws);
      __syncthreads();
      const V part = product(Ws, cols);  // minus T_IJ X_J
      if (uin) x = N::add(x, part);
      __syncthreads();  // Ws and Ys are rewritten by the next step
    }
    // 3. X_I = Z r_I, or by substitution in D (one wave per right-hand side,
    // lane = row: step k finishes x_k, broadcasts it by readlane, the other
    // lanes subtract D_ik x_k; DD broadcasts the unnormalised accumulator)
    if (uin && slice == 0)
#pragma unroll
      for (int c = 0; c < P; c++) Ys[c][ui][uc] = N::get(x, c);
    for (int k = rows + t; k < TB; k += 1024)  // rows past the matrix: r = 0
      for (int cc = 0; cc < nr; cc++)
#pragma unroll
        for (int c = 0; c < P; c++) Ys[c][k][cc] = 0.0;
    __syncthreads();  // r_I and Z (or D) are in LDS
    if (by_inverse) {
      const V xs = N::sub(N::zero(), product(Zs, TB));
      __syncthreads();  // every thread has read r_I
      if (uin && slice == 0)
#pragma unroll
        for (int c = 0; c < P; c++) Ys[c][ui][uc] = N::get(xs, c);
    } else if (wave < nr) {
      auto dval = [&](int i, int k) {
        V r;
#pragma unroll
        for (int c = 0; c < P; c++) N::put(r, c, Zs[c][i][k]);
        return r;
      };
      V xinit = N::zero();
      if (lane < TB)
#pragma unroll
        for (int c = 0; c < P; c++) N::put(xinit, c, Ys[c][lane][wave]);
      typename N::Acc acc = N::acc(xinit);
      if (!upper) {
        for (int k = 0; k < TB - 1; k++) {
          const V xk = readlane_words<P>(acc, k);
          if (lane > k && lane < TB) N::acc_sub(acc, dval(lane, k), xk);
        }
      } else {
        const V inv = lane < TB ? N::div(N::one(), dval(lane, lane)) : N::zero();
        for (int k = TB - 1; k >= 0; k--) {
          const V xk = N::mul(readlane_words<P>(acc, k), readlane_num<P>(inv, k));
          if (lane == k)
            acc = N::acc(xk);
          else if (lane < k)
            N::acc_sub(acc, dval(lane, k), xk);
        }
      }
      // lane and wave own entry (lane, wave) of Ys alone
      if (lane < TB) {
        const V xs = N::value(acc);
#pragma unroll
        for (int c = 0; c < P; c++) Ys[c][lane][wave] = N::get(xs, c);
      }
    }
    __syncthreads();
    if (wave < nr) {
      if (lane < rows)
#pragma unroll
        for (int c = 0; c < P; c++)
          __hip_atomic_store(X + c * psx + (i0 + lane) * nrhs + wave, Ys[c][lane][wave],
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // this wave's stores are complete and visible at device scope
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();  // every value of X_I is stored
    if (t == 0) __hip_atomic_store(flags + I, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();  // Ws, Zs and Ys are reused by the next step
  }
}


// ---- the paper's row-wise parallel LU (its comparator) --------------------
//
// Unblocked elimination without pivoting, one launch per step k (Sec. 4
// compares its blocked LU against this row-parallel form): a workgroup takes
// kRwRows rows by kRwCols columns of the trailing matrix, forms its rows'
// multipliers l_ik = a_ik / a_kk in LDS and updates a_ij -= l_ik a_kj.  Column
// k keeps the unscaled a_ik (other workgroups of the same step still read
// it); one last launch divides every sub-diagonal column by its pivot, with
// the same division, so L is what the steps used.  An exactly zero pivot sets
// info (first one) and its step is skipped, as in the blocked form.
constexpr int kRwRows = 16, kRwCols = 256;

template <int P>
__global__ __launch_bounds__(256) void rowwise_step_kernel(double* A, int64_t lda, int64_t ps,
                                                           int64_t n, int64_t k,
                                                           int32_t* info) {
  using N = LuArith<P>;
  using V = typename N::T;
  __shared__ double lsh[P][kRwRows];
  __shared__ double ush[P][kRwCols];
  const V u = ld_num<P>(A, ps, k * lda + k);
  if (N::is_zero(u)) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && *info == 0)
      *info = (int32_t)(k + 1);
    return;  // uniform: every thread read the same pivot
  }
  const int t = threadIdx.x;
  const int64_t i0 = k + 1 + (int64_t)blockIdx.y * kRwRows;
  const int64_t j0 = k + 1 + (int64_t)blockIdx.x * kRwCols;
  if (t < kRwRows) {
    const int64_t i = i0 + t;
    V l = N::zero();
    if (i < n) l = N::div_digits(ld_num<P>(A, ps, i * lda + k), u, 1.0 / N::get(u, 0));
#pragma unroll
    for (int c = 0; c < P; c++) lsh[c][t] = N::get(l, c);
  }
  const int64_t j = j0 + t;
  {
    V x = N::zero();
    if (j < n) x = ld_num<P>(A, ps, k * lda + j);
#pragma unroll
    for (int c = 0; c < P; c++) ush[c][t] = N::get(x, c);
  }
  __syncthreads();
  if (j >= n) return;
  V ukj;
#pragma unroll
  for (int c = 0; c < P; c++) N::put(ukj, c, ush[c][t]);
  for (int r = 0; r < kRwRows; r++) {
    const int64_t i = i0 + r;
    if (i >= n) break;
    V l;
#pragma unroll
    for (int c = 0; c < P; c++) N::put(l, c, lsh[c][r]);
    st_num<P>(A, ps, i * lda + j, N::sub(ld_num<P>(A, ps, i * lda + j), N::mul(l, ukj)));
  }
}

// L from the unscaled columns: a_ik := a_ik / a_kk for i > k (columns with a
// zero pivot stay as they are); the last pivot's zero test; ipiv := identity.
template <int P>
__global__ __launch_bounds__(256) void rowwise_scale_kernel(double* A, int64_t lda, int64_t ps,
                                                            int64_t n, int32_t* ipiv,
                                                            int32_t* info) {
  using N = LuArith<P>;
  using V = typename N::T;
  const int64_t i = blockIdx.y;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && k < n) ipiv[k] = (int32_t)k;
  if (i == n - 1 && k == 0 && N::is_zero(ld_num<P>(A, ps, (n - 1) * lda + n - 1)) && *info == 0)
    *info = (int32_t)n;
  if (k >= i) return;
  const V u = ld_num<P>(A, ps, k * lda + k);
  if (N::is_zero(u)) return;
  st_num<P>(A, ps, i * lda + k,
            N::div_digits(ld_num<P>(A, ps, i * lda + k), u, 1.0 / N::get(u, 0)));
}

}  // namespace

// ---- launchers ---------------------------------------------------------------

// The row-wise comparator: n - 1 step launches and the scaling launch.
int launch_rowwise_lu(int P, double* A, int64_t lda, int64_t ps, int64_t n, int32_t* ipiv,
                      int32_t* info, hipStream_t s) {
  if (n > 65535) return set_error(DDQD_E_UNSUPPORTED, "row-wise LU of order above 65535");
  for (int64_t k = 0; k + 1 < n; k++) {
    const int64_t m = n - k - 1;
    const dim3 grid((unsigned)((m + kRwCols - 1) / kRwCols), (unsigned)((m + kRwRows - 1) / kRwRows));
    prof_begin(s);
    if (P == 2)
      hipLaunchKernelGGL(rowwise_step_kernel<2>, grid, dim3(256), 0, s, A, lda, ps, n, k, info);
    else
      hipLaunchKernelGGL(rowwise_step_kernel<4>, grid, dim3(256), 0, s, A, lda, ps, n, k, info);
    prof_record("rowwise_step_kernel", s);
  }
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  prof_begin(s);
  if (P == 2)
    hipLaunchKernelGGL(rowwise_scale_kernel<2>, grid, dim3(256), 0, s, A, lda, ps, n, ipiv, info);
  else
    hipLaunchKernelGGL(rowwise_scale_kernel<4>, grid, dim3(256), 0, s, A, lda, ps, n, ipiv, info);
  prof_record("rowwise_scale_kernel", s);
  return check_launch("rowwise LU");
}

int launch_lu_init(int32_t* info, int32_t* perm, int64_t n, hipStream_t s) {
  prof_begin(s);
  hipLaunchKernelGGL(lu_init_kernel, dim3((unsigned)((n + 256) / 256)), dim3(256), 0, s, info,
                     perm, n);
  prof_record("lu_init_kernel", s);
  return check_launch("lu_init_kernel");
}

// Strip shape by panel height: threads, rows per thread, strip width.  The
// register tile (RPT x W values of P words) stays within what one thread can
// hold; taller strips (and QD) are narrower.
int getf2_width(int P, int64_t m) {
  if (P == 2) return m <= 2048 ? 8 : (m <= 4096 ? 4 : 2);
  return m <= 512 ? 8 : (m <= 1024 ? 4 : (m <= 2048 ? 2 : 1));
}

int trsm_max_rows(int P) { return P == 2 ? trsm_rows<2>() : trsm_rows<4>(); }

int launch_getf2(int P, double* A, int64_t lda, int64_t ps, int64_t r0, int64_t m, int64_t c0,
                 int w, int32_t* ipiv, int32_t* info, int pivot, hipStream_t s) {
  if (m <= 0 || w <= 0) return 0;
  if (m > 8192) return set_error(4, "LU of more than 8192 rows is not supported");
  if (w > getf2_width(P, m)) return set_error(4, "getf2 strip too wide");
#define GETF2(PP, T, R, W)                                                                    \
  do {                                                                                        \
    prof_begin(s);                                                                            \
    hipLaunchKernelGGL((getf2_kernel<PP, T, R, W>), dim3(1), dim3(T), 0, s, A, lda, ps, r0, m, \
                       c0, w, ipiv, info, pivot);                                             \
    prof_record("getf2_kernel", s);                                                          \
  } while (0)
  if (P == 2) {
    if (m <= 256) GETF2(2, 256, 1, 8);
    else if (m <= 512) GETF2(2, 512, 1, 8);
    else if (m <= 1024) GETF2(2, 1024, 1, 8);
    else if (m <= 2048) GETF2(2, 1024, 2, 8);
    else if (m <= 4096) GETF2(2, 512, 8, 4);
    else GETF2(2, 1024, 8, 2);
  } else {
    // QD values take four registers: at most 512 threads (256 registers each)
    if (m <= 256) GETF2(4, 256, 1, 8);
    else if (m <= 512) GETF2(4, 512, 1, 8);
    else if (m <= 1024) GETF2(4, 512, 2, 4);
    else if (m <= 2048) GETF2(4, 512, 4, 2);
    else if (m <= 4096) GETF2(4, 512, 8, 1);
    else GETF2(4, 1024, 8, 1);
  }
#undef GETF2
  return check_launch("getf2_kernel");
}

int launch_laswp(int P, double* A, int64_t lda, int64_t ps, int64_t n_cols, int64_t skip0,
                 int64_t skip1, int64_t k0, int64_t k1, const int32_t* ipiv, int32_t* perm,
                 hipStream_t s) {
  if (k1 <= k0) return 0;
  prof_begin(s);
  hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)((n_cols + 1 + 255) / 256)), dim3(256), 0, s,
                     A, lda, ps, P, n_cols, skip0, skip1, k0, k1, ipiv, perm);
  prof_record("laswp_kernel", s);
  return check_launch("laswp_kernel");
}

int launch_trsm_wave(int P, double* A, int64_t lda, int64_t ps, int64_t r0, int64_t c0, int nb,
                     int64_t x0, int64_t ncols, hipStream_t s) {
  if (nb <= 0 || ncols <= 0) return 0;
  if (nb > trsm_max_rows(P)) return set_error(4, "trsm_wave: block too large");
  // enough workgroups to reach every compute unit before stacking columns
  int64_t cpb = (ncols + 255) / 256;
  if (cpb > kTrsmCols) cpb = kTrsmCols;
  if (cpb > ncols) cpb = ncols;
  const int64_t blocks = (ncols + cpb - 1) / cpb;
  prof_begin(s);
  if (P == 2)
    hipLaunchKernelGGL(trsm_wave_kernel<2>, dim3((unsigned)blocks), dim3((unsigned)(64 * cpb)), 0,
                       s, A, lda, ps, r0, c0, nb, x0, ncols);
  else
    hipLaunchKernelGGL(trsm_wave_kernel<4>, dim3((unsigned)blocks), dim3((unsigned)(64 * cpb)), 0,
                       s, A, lda, ps, r0, c0, nb, x0, ncols);
  prof_record("trsm_wave_kernel", s);
  return check_launch("trsm_wave_kernel");
}

int launch_trsm_update(int P, double* A, int64_t lda, int64_t ps, int64_t r0, int nb,
                       int64_t x0, int64_t ncols, int64_t mb, hipStream_t s) {
  if (nb <= 0 || ncols <= 0) return 0;
  if (nb > trsm_max_rows(P)) return set_error(4, "trsm_update: block too large");
  if (mb <= 0) return set_error(4, "trsm_update: no rows to update");
  const int64_t cpb = ncols < kTrsmCols ? ncols : kTrsmCols;
  const int64_t gx = (ncols + cpb - 1) / cpb, gy = (mb + kTrsmUpdRows - 1) / kTrsmUpdRows;
  if (gx > INT32_MAX || gy > 65535) return set_error(4, "trsm_update: grid too large");
  prof_begin(s);
  if (P == 2)
    hipLaunchKernelGGL(trsm_update_kernel<2>, dim3((unsigned)gx, (unsigned)gy),
                       dim3((unsigned)(64 * cpb)), 0, s, A, lda, ps, r0, nb, x0, ncols, mb);
  else
    hipLaunchKernelGGL(trsm_update_kernel<4>, dim3((unsigned)gx, (unsigned)gy),
                       dim3((unsigned)(64 * cpb)), 0, s, A, lda, ps, r0, nb, x0, ncols, mb);
  prof_record("trsm_update_kernel", s);
  return check_launch("trsm_update_kernel");
}

int launch_trsm_nodes(int P, double* A, int64_t lda, int64_t ps, const TrsmNodes& nodes,
                      hipStream_t s) {
  if (nodes.count <= 0) return 0;
  if (nodes.count > kTrsmNodesMax) return set_error(4, "trsm_nodes: too many steps");
  int maxnc = 0;
  for (int q = 0; q < nodes.count; q++) {
    if (nodes.nb[q] > trsm_max_rows(P) || nodes.nb[q] <= 0 || nodes.nc[q] <= 0)
      return set_error(4, "trsm_nodes: bad step");
    if (nodes.nc[q] > maxnc) maxnc = nodes.nc[q];
  }
  const int cpb = maxnc < kTrsmCols ? maxnc : kTrsmCols;
  const int gx = (maxnc + cpb - 1) / cpb;
  prof_begin(s);
  if (P == 2)
    hipLaunchKernelGGL(trsm_nodes_kernel<2>, dim3((unsigned)gx, (unsigned)nodes.count),
                       dim3((unsigned)(64 * cpb)), 0, s, A, lda, ps, nodes);
  else
    hipLaunchKernelGGL(trsm_nodes_kernel<4>, dim3((unsigned)gx, (unsigned)nodes.count),
                       dim3((unsigned)(64 * cpb)), 0, s, A, lda, ps, nodes);
  prof_record("trsm_nodes_kernel", s);
  return check_launch("trsm_nodes_kernel");
}

int launch_lu_update(int P, const double* A, const double* B, double* C, int64_t ld, int64_t ps,
                     int64_t m, int64_t n, int64_t l, hipStream_t s) {
  if (m <= 0 || n <= 0 || l <= 0) return 0;
  const int64_t blocks = (m * n + 255) / 256;
  if (blocks > INT32_MAX) return set_error(4, "lu_update: grid too large");
  prof_begin(s);
  if (P == 2)
    hipLaunchKernelGGL(lu_update_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, A, B, C, ld,
                       ps, m, n, l);
  else
    hipLaunchKernelGGL(lu_update_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, s, A, B, C, ld,
                       ps, m, n, l);
  prof_record("lu_update_kernel", s);
  return check_launch("lu_update_kernel");
}

int launch_perm_from_ipiv(const int32_t* ipiv, int64_t n, int32_t* perm, hipStream_t s) {
  prof_begin(s);
  hipLaunchKernelGGL(perm_from_ipiv_kernel, dim3(1), dim3(64), 0, s, ipiv, n, perm);
  prof_record("perm_from_ipiv_kernel", s);
  return check_launch("perm_from_ipiv_kernel");
}

int launch_gather_rows(int P, const double* B, int64_t ldb, int64_t psb, const int32_t* perm,
                       int64_t n, int64_t nrhs, double* X, int* flags, int nflags,
                       hipStream_t s) {
  const int64_t items = n * nrhs > nflags ? n * nrhs : nflags;
  prof_begin(s);
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s,
                     B, ldb, psb, P, perm, n, nrhs, X, flags, nflags);
  prof_record("gather_rows_kernel", s);
  return check_launch("gather_rows_kernel");
}

int launch_scatter_rows(int P, const double* X, int64_t n, int64_t nrhs, double* B, int64_t ldb,
                        int64_t psb, hipStream_t s) {
  prof_begin(s);
  hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)((n * nrhs + 255) / 256)), dim3(256), 0,
                     s, X, n, nrhs, P, B, ldb, psb);
  prof_record("scatter_rows_kernel", s);
  return check_launch("scatter_rows_kernel");
}

int launch_trsv_chain(int P, const double* T, int64_t ldt, int64_t pst, double* X, int64_t n,
                      int64_t nrhs, int upper, int* flags, hipStream_t s) {
  const int TB = P == 2 ? trsv_block<2>() : trsv_block<4>();
  const int64_t nb = (n + TB - 1) / TB;
  if (nrhs > 16) return set_error(DDQD_E_UNSUPPORTED, "at most 16 right-hand sides per solve call");
  if (nb + 1 > trsv_flag_words(n)) return set_error(DDQD_E_HIP, "trsv flags out of range");
  const unsigned grid = (unsigned)(nb < kTrsvWgs ? nb : kTrsvWgs);
  prof_begin(s);
  if (P == 2)
    hipLaunchKernelGGL(trsv_chain_kernel<2>, dim3(grid), dim3(1024), 0, s, T, ldt, pst, X, n,
                       nrhs, upper, flags);
  else
    hipLaunchKernelGGL(trsv_chain_kernel<4>, dim3(grid), dim3(1024), 0, s, T, ldt, pst, X, n,
                       nrhs, upper, flags);
  prof_record("trsv_chain_kernel", s);
  return check_launch("trsv_chain_kernel");
}

}  // namespace ddqd
