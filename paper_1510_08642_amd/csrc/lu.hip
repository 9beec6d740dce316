// DD LU kernels: the narrow-panel factorisation (getf2), row interchanges
// (laswp), small triangular solves, and the blocked triangular solves of
// getrs.  The blocked right-looking driver that strings them together with
// the matrix product lives in lu_driver.hip.
//
// Paper: Sec. 4, steps 1-3 (factor A11, form U12 and L21, update A22 with a
// matrix product) and Eq. 2 (solve Ax = b).  Partial pivoting (largest
// |a_ic|, first index on ties, decided in DD) is an option the paper, which
// factors without pivoting, does not use.
#include "common.hpp"
#include "eft.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

__device__ __forceinline__ dd_t ld_dd(const double* A, int64_t ps, int64_t idx) {
  return dd_t{A[idx], A[ps + idx]};
}
__device__ __forceinline__ void st_dd(double* A, int64_t ps, int64_t idx, dd_t v) {
  A[idx] = v.hi;
  A[ps + idx] = v.lo;
}
__device__ __forceinline__ dd_t dd_abs(dd_t x) { return x.hi < 0.0 ? dd_neg(x) : x; }

// (x, i) beats (y, j): larger |value|; on equal values the smaller row index.
// i < 0 marks "no candidate".  The high words decide when they differ by more
// than the low words can make up (their difference is exact when they are
// within a factor 2, and far larger than the low words otherwise); only
// near-ties take the full DD comparison.
__device__ __forceinline__ bool better(dd_t x, int i, dd_t y, int j) {
  if (i < 0) return false;
  if (j < 0) return true;
  const double dh = fabs(x.hi) - fabs(y.hi);
  const double lim = 2.0 * (fabs(x.lo) + fabs(y.lo));
  if (dh > lim) return true;
  if (-dh > lim) return false;
  const int c = dd_abs_cmp(x, y);
  return c > 0 || (c == 0 && i < j);
}

// x / y by three long-division digits, each the leading remainder times an
// FP64 reciprocal of y.hi shared by the whole column (a digit may be off by
// an ulp; the next remainder, formed in DD, absorbs it).
__device__ __forceinline__ dd_t dd_div_digits(dd_t x, dd_t y, double yinv) {
  const double q1 = x.hi * yinv;
  dd_t r = dd_sub(x, dd_mul_d(y, q1));
  const double q2 = r.hi * yinv;
  r = dd_sub(r, dd_mul_d(y, q2));
  const double q3 = r.hi * yinv;
  dd_t q;
  fast_two_sum(q1, q2, q.hi, q.lo);
  return dd_add(q, dd_t{q3, 0.0});
}

// ---- getf2: factor an m x w strip (w <= W) held in registers ---------------
// One workgroup of T threads; thread t owns local rows t + T q, q < RPT.
// The strip moves between HBM and registers through an LDS tile, so that
// global accesses run along the rows (coalesced); all of a thread's loads of a
// chunk are issued before the first is used.
// Column c, with one barrier:
//   1. every wave finds its best candidate |a_ic| (rows i >= c; DD compare,
//      ties to the smaller row; see wave_argmax); it publishes the value, the
//      row index and the winning row's W values, and the owner of row c
//      publishes row c;
//   2. after the barrier every wave reduces the wave winners itself and reads
//      the pivot row p from the winning wave's slot; the owners of rows c and
//      p exchange them in registers;
//   3. the column below the pivot is divided by the pivot (DD long division)
//      and the remaining strip columns get the rank-1 update.
// The published slots are double-buffered by the parity of c: a slot is
// rewritten two columns later, after a barrier that every reader of its old
// contents has passed.
// ipiv[c0 + c] receives the global (0-based) pivot row; info the first
// 1-based global column whose pivot is exactly zero, if none was recorded
// before.  Other columns of the matrix are interchanged later by laswp.

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

template <int kCtrl>
__device__ __forceinline__ void argmax_step_dpp(dd_t& b, int& bi, int& tag) {
  const dd_t o{dpp_f64<kCtrl>(b.hi), dpp_f64<kCtrl>(b.lo)};
  const int oi = dpp_i32<kCtrl>(bi), ot = dpp_i32<kCtrl>(tag);
  if (better(o, oi, b, bi)) {
    b = o;
    bi = oi;
    tag = ot;
  }
}
__device__ __forceinline__ void argmax_step_shfl(dd_t& b, int& bi, int& tag, int off) {
  const dd_t o{__shfl_xor(b.hi, off, 64), __shfl_xor(b.lo, off, 64)};
  const int oi = __shfl_xor(bi, off, 64), ot = __shfl_xor(tag, off, 64);
  if (better(o, oi, b, bi)) {
    b = o;
    bi = oi;
    tag = ot;
  }
}
// after the four steps every lane of a 16-lane row holds the row's best
__device__ __forceinline__ void argmax_row16(dd_t& b, int& bi, int& tag) {
  argmax_step_dpp<kDppXor1>(b, bi, tag);
  argmax_step_dpp<kDppXor2>(b, bi, tag);
  argmax_step_dpp<kDppHalfMirror>(b, bi, tag);
  argmax_step_dpp<kDppMirror>(b, bi, tag);
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

// The lane holding the best candidate of a wave (largest |x| in DD, then the
// smallest index; idx < 0 marks "no candidate"), the same in every lane, or
// -1 if no lane has one.  FP64 maxima of |hi| and |lo| find the leader; a
// lane can equal or beat it only if the gap between its |hi| and the largest
// is within the low words' bound, and when that holds for one lane alone it
// is the winner.  Otherwise the DD comparison decides among those lanes.
// kRow0: candidates only in lanes 0..15.
template <bool kRow0>
__device__ __forceinline__ int wave_argmax(dd_t x, int idx) {
  const int lane = threadIdx.x % 64;
  const bool valid = idx >= 0;
  const double h = valid ? fabs(x.hi) : -1.0, l = valid ? fabs(x.lo) : -1.0;
  double M = row16_max(h), L = row16_max(l);
  if (kRow0) {
    M = readlane_f64(M, 0);
    L = readlane_f64(L, 0);
  } else {
    M = fmax(fmax(readlane_f64(M, 0), readlane_f64(M, 16)),
             fmax(readlane_f64(M, 32), readlane_f64(M, 48)));
    L = fmax(fmax(readlane_f64(L, 0), readlane_f64(L, 16)),
             fmax(readlane_f64(L, 32), readlane_f64(L, 48)));
  }
  if (!(M >= 0.0)) return -1;
  const bool close = valid && (M - h) <= 2.0 * (L + l);
  const uint64_t mask = __ballot(close);
  if (__popcll(mask) == 1) return __ffsll((unsigned long long)mask) - 1;
  dd_t b = close ? x : dd_t{0.0, 0.0};
  int bi = close ? idx : -1, tag = lane;
  argmax_row16(b, bi, tag);
  if (!kRow0) {
    argmax_step_shfl(b, bi, tag, 16);
    argmax_step_shfl(b, bi, tag, 32);
  }
  return __builtin_amdgcn_readlane(tag, 0);
}

template <int T, int RPT, int W>
__global__ __launch_bounds__(T) void getf2_kernel(double* A, int64_t lda, int64_t ps,
                                                   int64_t r0, int64_t m, int64_t c0, int w,
                                                   int32_t* ipiv, int32_t* info, int pivot) {
  constexpr int kLd = W + 1;  // padded LDS row of the staging tile
  constexpr int kWaves = T / 64;
  static_assert(kWaves == 4 || kWaves == 8 || kWaves == 16, "T must be 256, 512 or 1024");
  __shared__ double tile[T * kLd];
  __shared__ double s_val[2][kWaves][2];
  __shared__ int s_idx[2][kWaves];
  __shared__ double s_row[2][kWaves][2][W];
  __shared__ double s_rowc[2][2][W];
  const int t = threadIdx.x, lane = t % 64, wave = t / 64;
  dd_t v[RPT][W];
#pragma unroll
  for (int q = 0; q < RPT; q++) {
    const int64_t rows = min((int64_t)T, m - (int64_t)T * q);
    if (rows <= 0) {
#pragma unroll
      for (int k = 0; k < W; k++) v[q][k] = dd_t{0.0, 0.0};
      continue;
    }
    const int n = (int)rows * w;
    const double* src = A + (r0 + (int64_t)T * q) * lda + c0;
    double xh[W], xl[W];
#pragma unroll
    for (int j = 0; j < W; j++) {  // every load in flight before the first use
      const int e = min(t + T * j, n - 1), r = e / w, k = e - r * w;
      xh[j] = src[(int64_t)r * lda + k];
      xl[j] = src[ps + (int64_t)r * lda + k];
    }
#pragma unroll
    for (int plane = 0; plane < 2; plane++) {
#pragma unroll
      for (int j = 0; j < W; j++) {
        const int e = t + T * j, r = e / w, k = e - r * w;
        if (e < n) tile[r * kLd + k] = plane == 0 ? xh[j] : xl[j];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < W; k++) {
        const double x = (t < rows && k < w) ? tile[t * kLd + k] : 0.0;
        if (plane == 0)
          v[q][k].hi = x;
        else
          v[q][k].lo = x;
      }
      __syncthreads();
    }
  }
  // The column loop is unrolled so that every register index is a constant.
#pragma unroll
  for (int c = 0; c < W; c++) {
    if (c >= w) break;
    const int buf = c & 1;
    // 1. wave-local pivot search among local rows >= c
    dd_t best{0.0, 0.0};
    int bi = -1;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int i = t + T * q;
      if (i >= c && i < m) {
        const dd_t x = dd_abs(v[q][c]);
        if (better(x, i, best, bi)) {
          best = x;
          bi = i;
        }
      }
    }
    const int wl = wave_argmax<false>(best, bi);
    const int wbi = wl >= 0 ? __builtin_amdgcn_readlane(bi, wl) : -1;
    if (lane == 0) {
      s_val[buf][wave][0] = wl >= 0 ? readlane_f64(best.hi, wl) : 0.0;
      s_val[buf][wave][1] = wl >= 0 ? readlane_f64(best.lo, wl) : 0.0;
      s_idx[buf][wave] = wbi;
    }
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int i = t + T * q;
      if (lane == wl && i == wbi)
#pragma unroll
        for (int k = 0; k < W; k++) {
          s_row[buf][wave][0][k] = v[q][k].hi;
          s_row[buf][wave][1][k] = v[q][k].lo;
        }
      if (i == c)
#pragma unroll
        for (int k = 0; k < W; k++) {
          s_rowc[buf][0][k] = v[q][k].hi;
          s_rowc[buf][1][k] = v[q][k].lo;
        }
    }
    __syncthreads();
    // 2. the winners of all waves, reduced by every wave
    dd_t b{0.0, 0.0};
    int pi = -1;
    if (lane < kWaves) {
      b = dd_t{s_val[buf][lane][0], s_val[buf][lane][1]};
      pi = s_idx[buf][lane];
    }
    const int wv = wave_argmax<true>(b, pi);
    int p = wv >= 0 ? __builtin_amdgcn_readlane(pi, wv) : -1;
    const bool use_c = !pivot || p < 0;
    if (use_c) p = c;
    const double* rph = use_c ? s_rowc[buf][0] : s_row[buf][wv][0];
    const double* rpl = use_c ? s_rowc[buf][1] : s_row[buf][wv][1];
    if (t == 0) ipiv[c0 + c] = (int32_t)(r0 + p);
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int i = t + T * q;
      if (i == c) {
#pragma unroll
        for (int k = 0; k < W; k++) v[q][k] = dd_t{rph[k], rpl[k]};
      } else if (i == p) {
#pragma unroll
        for (int k = 0; k < W; k++) v[q][k] = dd_t{s_rowc[buf][0][k], s_rowc[buf][1][k]};
      }
    }
    // 3. division by the pivot and rank-1 update of the strip
    const dd_t u{rph[c], rpl[c]};
    if (t == 0 && u.hi == 0.0 && u.lo == 0.0 && *info == 0) *info = (int32_t)(c0 + c + 1);
    if (!(u.hi == 0.0 && u.lo == 0.0)) {
      const double uinv = 1.0 / u.hi;
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const int i = t + T * q;
        if (i > c && i < m) {
          const dd_t l = dd_div_digits(v[q][c], u, uinv);
          v[q][c] = l;
#pragma unroll
          for (int k = c + 1; k < W; k++)
            if (k < w) v[q][k] = dd_sub(v[q][k], dd_mul(l, dd_t{rph[k], rpl[k]}));
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
    for (int plane = 0; plane < 2; plane++) {
      __syncthreads();  // the tile's previous readers are done
      if (t < rows)
#pragma unroll
        for (int k = 0; k < W; k++) tile[t * kLd + k] = plane == 0 ? v[q][k].hi : v[q][k].lo;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < W; j++) {
        const int e = t + T * j, r = e / w, k = e - r * w;
        if (e < n) dst[plane * ps + (int64_t)r * lda + k] = tile[r * kLd + k];
      }
    }
  }
}

// ---- laswp: rows k <-> ipiv[k] for k in [k0, k1), in order ------------------
// One thread per column (coalesced across threads), columns [skip0, skip1)
// excluded; thread n_cols applies the same interchanges to perm (if given).
__global__ __launch_bounds__(256) void laswp_kernel(double* A, int64_t lda, int64_t ps,
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
      const double h = A[a], l = A[ps + a];
      A[a] = A[b];
      A[ps + a] = A[ps + b];
      A[b] = h;
      A[ps + b] = l;
    }
  }
}

// ---- C -= A B for the thin products inside the panel ------------------------
// A (m x l), B (l x n), C (m x n) are blocks of one plane-layout matrix (same
// ld and plane stride).  One thread per entry of C; the products are summed
// without renormalisation (TwoSum of the high parts, the low parts and the
// TwoSum errors gathered in a second word), then subtracted from C in DD.
__global__ __launch_bounds__(256) void lu_update_kernel(const double* A, const double* B,
                                                        double* C, int64_t ld, int64_t ps,
                                                        int64_t m, int64_t n, int64_t l) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e / n, j = e - i * n;
  const double* a = A + i * ld;
  const double* b = B + j;
  double s = 0.0, r = 0.0;
  for (int64_t k = 0; k < l; k++) {
    const double ah = a[k], al = a[ps + k], bh = b[k * ld], bl = b[ps + k * ld];
    const double p = ah * bh;
    const double pe = fma(ah, bl, fma(al, bh, fma(ah, bh, -p)));
    double t;
    two_sum(s, p, s, t);
    r += t + pe;
  }
  dd_t x;
  two_sum(s, r, x.hi, x.lo);
  const dd_t c = ld_dd(C, ps, i * ld + j);
  st_dd(C, ps, i * ld + j, dd_sub(c, x));
}

// ---- unit-lower triangular solve with one wave per column: X := L^-1 X -----
// L = A[r0 .. r0+nb, c0 .. c0+nb) (unit diagonal, nb <= 64), X = the nb rows
// r0.. of columns [x0, x0 + ncols).  Lane i of a wave holds x_i of one column
// as an unrenormalised pair (s, r); step k renormalises x_k, broadcasts it
// with readlane, and the lanes below subtract L_ik x_k (TwoSum of the high
// product into s, the low parts and the TwoSum error into r): forward
// substitution with one rounding to DD per unknown.  A workgroup takes up to
// 16 adjacent columns, staging L (transposed, so a step reads one LDS row)
// and its X tile through LDS so that global accesses run along the rows.
constexpr int kTrsmRows = 64, kTrsmCols = 16;

__global__ __launch_bounds__(1024) void trsm_wave_kernel(double* A, int64_t lda, int64_t ps,
                                                         int64_t r0, int64_t c0, int nb,
                                                         int64_t x0, int64_t ncols) {
  __shared__ double Lh[kTrsmRows][kTrsmRows + 1], Ll[kTrsmRows][kTrsmRows + 1];
  __shared__ double Xh[kTrsmRows][kTrsmCols + 1], Xl[kTrsmRows][kTrsmCols + 1];
  const int t = threadIdx.x, lane = t % 64, wave = t / 64, nt = blockDim.x;
  const int cpb = nt / 64;  // columns per workgroup
  const int64_t j0 = (int64_t)blockIdx.x * cpb;
  const int nc = (int)min((int64_t)cpb, ncols - j0);
  for (int e = t; e < nb * nb; e += nt) {
    const int i = e / nb, k = e - i * nb;
    Lh[k][i] = A[(r0 + i) * lda + c0 + k];
    Ll[k][i] = A[ps + (r0 + i) * lda + c0 + k];
  }
  for (int e = t; e < nb * nc; e += nt) {
    const int i = e / nc, c = e - i * nc;
    Xh[i][c] = A[(r0 + i) * lda + x0 + j0 + c];
    Xl[i][c] = A[ps + (r0 + i) * lda + x0 + j0 + c];
  }
  __syncthreads();
  if (wave < nc) {
    double s = 0.0, r = 0.0;
    if (lane < nb) {
      s = Xh[lane][wave];
      r = Xl[lane][wave];
    }
    for (int k = 0; k < nb - 1; k++) {
      double kh, kl;
      two_sum(readlane_f64(s, k), readlane_f64(r, k), kh, kl);
      if (lane > k && lane < nb) {
        const double lh = Lh[k][lane], ll = Ll[k][lane];
        const double p = lh * kh;
        const double pe = fma(lh, kl, fma(ll, kh, fma(lh, kh, -p)));
        double e;
        two_sum(s, -p, s, e);
        r += e - pe;
      }
    }
    if (lane < nb) {
      double h, l;
      two_sum(s, r, h, l);
      Xh[lane][wave] = h;
      Xl[lane][wave] = l;
    }
  }
  __syncthreads();
  for (int e = t; e < nb * nc; e += nt) {
    const int i = e / nc, c = e - i * nc;
    A[(r0 + i) * lda + x0 + j0 + c] = Xh[i][c];
    A[ps + (r0 + i) * lda + x0 + j0 + c] = Xl[i][c];
  }
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

// X[i][:] = B[perm[i]][:] (X tight, n x nrhs)
__global__ __launch_bounds__(256) void gather_rows_kernel(const double* B, int64_t ldb,
                                                          int64_t psb, const int32_t* perm,
                                                          int64_t n, int64_t nrhs, double* X) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t i = e / nrhs, c = e % nrhs;
  const int64_t src = (int64_t)perm[i] * ldb + c;
  X[e] = B[src];
  X[n * nrhs + e] = B[psb + src];
}

__global__ __launch_bounds__(256) void scatter_rows_kernel(const double* X, int64_t n,
                                                           int64_t nrhs, double* B, int64_t ldb,
                                                           int64_t psb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t i = e / nrhs, c = e % nrhs;
  B[i * ldb + c] = X[e];
  B[psb + i * ldb + c] = X[n * nrhs + e];
}

constexpr int kTB = 64;  // block size of the blocked triangular solves

// Forward (lower, unit) or backward (upper) step for block I of X (n x nrhs,
// nrhs <= 16).  Every workgroup solves the diagonal block redundantly (one
// wave per right-hand side, lane = row); the workgroup of block I stores it,
// every other workgroup W updates its rows X_W -= T_WI X_I.  The diagonal
// block, T_WI, X_I and X_W are all requested from memory before any of them
// is used (one round trip), and staged in LDS.  In the solve, lane i keeps
// x_i as an unrenormalised pair (s, r); step k renormalises x_k, broadcasts
// it with readlane, and the other lanes subtract T_ik x_k (TwoSum of the high
// product into s, low parts and TwoSum errors into r).  The backward solve
// multiplies by the diagonal's DD reciprocals, formed by all lanes at once
// before the sequential steps begin.
// Lower: blocks W > I are blockIdx.x + 1 + I; upper: W = blockIdx.x - 1 ... .
__global__ __launch_bounds__(1024) void trsv_block_kernel(const double* T, int64_t ldt,
                                                          int64_t pst, double* X, int64_t n,
                                                          int64_t nrhs, int64_t I, int upper) {
  __shared__ double Th[kTB][kTB + 1], Tl[kTB][kTB + 1];
  __shared__ double Wh[kTB][kTB + 1], Wl[kTB][kTB + 1];
  __shared__ double Xh[kTB][17], Xl[kTB][17];
  const int64_t nb = (n + kTB - 1) / kTB;
  const int64_t Wb = upper ? (I - (int64_t)blockIdx.x) : (I + (int64_t)blockIdx.x);
  if (Wb < 0 || Wb >= nb) return;
  const int64_t i0 = I * kTB, w0 = Wb * kTB;
  const int rows = (int)(n - i0 < kTB ? n - i0 : kTB);
  const int wrows = (int)(n - w0 < kTB ? n - w0 : kTB);
  const bool upd = Wb != I;
  const int t = threadIdx.x, lane = t % 64, wave = t / 64;
  const int nr = (int)nrhs;
  const int64_t psx = n * nrhs;
  constexpr int kPer = kTB * kTB / 1024;  // 4 tile elements per thread
  double dh[kPer], dl[kPer], oh[kPer], ol[kPer];
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const int e = t + 1024 * j, i = e / kTB, k = e % kTB;
    const bool in = i < rows && k < rows;
    const int64_t o = (i0 + (in ? i : 0)) * ldt + i0 + (in ? k : 0);
    dh[j] = T[o];
    dl[j] = T[pst + o];
    if (!in) {
      dh[j] = i == k ? 1.0 : 0.0;
      dl[j] = 0.0;
    }
    const bool win = upd && i < wrows && k < rows;
    const int64_t ow = (w0 + (win ? i : 0)) * ldt + i0 + (win ? k : 0);
    oh[j] = win ? T[ow] : 0.0;
    ol[j] = win ? T[pst + ow] : 0.0;
  }
  // X_I (as staged) and this thread's entry of X_W
  const int xi = t / 16, xc = t % 16;
  const bool xin = xi < rows && xc < nr;
  const double xih = xin ? X[(i0 + xi) * nrhs + xc] : 0.0;
  const double xil = xin ? X[psx + (i0 + xi) * nrhs + xc] : 0.0;
  const int ui = nr > 0 ? t / nr : 0, uc = nr > 0 ? t % nr : 0;
  const bool uin = upd && t < wrows * nr;
  const int64_t xo = (w0 + (uin ? ui : 0)) * nrhs + (uin ? uc : 0);
  const double xwh = uin ? X[xo] : 0.0, xwl = uin ? X[psx + xo] : 0.0;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const int e = t + 1024 * j, i = e / kTB, k = e % kTB;
    Th[i][k] = dh[j];
    Tl[i][k] = dl[j];
    Wh[i][k] = oh[j];
    Wl[i][k] = ol[j];
  }
  Xh[xi][xc] = xih;
  Xl[xi][xc] = xil;
  __syncthreads();
  if (wave < nr) {
    double s = Xh[lane][wave], r = Xl[lane][wave];
    if (!upper) {
      for (int k = 0; k < rows - 1; k++) {
        double kh, kl;
        two_sum(readlane_f64(s, k), readlane_f64(r, k), kh, kl);
        if (lane > k && lane < rows) {
          const double th = Th[lane][k], tl = Tl[lane][k];
          const double p = th * kh;
          const double pe = fma(th, kl, fma(tl, kh, fma(th, kh, -p)));
          double e;
          two_sum(s, -p, s, e);
          r += e - pe;
        }
      }
    } else {
      // reciprocals of the diagonal, all lanes at once
      const dd_t inv = lane < rows ? dd_div(dd_t{1.0, 0.0}, dd_t{Th[lane][lane], Tl[lane][lane]})
                                   : dd_t{0.0, 0.0};
      for (int k = rows - 1; k >= 0; k--) {
        dd_t xk;
        two_sum(readlane_f64(s, k), readlane_f64(r, k), xk.hi, xk.lo);
        xk = dd_mul(xk, dd_t{readlane_f64(inv.hi, k), readlane_f64(inv.lo, k)});
        if (lane == k) {
          s = xk.hi;
          r = xk.lo;
        } else if (lane < k) {
          const double th = Th[lane][k], tl = Tl[lane][k];
          const double p = th * xk.hi;
          const double pe = fma(th, xk.lo, fma(tl, xk.hi, fma(th, xk.hi, -p)));
          double e;
          two_sum(s, -p, s, e);
          r += e - pe;
        }
      }
    }
    double h, l;
    two_sum(s, r, h, l);
    Xh[lane][wave] = h;
    Xl[lane][wave] = l;
  }
  __syncthreads();
  if (!upd) {
    if (xin) {
      X[(i0 + xi) * nrhs + xc] = Xh[xi][xc];
      X[psx + (i0 + xi) * nrhs + xc] = Xl[xi][xc];
    }
    return;
  }
  // update rows of block Wb: X_W -= T_W,I X_I (one thread per entry)
  if (uin) {
    double s = 0.0, err = 0.0;
    for (int k = 0; k < rows; k++) {
      const double ah = Wh[ui][k], al = Wl[ui][k], bh = Xh[k][uc], bl = Xl[k][uc];
      const double p = ah * bh;
      const double q = fma(ah, bl, fma(al, bh, fma(ah, bh, -p)));
      double e2;
      two_sum(s, p, s, e2);
      err += e2 + q;
    }
    dd_t d;
    two_sum(s, err, d.hi, d.lo);
    const dd_t x = dd_sub(dd_t{xwh, xwl}, d);
    X[xo] = x.hi;
    X[psx + xo] = x.lo;
  }
}

}  // namespace

// ---- launchers ---------------------------------------------------------------

int launch_lu_init(int32_t* info, int32_t* perm, int64_t n, hipStream_t s) {
  prof_begin(s);
  hipLaunchKernelGGL(lu_init_kernel, dim3((unsigned)((n + 256) / 256)), dim3(256), 0, s, info,
                     perm, n);
  prof_record("lu_init_kernel", s);
  return check_launch("lu_init_kernel");
}

// Strip width for an m-row strip: the strip lives in registers, 1024 threads
// of at most 128 registers each, so taller strips are narrower.
// Strip shape by panel height: threads, rows per thread, strip width.  The
// register tile (RPT x W DD values) stays within what one thread can hold.
int getf2_width(int64_t m) { return m <= 2048 ? 8 : (m <= 4096 ? 4 : 2); }

int launch_getf2(double* A, int64_t lda, int64_t ps, int64_t r0, int64_t m, int64_t c0, int w,
                 int32_t* ipiv, int32_t* info, int pivot, hipStream_t s) {
  if (m <= 0 || w <= 0) return 0;
  if (w > getf2_width(m)) return set_error(4, "getf2 strip too wide");
#define GETF2(T, R, W)                                                                          \
  do {                                                                                          \
    prof_begin(s);                                                                              \
    hipLaunchKernelGGL((getf2_kernel<T, R, W>), dim3(1), dim3(T), 0, s, A, lda, ps, r0, m, c0, \
                       w, ipiv, info, pivot);                                                   \
    prof_record("getf2_kernel", s);                                                            \
  } while (0)
  if (m <= 256) GETF2(256, 1, 8);
  else if (m <= 512) GETF2(512, 1, 8);
  else if (m <= 1024) GETF2(1024, 1, 8);
  else if (m <= 2048) GETF2(1024, 2, 8);
  else if (m <= 4096) GETF2(512, 8, 4);
  else if (m <= 8192) GETF2(1024, 8, 2);
  else return set_error(4, "LU of more than 8192 rows is not supported");
#undef GETF2
  return check_launch("getf2_kernel");
}

int launch_laswp(double* A, int64_t lda, int64_t ps, int64_t n_cols, int64_t skip0,
                 int64_t skip1, int64_t k0, int64_t k1, const int32_t* ipiv, int32_t* perm,
                 hipStream_t s) {
  if (k1 <= k0) return 0;
  prof_begin(s);
  hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)((n_cols + 1 + 255) / 256)), dim3(256), 0, s,
                     A, lda, ps, n_cols, skip0, skip1, k0, k1, ipiv, perm);
  prof_record("laswp_kernel", s);
  return check_launch("laswp_kernel");
}

int launch_trsm_wave(double* A, int64_t lda, int64_t ps, int64_t r0, int64_t c0, int nb,
                     int64_t x0, int64_t ncols, hipStream_t s) {
  if (nb <= 0 || ncols <= 0) return 0;
  if (nb > kTrsmRows) return set_error(4, "trsm_wave: block too large");
  // enough workgroups to reach every compute unit before stacking columns
  int64_t cpb = (ncols + 255) / 256;
  if (cpb > kTrsmCols) cpb = kTrsmCols;
  if (cpb > ncols) cpb = ncols;
  const int64_t blocks = (ncols + cpb - 1) / cpb;
  prof_begin(s);
  hipLaunchKernelGGL(trsm_wave_kernel, dim3((unsigned)blocks), dim3((unsigned)(64 * cpb)), 0, s,
                     A, lda, ps, r0, c0, nb, x0, ncols);
  prof_record("trsm_wave_kernel", s);
  return check_launch("trsm_wave_kernel");
}

int launch_lu_update(const double* A, const double* B, double* C, int64_t ld, int64_t ps,
                     int64_t m, int64_t n, int64_t l, hipStream_t s) {
  if (m <= 0 || n <= 0 || l <= 0) return 0;
  const int64_t blocks = (m * n + 255) / 256;
  if (blocks > INT32_MAX) return set_error(4, "lu_update: grid too large");
  prof_begin(s);
  hipLaunchKernelGGL(lu_update_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, B, C, ld, ps, m,
                     n, l);
  prof_record("lu_update_kernel", s);
  return check_launch("lu_update_kernel");
}

int launch_perm_from_ipiv(const int32_t* ipiv, int64_t n, int32_t* perm, hipStream_t s) {
  prof_begin(s);
  hipLaunchKernelGGL(perm_from_ipiv_kernel, dim3(1), dim3(64), 0, s, ipiv, n, perm);
  prof_record("perm_from_ipiv_kernel", s);
  return check_launch("perm_from_ipiv_kernel");
}

int launch_gather_rows(const double* B, int64_t ldb, int64_t psb, const int32_t* perm, int64_t n,
                       int64_t nrhs, double* X, hipStream_t s) {
  prof_begin(s);
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((n * nrhs + 255) / 256)), dim3(256), 0,
                     s, B, ldb, psb, perm, n, nrhs, X);
  prof_record("gather_rows_kernel", s);
  return check_launch("gather_rows_kernel");
}

int launch_scatter_rows(const double* X, int64_t n, int64_t nrhs, double* B, int64_t ldb,
                        int64_t psb, hipStream_t s) {
  prof_begin(s);
  hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)((n * nrhs + 255) / 256)), dim3(256), 0,
                     s, X, n, nrhs, B, ldb, psb);
  prof_record("scatter_rows_kernel", s);
  return check_launch("scatter_rows_kernel");
}

int launch_trsv_blocks(const double* T, int64_t ldt, int64_t pst, double* X, int64_t n,
                       int64_t nrhs, int upper, hipStream_t s) {
  const int64_t nb = (n + kTB - 1) / kTB;
  if (nrhs > 16) return set_error(4, "at most 16 right-hand sides per solve call");
  for (int64_t step = 0; step < nb; step++) {
    const int64_t I = upper ? nb - 1 - step : step;
    const int64_t blocks = upper ? I + 1 : nb - I;
    prof_begin(s);
    hipLaunchKernelGGL(trsv_block_kernel, dim3((unsigned)blocks), dim3(1024), 0, s, T, ldt, pst,
                       X, n, nrhs, I, upper);
    prof_record("trsv_block_kernel", s);
    int rc = check_launch("trsv_block_kernel");
    if (rc) return rc;
  }
  return 0;
}

}  // namespace ddqd
