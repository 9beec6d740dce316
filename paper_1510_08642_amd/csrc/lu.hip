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
// i < 0 marks "no candidate".
__device__ __forceinline__ bool better(dd_t x, int i, dd_t y, int j) {
  if (i < 0) return false;
  if (j < 0) return true;
  const int c = dd_abs_cmp(x, y);
  return c > 0 || (c == 0 && i < j);
}

// ---- getf2: factor an m x w strip (w <= W) held in registers ---------------
// One 1024-thread workgroup; thread t owns local rows t + 1024 q, q < RPT.
// Column by column: pivot search (wave shuffles, then LDS), interchange of the
// two rows inside the strip, division of the column below the pivot by the
// pivot (DD division), rank-1 update of the strip's remaining columns.
// ipiv[c0 + c] receives the global (0-based) pivot row; info the first
// 1-based global column whose pivot is exactly zero, if none was recorded
// before.  Other columns of the matrix are interchanged later by laswp.
template <int RPT, int W>
__global__ __launch_bounds__(1024) void getf2_kernel(double* A, int64_t lda, int64_t ps,
                                                      int64_t r0, int64_t m, int64_t c0, int w,
                                                      int32_t* ipiv, int32_t* info, int pivot) {
  __shared__ double s_hi[16], s_lo[16];
  __shared__ int s_idx[16];
  __shared__ double rowp_hi[W], rowp_lo[W], rowc_hi[W], rowc_lo[W];
  __shared__ int s_p;
  const int t = threadIdx.x, lane = t % 64, wave = t / 64;
  dd_t v[RPT][W];
#pragma unroll
  for (int q = 0; q < RPT; q++)
#pragma unroll
    for (int k = 0; k < W; k++) {
      const int64_t i = t + 1024 * q;
      v[q][k] = (i < m && k < w) ? ld_dd(A, ps, (r0 + i) * lda + c0 + k) : dd_t{0.0, 0.0};
    }
  for (int c = 0; c < w; c++) {
    // 1. pivot search among local rows >= c
    dd_t best{0.0, 0.0};
    int bi = -1;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const int i = t + 1024 * q;
      if (i >= c && i < m) {
        dd_t x;
#pragma unroll
        for (int k = 0; k < W; k++)
          if (k == c) x = dd_abs(v[q][k]);
        if (better(x, i, best, bi)) {
          best = x;
          bi = i;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      dd_t o{__shfl_xor(best.hi, off, 64), __shfl_xor(best.lo, off, 64)};
      int oi = __shfl_xor(bi, off, 64);
      if (better(o, oi, best, bi)) {
        best = o;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_hi[wave] = best.hi;
      s_lo[wave] = best.lo;
      s_idx[wave] = bi;
    }
    __syncthreads();
    if (t == 0) {
      dd_t b{s_hi[0], s_lo[0]};
      int p = s_idx[0];
      for (int z = 1; z < 16; z++) {
        dd_t o{s_hi[z], s_lo[z]};
        if (better(o, s_idx[z], b, p)) {
          b = o;
          p = s_idx[z];
        }
      }
      if (!pivot || p < 0) p = c;
      s_p = p;
      ipiv[c0 + c] = (int32_t)(r0 + p);
    }
    __syncthreads();
    const int p = s_p;
    // 2. interchange rows c and p of the strip through LDS
    const int qc = c / 1024, tc = c % 1024, qp = p / 1024, tp = p % 1024;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      if (t == tp && q == qp)
#pragma unroll
        for (int k = 0; k < W; k++) {
          rowp_hi[k] = v[q][k].hi;
          rowp_lo[k] = v[q][k].lo;
        }
      if (p != c && t == tc && q == qc)
#pragma unroll
        for (int k = 0; k < W; k++) {
          rowc_hi[k] = v[q][k].hi;
          rowc_lo[k] = v[q][k].lo;
        }
    }
    __syncthreads();
    if (p != c) {
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        if (t == tc && q == qc)
#pragma unroll
          for (int k = 0; k < W; k++) v[q][k] = dd_t{rowp_hi[k], rowp_lo[k]};
        if (t == tp && q == qp)
#pragma unroll
          for (int k = 0; k < W; k++) v[q][k] = dd_t{rowc_hi[k], rowc_lo[k]};
      }
    }
    // 3. the pivot row is now row c; its values are rowp
    const dd_t u{rowp_hi[c], rowp_lo[c]};
    if (t == 0 && u.hi == 0.0 && u.lo == 0.0 && *info == 0) *info = (int32_t)(c0 + c + 1);
    if (!(u.hi == 0.0 && u.lo == 0.0)) {
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const int i = t + 1024 * q;
        if (i > c && i < m) {
          dd_t l;
#pragma unroll
          for (int k = 0; k < W; k++)
            if (k == c) {
              l = dd_div(v[q][k], u);
              v[q][k] = l;
            }
#pragma unroll
          for (int k = 0; k < W; k++)
            if (k > c && k < w) v[q][k] = dd_sub(v[q][k], dd_mul(l, dd_t{rowp_hi[k], rowp_lo[k]}));
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RPT; q++)
#pragma unroll
    for (int k = 0; k < W; k++) {
      const int64_t i = t + 1024 * q;
      if (i < m && k < w) st_dd(A, ps, (r0 + i) * lda + c0 + k, v[q][k]);
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

// ---- small unit-lower triangular solve: X := L^-1 X ------------------------
// L = A[r0 .. r0+nb, c0 .. c0+nb) (unit diagonal, nb <= 16), X = the nb rows
// r0.. of columns [x0, x0 + ncols).  One thread per column.
__global__ __launch_bounds__(256) void trsm_small_kernel(double* A, int64_t lda, int64_t ps,
                                                         int64_t r0, int64_t c0, int nb,
                                                         int64_t x0, int64_t ncols) {
  __shared__ double Lh[16][16], Ll[16][16];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, k = e % nb;
    Lh[i][k] = A[(r0 + i) * lda + c0 + k];
    Ll[i][k] = A[ps + (r0 + i) * lda + c0 + k];
  }
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= ncols) return;
  dd_t x[16];
#pragma unroll
  for (int i = 0; i < 16; i++)
    x[i] = i < nb ? ld_dd(A, ps, (r0 + i) * lda + x0 + j) : dd_t{0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 16; k++)
#pragma unroll
    for (int i = k + 1; i < 16; i++)
      if (i < nb) x[i] = dd_sub(x[i], dd_mul(dd_t{Lh[i][k], Ll[i][k]}, x[k]));
#pragma unroll
  for (int i = 0; i < 16; i++)
    if (i < nb) st_dd(A, ps, (r0 + i) * lda + x0 + j, x[i]);
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
// wave per right-hand side, lane = row, values shared by shuffles); the
// workgroup of block I stores it, every other workgroup W updates its rows
// X_W -= T_WI X_I with a lazily accumulated DD dot product.
// Lower: blocks W > I are blockIdx.x + 1 + I; upper: W = blockIdx.x - 1 ... .
__global__ __launch_bounds__(1024) void trsv_block_kernel(const double* T, int64_t ldt,
                                                          int64_t pst, double* X, int64_t n,
                                                          int64_t nrhs, int64_t I, int upper) {
  __shared__ double Th[kTB][kTB + 1], Tl[kTB][kTB + 1];
  __shared__ double Xh[kTB][16], Xl[kTB][16];
  const int64_t nb = (n + kTB - 1) / kTB;
  const int64_t Wb = upper ? (I - (int64_t)blockIdx.x) : (I + (int64_t)blockIdx.x);
  if (Wb < 0 || Wb >= nb) return;
  const int64_t i0 = I * kTB, rows = n - i0 < kTB ? n - i0 : kTB;
  const int t = threadIdx.x, lane = t % 64, wave = t / 64;
  const int64_t psx = n * nrhs;
  for (int e = t; e < kTB * kTB; e += 1024) {
    const int i = e / kTB, k = e % kTB;
    const bool in = i < rows && k < rows;
    Th[i][k] = in ? T[(i0 + i) * ldt + i0 + k] : (i == k ? 1.0 : 0.0);
    Tl[i][k] = in ? T[pst + (i0 + i) * ldt + i0 + k] : 0.0;
  }
  for (int e = t; e < kTB * 16; e += 1024) {
    const int i = e / 16, c = e % 16;
    const bool in = i < rows && c < nrhs;
    Xh[i][c] = in ? X[(i0 + i) * nrhs + c] : 0.0;
    Xl[i][c] = in ? X[psx + (i0 + i) * nrhs + c] : 0.0;
  }
  __syncthreads();
  if (wave < nrhs) {
    dd_t x{Xh[lane][wave], Xl[lane][wave]};
    if (!upper) {
      for (int k = 0; k < kTB; k++) {
        dd_t xk{__shfl(x.hi, k, 64), __shfl(x.lo, k, 64)};
        if (lane > k) x = dd_sub(x, dd_mul(dd_t{Th[lane][k], Tl[lane][k]}, xk));
      }
    } else {
      for (int k = kTB - 1; k >= 0; k--) {
        if (lane == k) x = dd_div(x, dd_t{Th[k][k], Tl[k][k]});
        dd_t xk{__shfl(x.hi, k, 64), __shfl(x.lo, k, 64)};
        if (lane < k) x = dd_sub(x, dd_mul(dd_t{Th[lane][k], Tl[lane][k]}, xk));
      }
    }
    Xh[lane][wave] = x.hi;
    Xl[lane][wave] = x.lo;
  }
  __syncthreads();
  if (Wb == I) {
    for (int e = t; e < rows * nrhs; e += 1024) {
      const int i = e / (int)nrhs, c = e % (int)nrhs;
      X[(i0 + i) * nrhs + c] = Xh[i][c];
      X[psx + (i0 + i) * nrhs + c] = Xl[i][c];
    }
    return;
  }
  // update rows of block Wb: X_W -= T_W,I X_I
  const int64_t w0 = Wb * kTB, wrows = n - w0 < kTB ? n - w0 : kTB;
  for (int e = t; e < wrows * nrhs; e += 1024) {
    const int i = e / (int)nrhs, c = e % (int)nrhs;
    double s = 0.0, err = 0.0;
    for (int k = 0; k < rows; k++) {
      const int64_t o = (w0 + i) * ldt + i0 + k;
      const double ah = T[o], al = T[pst + o], bh = Xh[k][c], bl = Xl[k][c];
      double p = ah * bh;
      double q = __builtin_fma(ah, bh, -p);
      q = __builtin_fma(ah, bl, q);
      q = __builtin_fma(al, bh, q);
      double sn, e2;
      two_sum(s, p, sn, e2);
      s = sn;
      err = err + (e2 + q);
    }
    dd_t d;
    two_sum(s, err, d.hi, d.lo);
    const int64_t xo = (w0 + i) * nrhs + c;
    dd_t x = dd_sub(dd_t{X[xo], X[psx + xo]}, d);
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
int getf2_width(int64_t m) { return m <= 2048 ? 8 : (m <= 4096 ? 4 : 2); }

int launch_getf2(double* A, int64_t lda, int64_t ps, int64_t r0, int64_t m, int64_t c0, int w,
                 int32_t* ipiv, int32_t* info, int pivot, hipStream_t s) {
  if (m <= 0 || w <= 0) return 0;
  const int rpt = (int)((m + 1023) / 1024);
  if (w > getf2_width(m)) return set_error(4, "getf2 strip too wide");
#define GETF2(R, W)                                                                        \
  do {                                                                                     \
    prof_begin(s);                                                                         \
    hipLaunchKernelGGL((getf2_kernel<R, W>), dim3(1), dim3(1024), 0, s, A, lda, ps, r0, m, c0, \
                       w, ipiv, info, pivot);                                              \
    prof_record("getf2_kernel", s);                                                        \
  } while (0)
  if (rpt <= 1) GETF2(1, 8);
  else if (rpt <= 2) GETF2(2, 8);
  else if (rpt <= 4) GETF2(4, 4);
  else if (rpt <= 8) GETF2(8, 2);
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

int launch_trsm_small(double* A, int64_t lda, int64_t ps, int64_t r0, int64_t c0, int nb,
                      int64_t x0, int64_t ncols, hipStream_t s) {
  if (nb <= 0 || ncols <= 0) return 0;
  if (nb > 16) return set_error(4, "trsm_small: block too large");
  prof_begin(s);
  hipLaunchKernelGGL(trsm_small_kernel, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, s, A,
                     lda, ps, r0, c0, nb, x0, ncols);
  prof_record("trsm_small_kernel", s);
  return check_launch("trsm_small_kernel");
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
