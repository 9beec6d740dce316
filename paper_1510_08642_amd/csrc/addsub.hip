// Fused add/sub kernels of one Strassen or Strassen-Winograd level.
//
// The paper's Strassen and Winograd products (Sec. 2; its figures of the
// parallel schemes are not available) are read as the textbook formulas.
// With X = [X11 X12; X21 X22] split into quadrants:
//
// Strassen (1969), operands of the seven products M1..M7:
//   left   A11+A22, A21+A22, A11, A22, A11+A12, A21-A11, A12-A22
//   right  B11+B22, B11, B12-B22, B21-B11, B22, B11+B12, B21+B22
//   C11 = M1+M4-M5+M7, C12 = M3+M5, C21 = M2+M4, C22 = M1-M2+M3+M6
// Strassen-Winograd (7 products, 15 additions), products P1..P7:
//   S1 = A21+A22, S2 = S1-A11, S3 = A11-A21, S4 = A12-S2
//   T1 = B12-B11, T2 = B22-T1, T3 = B22-B12, T4 = T2-B21
//   left   A11, A12, S4, A22, S1, S2, S3
//   right  B11, B21, B22, T4, T1, T2, T3
//   U2 = P1+P6, U3 = U2+P7, U4 = U2+P5
//   C11 = P1+P2, C12 = U4+P3, C21 = U3-P4, C22 = U3+P5
//
// One pre-add kernel per operand side reads the four quadrants of every
// parent once and writes all seven operands of its children (chains such as
// S1 -> S2 -> S4 stay in registers); one post-add kernel reads the seven
// products once and writes the four quadrants of the parent, applying
// C := beta*C + alpha*result at the top level.  At the top level the operands
// are also equilibrated: row r of A is scaled by 2^-ea[r] and column c of B by
// 2^-fb[c] as they are read (exact), and the result is scaled back by
// 2^(ea[r] + fb[c]), so the sums never mix rows or columns of different
// magnitude.  All sums are accurate DD
// (or QD) additions.  These kernels are HBM-bound: per output element a
// pre-add moves 4 reads + 7 writes, a post-add 7 reads + 4 writes (+4 reads
// when beta = 1), P doubles each.
#include "common.hpp"
#include "ddqd.h"
#include "eft.hpp"
#include "qd.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

// expo (top level only, else NULL): the equilibration exponents, per row of
// A (side 0) or per column of B (side 1); each input is scaled by 2^-expo.
// src_rows x src_cols is the part of the 2 rows x 2 cols source that exists
// (the caller's matrix, padded up to an even split at every level): entries
// outside it are zeros.
template <class N>
__global__ __launch_bounds__(256) void preadd_kernel(CMat src, Mat dst, int64_t rows,
                                                     int64_t cols, int64_t src_rows,
                                                     int64_t src_cols, int algo, int side,
                                                     const int* expo) {
  using T = typename N::T;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t p = blockIdx.y;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e % cols;
  const double* s = src.p + p * src.bstride;
  const bool r1 = i < src_rows, r2 = i + rows < src_rows;
  const bool c1 = j < src_cols, c2 = j + cols < src_cols;
  T x11{}, x12{}, x21{}, x22{};
  if (r1 && c1) x11 = N::load(s, src.ps, i * src.ld + j);
  if (r1 && c2) x12 = N::load(s, src.ps, i * src.ld + j + cols);
  if (r2 && c1) x21 = N::load(s, src.ps, (i + rows) * src.ld + j);
  if (r2 && c2) x22 = N::load(s, src.ps, (i + rows) * src.ld + j + cols);
  if (expo) {
    if (side == 0) {  // rows i and i + rows
      if (r1) x11 = N::scale(x11, -expo[i]);
      if (r1) x12 = N::scale(x12, -expo[i]);
      if (r2) x21 = N::scale(x21, -expo[i + rows]);
      if (r2) x22 = N::scale(x22, -expo[i + rows]);
    } else {  // columns j and j + cols
      if (c1) x11 = N::scale(x11, -expo[j]);
      if (c1) x21 = N::scale(x21, -expo[j]);
      if (c2) x12 = N::scale(x12, -expo[j + cols]);
      if (c2) x22 = N::scale(x22, -expo[j + cols]);
    }
  }
  T o[7];
  if (algo == 2) {  // Strassen
    if (side == 0) {
      o[0] = N::add(x11, x22);
      o[1] = N::add(x21, x22);
      o[2] = x11;
      o[3] = x22;
      o[4] = N::add(x11, x12);
      o[5] = N::sub(x21, x11);
      o[6] = N::sub(x12, x22);
    } else {
      o[0] = N::add(x11, x22);
      o[1] = x11;
      o[2] = N::sub(x12, x22);
      o[3] = N::sub(x21, x11);
      o[4] = x22;
      o[5] = N::add(x11, x12);
      o[6] = N::add(x21, x22);
    }
  } else {  // Winograd
    if (side == 0) {
      T s1 = N::add(x21, x22);
      T s2 = N::sub(s1, x11);
      T s3 = N::sub(x11, x21);
      T s4 = N::sub(x12, s2);
      o[0] = x11;
      o[1] = x12;
      o[2] = s4;
      o[3] = x22;
      o[4] = s1;
      o[5] = s2;
      o[6] = s3;
    } else {
      T t1 = N::sub(x12, x11);
      T t2 = N::sub(x22, t1);
      T t3 = N::sub(x22, x12);
      T t4 = N::sub(t2, x21);
      o[0] = x11;
      o[1] = x21;
      o[2] = x22;
      o[3] = t4;
      o[4] = t1;
      o[5] = t2;
      o[6] = t3;
    }
  }
#pragma unroll
  for (int t = 0; t < 7; t++) N::store(dst.p + (7 * p + t) * dst.bstride, dst.ps, i * dst.ld + j, o[t]);
}

// ea, fb (top level only, else NULL): equilibration exponents of A's rows and
// B's columns; entry (r, c) of the result is scaled by 2^(ea[r] + fb[c]).
// Only the dst_rows x dst_cols part of the 2 rows x 2 cols result is written
// (the rest is the padding's).
template <class N>
__global__ __launch_bounds__(256) void postadd_kernel(CMat prod, Mat dst, int64_t rows,
                                                      int64_t cols, int64_t dst_rows,
                                                      int64_t dst_cols, int algo, int alpha,
                                                      int beta, const int* ea, const int* fb) {
  using T = typename N::T;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t p = blockIdx.y;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e % cols;
  T M[7];
#pragma unroll
  for (int t = 0; t < 7; t++)
    M[t] = N::load(prod.p + (7 * p + t) * prod.bstride, prod.ps, i * prod.ld + j);
  T c[4];
  if (algo == 2) {
    c[0] = N::add(N::sub(N::add(M[0], M[3]), M[4]), M[6]);
    c[1] = N::add(M[2], M[4]);
    c[2] = N::add(M[1], M[3]);
    c[3] = N::add(N::add(N::sub(M[0], M[1]), M[2]), M[5]);
  } else {
    T u2 = N::add(M[0], M[5]);
    T u3 = N::add(u2, M[6]);
    T u4 = N::add(u2, M[4]);
    c[0] = N::add(M[0], M[1]);
    c[1] = N::add(u4, M[2]);
    c[2] = N::sub(u3, M[3]);
    c[3] = N::add(u3, M[4]);
  }
  double* d = dst.p + p * dst.bstride;
  const int64_t off[4] = {i * dst.ld + j, i * dst.ld + j + cols, (i + rows) * dst.ld + j,
                          (i + rows) * dst.ld + j + cols};
#pragma unroll
  for (int q = 0; q < 4; q++) {
    if (i + (q >> 1) * rows >= dst_rows || j + (q & 1) * cols >= dst_cols) continue;
    T v = alpha < 0 ? N::neg(c[q]) : c[q];
    if (ea) v = N::scale(v, ea[i + (q >> 1) * rows] + fb[j + (q & 1) * cols]);
    if (beta) v = N::add(N::load(d, dst.ps, off[q]), v);
    N::store(d, dst.ps, off[q], v);
  }
}

}  // namespace

template <class N>
int launch_preadd(CMat src, Mat dst, int64_t rows, int64_t cols, int64_t src_rows,
                  int64_t src_cols, int64_t parents, int algo, int side, const int* expo,
                  hipStream_t stream) {
  if (rows <= 0 || cols <= 0 || parents <= 0) return 0;
  if (parents > 65535) return set_error(4, "too many recursion parents");
  dim3 grid((unsigned)((rows * cols + 255) / 256), (unsigned)parents);
  prof_begin(stream);
  hipLaunchKernelGGL(preadd_kernel<N>, grid, dim3(256), 0, stream, src, dst, rows, cols,
                     src_rows, src_cols, algo, side, expo);
  prof_record("preadd_kernel", stream);
  return check_launch("preadd_kernel");
}

template <class N>
int launch_postadd(CMat prod, Mat dst, int64_t rows, int64_t cols, int64_t dst_rows,
                   int64_t dst_cols, int64_t parents, int algo, int alpha, int beta,
                   const int* ea, const int* fb, hipStream_t stream) {
  if (rows <= 0 || cols <= 0 || parents <= 0) return 0;
  if (parents > 65535) return set_error(4, "too many recursion parents");
  dim3 grid((unsigned)((rows * cols + 255) / 256), (unsigned)parents);
  prof_begin(stream);
  hipLaunchKernelGGL(postadd_kernel<N>, grid, dim3(256), 0, stream, prod, dst, rows, cols,
                     dst_rows, dst_cols, algo, alpha, beta, ea, fb);
  prof_record("postadd_kernel", stream);
  return check_launch("postadd_kernel");
}

// Equilibration exponents: e such that the largest |leading component| of
// row r of A, or column c of B, lies in [2^(e-1), 2^e); kNoExp, far below any
// exponent, for an all-zero row or column: its inputs stay zero when scaled,
// and the rounding residue the recursion leaves in its (exactly zero) row or
// column of the product is scaled away to zero.
constexpr int kNoExp = -(1 << 20);

// One wave per row of A, all of a lane's loads in flight before the
// reduction; the same launch presets B's column exponents to kNoExp.
__global__ __launch_bounds__(256) void row_exponent_kernel(CMat A, int64_t m, int64_t l, int* e,
                                                           int* fb, int64_t n) {
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * 256)
    fb[c] = kNoExp;
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (r >= m) return;
  const double* p = A.p + r * A.ld;
  double mx = 0.0;
  int64_t k = lane;
  for (; k + 960 < l; k += 1024) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; q++) v[q] = p[k + 64 * q];
#pragma unroll
    for (int q = 0; q < 16; q++) mx = fmax(mx, fabs(v[q]));
  }
  for (; k < l; k += 64) mx = fmax(mx, fabs(p[k]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) {
    int ex = kNoExp;
    if (mx > 0.0) frexp(mx, &ex);
    e[r] = ex;
  }
}

// A workgroup takes 64 columns by a 32-row slab of B and raises each column's
// exponent to its slab maximum's (atomic maximum; exponents are monotone in
// |x|, so the maximum of the slab exponents is the column maximum's, in any
// order).  All-zero columns keep kNoExp.
__global__ __launch_bounds__(256) void col_exponent_kernel(CMat B, int64_t l, int64_t n,
                                                           int* e) {
  __shared__ double red[4][64];
  const int c_in = threadIdx.x % 64, r = threadIdx.x / 64;
  const int64_t c = (int64_t)blockIdx.x * 64 + c_in;
  const int64_t k0 = (int64_t)blockIdx.y * 32 + r * 8;
  double mx = 0.0;
  if (c < n) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; q++) v[q] = k0 + q < l ? B.p[(k0 + q) * B.ld + c] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; q++) mx = fmax(mx, fabs(v[q]));
  }
  red[r][c_in] = mx;
  __syncthreads();
  if (r == 0 && c < n) {
    mx = fmax(fmax(red[0][c_in], red[1][c_in]), fmax(red[2][c_in], red[3][c_in]));
    if (mx > 0.0) {
      int ex;
      frexp(mx, &ex);
      atomicMax(&e[c], ex);
    }
  }
}

int launch_exponents(CMat A, CMat B, int64_t m, int64_t n, int64_t l, int* ea, int* fb,
                     hipStream_t stream) {
  if ((l + 31) / 32 > 65535) return set_error(DDQD_E_UNSUPPORTED, "inner dimension too large");
  prof_begin(stream);
  hipLaunchKernelGGL(row_exponent_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, stream,
                     A, m, l, ea, fb, n);
  prof_record("row_exponent_kernel", stream);
  int rc = check_launch("row_exponent_kernel");
  if (rc) return rc;
  prof_begin(stream);
  hipLaunchKernelGGL(col_exponent_kernel, dim3((unsigned)((n + 63) / 64), (unsigned)((l + 31) / 32)),
                     dim3(256), 0, stream, B, l, n, fb);
  prof_record("col_exponent_kernel", stream);
  return check_launch("col_exponent_kernel");
}

template int launch_preadd<DDNum>(CMat, Mat, int64_t, int64_t, int64_t, int64_t, int64_t, int,
                                  int, const int*, hipStream_t);
template int launch_postadd<DDNum>(CMat, Mat, int64_t, int64_t, int64_t, int64_t, int64_t, int,
                                   int, int, const int*, const int*, hipStream_t);
template int launch_preadd<QDNum>(CMat, Mat, int64_t, int64_t, int64_t, int64_t, int64_t, int,
                                  int, const int*, hipStream_t);
template int launch_postadd<QDNum>(CMat, Mat, int64_t, int64_t, int64_t, int64_t, int64_t, int,
                                   int, int, const int*, const int*, hipStream_t);

}  // namespace ddqd
