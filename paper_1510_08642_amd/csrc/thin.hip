// Thin products: C := beta*C + alpha*A B where A has at most 32 rows or B at
// most 32 columns while K is long.  The Strassen/Winograd driver peels such
// products off orders that 2^L does not divide (the paper's Sec. 3 runs
// n = 1023 and 1025, where the peel is a single row and a single column).
// The Block kernels would give such a shape a few mostly idle 64x64 tiles,
// each running the whole K loop alone; these kernels spread K instead.
//
//  * few rows (m <= 32): a 512-thread workgroup owns 16 columns and R rows
//    of C; its 32 lane groups of 16 take interleaved K slices (k = s, s + 32,
//    ...), B read coalesced along the row, A's few rows read as broadcasts.
//    The 32 slice sums are added pairwise in LDS (a fixed tree).
//  * few columns (n <= 32): one wave per row of C and NC columns; the wave's
//    lanes take interleaved K (A's row read coalesced, B's few columns from
//    L2), then a butterfly of shuffles adds the 64 lane sums.
//
// Every sum is the multiply-add of the Block kernel of the same precision
// (DD: the lazy 12-operation dd_mac; QD: the order-bucket qd_mac), with the
// accumulators renormalised every 16 steps, and slice sums added by the
// accurate DD or QD addition: the bound of the Block product holds with l
// replaced by the longest slice plus the depth of the reduction tree.
#include "common.hpp"
#include "ddqd.h"
#include "qd.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

struct DDArith {
  using N = DDNum;
  using T = dd_t;
  static constexpr int P = 2;
  struct Acc {
    double s, e;
  };
  __device__ static Acc zero() { return Acc{0.0, 0.0}; }
  __device__ static void mac(Acc& x, const double* a, const double* b) {
    dd_mac(x.s, x.e, a[0], a[1], b[0], b[1]);
  }
  __device__ static void norm(Acc& x) { two_sum(x.s, x.e, x.s, x.e); }
  __device__ static T value(Acc x) {
    T v;
    two_sum(x.s, x.e, v.hi, v.lo);
    return v;
  }
  __device__ static T shfl_xor(T v, int m) {
    return T{__shfl_xor(v.hi, m, 64), __shfl_xor(v.lo, m, 64)};
  }
};

struct QDArith {
  using N = QDNum;
  using T = qd_t;
  static constexpr int P = 4;
  using Acc = qd_acc;
  __device__ static Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ static void mac(Acc& x, const double* a, const double* b) { qd_mac(x, a, b); }
  __device__ static void norm(Acc& x) { qd_renorm(x.s0, x.s1, x.s2, x.s3); }
  __device__ static T value(Acc x) {
    qd_renorm(x.s0, x.s1, x.s2, x.s3);
    return T{{x.s0, x.s1, x.s2, x.s3}};
  }
  __device__ static T shfl_xor(T v, int m) {
    return T{{__shfl_xor(v.c[0], m, 64), __shfl_xor(v.c[1], m, 64), __shfl_xor(v.c[2], m, 64),
              __shfl_xor(v.c[3], m, 64)}};
  }
};

constexpr int kRenorm = 16;  // multiply-adds between renormalisations

// ---- few rows ---------------------------------------------------------------
constexpr int kRowCols = 16;
constexpr int kRowThreads = 512;
constexpr int kSlices = kRowThreads / kRowCols;  // 32

template <class Ar, int R>
__global__ __launch_bounds__(kRowThreads) void thin_rows_kernel(GemmBatch g) {
  using T = typename Ar::T;
  using N = typename Ar::N;
  constexpr int P = Ar::P;
  // DD with R = 8 and QD with R = 4 fill 64 KB
  __shared__ T part[kSlices][R][kRowCols];
  const int c = threadIdx.x % kRowCols, sl = threadIdx.x / kRowCols;
  const int64_t j0 = (int64_t)blockIdx.x * kRowCols;
  const int64_t i0 = (int64_t)blockIdx.y * R;
  const int64_t j = j0 + c;
  const bool jok = j < g.n;
  typename Ar::Acc acc[R];
#pragma unroll
  for (int r = 0; r < R; r++) acc[r] = Ar::zero();
  for (int64_t k0 = sl; k0 < g.l; k0 += (int64_t)kRenorm * kSlices) {
#pragma unroll 4
    for (int u = 0; u < kRenorm; u++) {
      const int64_t k = k0 + (int64_t)u * kSlices;
      if (k >= g.l) break;
      double b[P], a[R][P];
#pragma unroll
      for (int q = 0; q < P; q++) b[q] = jok ? g.B.p[q * g.B.ps + k * g.B.ld + j] : 0.0;
#pragma unroll
      for (int r = 0; r < R; r++) {
        const bool ok = i0 + r < g.m;
#pragma unroll
        for (int q = 0; q < P; q++)
          a[r][q] = ok ? g.A.p[q * g.A.ps + (i0 + r) * g.A.ld + k] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < R; r++) Ar::mac(acc[r], a[r], b);
    }
#pragma unroll
    for (int r = 0; r < R; r++) Ar::norm(acc[r]);
  }
#pragma unroll
  for (int r = 0; r < R; r++) part[sl][r][c] = Ar::value(acc[r]);
  __syncthreads();
  for (int h = kSlices / 2; h >= 1; h /= 2) {
    for (int it = threadIdx.x; it < h * R * kRowCols; it += kRowThreads) {
      const int s = it / (R * kRowCols), rc = it % (R * kRowCols);
      T* x = &part[s][0][0] + rc;
      const T* y = &part[s + h][0][0] + rc;
      *x = N::add(*x, *y);
    }
    __syncthreads();
  }
  if (threadIdx.x < R * kRowCols) {
    const int r = threadIdx.x / kRowCols, cc = threadIdx.x % kRowCols;
    const int64_t i = i0 + r, jj = j0 + cc;
    if (i < g.m && jj < g.n) {
      T v = part[0][r][cc];
      if (g.alpha < 0) v = N::neg(v);
      const int64_t o = i * g.C.ld + jj;
      if (g.beta) v = N::add(N::load(g.C.p, g.C.ps, o), v);
      N::store(g.C.p, g.C.ps, o, v);
    }
  }
}

// ---- few columns --------------------------------------------------------------
constexpr int kColWaves = 4;

template <class Ar, int NC>
__global__ __launch_bounds__(64 * kColWaves) void thin_cols_kernel(GemmBatch g) {
  using T = typename Ar::T;
  using N = typename Ar::N;
  constexpr int P = Ar::P;
  const int lane = threadIdx.x % 64;
  const int64_t i = (int64_t)blockIdx.x * kColWaves + threadIdx.x / 64;
  const int64_t j0 = (int64_t)blockIdx.y * NC;
  if (i >= g.m) return;  // the whole wave: i is one row per wave
  typename Ar::Acc acc[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) acc[c] = Ar::zero();
  for (int64_t k0 = lane; k0 < g.l; k0 += (int64_t)kRenorm * 64) {
#pragma unroll 4
    for (int u = 0; u < kRenorm; u++) {
      const int64_t k = k0 + (int64_t)u * 64;
      if (k >= g.l) break;
      double a[P], b[NC][P];
#pragma unroll
      for (int q = 0; q < P; q++) a[q] = g.A.p[q * g.A.ps + i * g.A.ld + k];
#pragma unroll
      for (int c = 0; c < NC; c++) {
        const bool ok = j0 + c < g.n;
#pragma unroll
        for (int q = 0; q < P; q++) b[c][q] = ok ? g.B.p[q * g.B.ps + k * g.B.ld + j0 + c] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < NC; c++) Ar::mac(acc[c], a, b[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; c++) Ar::norm(acc[c]);
  }
  T v[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) v[c] = Ar::value(acc[c]);
#pragma unroll
  for (int off = 32; off >= 1; off /= 2)
#pragma unroll
    for (int c = 0; c < NC; c++) v[c] = N::add(v[c], Ar::shfl_xor(v[c], off));
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NC; c++) {
      if (j0 + c >= g.n) break;
      T w = g.alpha < 0 ? N::neg(v[c]) : v[c];
      const int64_t o = i * g.C.ld + j0 + c;
      if (g.beta) w = N::add(N::load(g.C.p, g.C.ps, o), w);
      N::store(g.C.p, g.C.ps, o, w);
    }
  }
}

template <class Ar, int R>
int rows_launch(const GemmBatch& g, hipStream_t s) {
  dim3 grid((unsigned)((g.n + kRowCols - 1) / kRowCols), (unsigned)((g.m + R - 1) / R));
  prof_begin(s);
  hipLaunchKernelGGL((thin_rows_kernel<Ar, R>), grid, dim3(kRowThreads), 0, s, g);
  prof_record("thin_rows_kernel", s);
  return check_launch("thin_rows_kernel");
}

template <class Ar, int NC>
int cols_launch(const GemmBatch& g, hipStream_t s) {
  dim3 grid((unsigned)((g.m + kColWaves - 1) / kColWaves), (unsigned)((g.n + NC - 1) / NC));
  prof_begin(s);
  hipLaunchKernelGGL((thin_cols_kernel<Ar, NC>), grid, dim3(64 * kColWaves), 0, s, g);
  prof_record("thin_cols_kernel", s);
  return check_launch("thin_cols_kernel");
}

// R (or NC): the smallest power of two covering d, at most cap
int width(int64_t d, int cap) {
  int w = 1;
  while (w < d && w < cap) w *= 2;
  return w;
}

template <class Ar, int Cap>
int launch_thin_p(const GemmBatch& g, hipStream_t s) {
  if (g.m <= g.n) {
    switch (width(g.m, Cap)) {
      case 1: return rows_launch<Ar, 1>(g, s);
      case 2: return rows_launch<Ar, 2>(g, s);
      case 4: return rows_launch<Ar, 4>(g, s);
      default: return rows_launch<Ar, Cap>(g, s);
    }
  }
  switch (width(g.n, Cap)) {
    case 1: return cols_launch<Ar, 1>(g, s);
    case 2: return cols_launch<Ar, 2>(g, s);
    case 4: return cols_launch<Ar, 4>(g, s);
    default: return cols_launch<Ar, Cap>(g, s);
  }
}

}  // namespace

constexpr int64_t kThinMax = 32;

bool thin_shape(const GemmBatch& g) {
  return g.batch == 1 && (g.m <= kThinMax || g.n <= kThinMax);
}

// Few rows (m <= n) or few columns; a single product (batch 1).
int launch_thin(int P, const GemmBatch& g, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0) return DDQD_OK;
  if (!thin_shape(g)) return set_error(DDQD_E_UNSUPPORTED, "not a thin product");
  if (g.n > 2147483647LL * kRowCols || g.m > 2147483647LL * kColWaves)
    return set_error(DDQD_E_UNSUPPORTED, "grid too large");
  return P == 2 ? launch_thin_p<DDArith, 8>(g, s) : launch_thin_p<QDArith, 4>(g, s);
}

}  // namespace ddqd
