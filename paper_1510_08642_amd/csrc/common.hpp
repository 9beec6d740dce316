// Shared host/device structures of libddqd: strided batches of matrices in
// plane layout, launch helpers and the XCD-aware block remap.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddqd {

// A batch of equally shaped plane-layout matrices: component c of element
// (i, j) of matrix b is p[b*bstride + c*ps + i*ld + j].
struct CMat {
  const double* p;
  int64_t ld, ps, bstride;
};
struct Mat {
  double* p;
  int64_t ld, ps, bstride;
};

// One batched product: C_b := beta*C_b + alpha*A_b B_b for b < batch.
struct GemmBatch {
  int64_t m, n, l;
  int alpha, beta;
  CMat A, B;
  Mat C;
  int64_t batch;
};

inline CMat cview(const Mat& M) { return CMat{M.p, M.ld, M.ps, M.bstride}; }

// Unrelated products of one grouped launch (kernel argument, <= 4 KB):
// problem p owns tiles [start[p], start[p+1]) of the concatenated list.
constexpr int kMaxGroup = 24;
struct GroupArgs {
  int count;
  GemmBatch g[kMaxGroup];
  int64_t start[kMaxGroup + 1];
};

// Steps of a factored panel whose triangular solve X := L^-1 X is still to be
// stored (kernel argument): L at (r0[q], r0[q]), nb[q] rows; X = those rows of
// columns [x0[q], x0[q] + nc[q]).
constexpr int kTrsmNodesMax = 64;
struct TrsmNodes {
  int count;
  int r0[kTrsmNodesMax], nb[kTrsmNodesMax], x0[kTrsmNodesMax], nc[kTrsmNodesMax];
};

// Block rows of the triangular solves of getrs (DD, QD), and the flag words
// their chained launches use: one per block row of the smaller block, and
// one for the wait-limit record.
constexpr int kTrsvBlockDD = 64, kTrsvBlockQD = 32;
constexpr int64_t trsv_flag_words(int64_t n) { return (n + kTrsvBlockQD - 1) / kTrsvBlockQD + 1; }

// Round-robin dispatch places workgroup b on XCD b % 8.  This permutation
// gives each XCD one contiguous range of logical tiles, so tiles that share
// operand panels share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblk) {
  constexpr int64_t kXcd = 8;
  int64_t x = b % kXcd, local = b / kXcd;
  int64_t q = nblk / kXcd, r = nblk % kXcd;
  return x * q + (x < r ? x : r) + local;
}

// Row and column of logical tile t in a rows x cols grid whose tiles are
// taken in bands of `band` rows, column by column inside a band.  The tiles
// one XCD runs at the same time (consecutive t) then form a compact block
// (band rows by a few columns) that shares A row panels and B column panels
// in its L2, instead of one long row.
__device__ __forceinline__ void banded_tile(int64_t t, int64_t rows, int64_t cols, int64_t band,
                                            int64_t& r, int64_t& c) {
  const int64_t per = band * cols;
  const int64_t first = (t / per) * band;
  const int64_t h = rows - first < band ? rows - first : band;
  const int64_t k = t % per;
  r = first + k % h;
  c = k / h;
}

// Host-side status plumbing shared by the launchers.
int set_error(int status, const char* fmt, ...);
int check_launch(const char* what);

// Optional per-kernel timing (ddqd_profile_enable): when on, every launch is
// bracketed by HIP events recorded on its stream; no effect when off.
void prof_begin(hipStream_t s);
void prof_record(const char* kernel, hipStream_t s);

// The same timing for the kernels the roofline figures are taken from, read
// at the kernel's own start and end: the launch carries the two events
// (hipExtLaunchKernel), so no marker sits between them and the kernel.
struct ProfEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
ProfEvents prof_events(hipStream_t s);  // null events when timing is off
void prof_commit(const char* kernel, const ProfEvents& e);
template <typename F, typename... Args>
inline void launch_timed(const char* kernel, F fn, dim3 grid, dim3 block, uint32_t lds,
                         hipStream_t s, Args... args) {
  const ProfEvents e = prof_events(s);
  hipExtLaunchKernelGGL(fn, grid, block, lds, s, e.start, e.stop, 0, args...);
  prof_commit(kernel, e);
}

}  // namespace ddqd
