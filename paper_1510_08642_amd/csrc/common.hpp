// Shared host/device structures of libddqd: strided batches of matrices in
// plane layout, launch helpers and the XCD-aware block remap.
#pragma once
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

// Round-robin dispatch places workgroup b on XCD b % 8.  This permutation
// gives each XCD one contiguous range of logical tiles, so tiles that share
// operand panels share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblk) {
  constexpr int64_t kXcd = 8;
  int64_t x = b % kXcd, local = b / kXcd;
  int64_t q = nblk / kXcd, r = nblk % kXcd;
  return x * q + (x < r ? x : r) + local;
}

// Host-side status plumbing shared by the launchers.
int set_error(int status, const char* fmt, ...);
int check_launch(const char* what);

// Optional per-kernel timing (ddqd_profile_enable): when on, every launch is
// bracketed by HIP events recorded on its stream; no effect when off.
void prof_begin(hipStream_t s);
void prof_record(const char* kernel, hipStream_t s);

}  // namespace ddqd
