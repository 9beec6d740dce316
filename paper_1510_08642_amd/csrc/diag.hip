// Diagnostic kernel: dependent-chain latencies of the operations the LU's
// column step is built from (FP64 add and FMA, TwoSum, a lane exchange,
// readlane broadcasts, an LDS round trip, barriers), timed with the shader's
// s_memtime counter inside one workgroup.  It computes nothing the library
// uses; the profile of the strip kernel compares its cycles per column with
// these latencies.
#include "common.hpp"
#include "ddqd.h"

#pragma clang fp contract(off)

namespace ddqd {

int check_device();
void clear_error();

namespace {

__device__ __forceinline__ long long ticks() { return (long long)__builtin_amdgcn_s_memtime(); }

// out[0..7]: ticks per step of a dependent FMA chain, a dependent add chain,
// a TwoSum chain, a shuffle + max chain, a two-readlane + add chain, an LDS
// write / read chain, a chain of two barriers with an LDS exchange, and four
// independent FMA chains (one step of each)
__global__ __launch_bounds__(1024) void latency_kernel(double* out, double a, double b,
                                                       int steps) {
  __shared__ double lds[1024];
  const int t = threadIdx.x;
  double x = a + t * 1e-9, e = 0.0;
  long long c0, c1;
  __syncthreads();
  c0 = ticks();
  for (int i = 0; i < steps; i++) x = fma(x, a, b);
  c1 = ticks();
  if (t == 0) out[0] = (double)(c1 - c0) / steps;
  __syncthreads();
  c0 = ticks();
  for (int i = 0; i < steps; i++) x = x + b;
  c1 = ticks();
  if (t == 0) out[1] = (double)(c1 - c0) / steps;
  __syncthreads();
  c0 = ticks();
  for (int i = 0; i < steps; i++) {
    const double s = x + b, bb = s - x;
    e += (x - (s - bb)) + (b - bb);
    x = s;
  }
  c1 = ticks();
  if (t == 0) out[2] = (double)(c1 - c0) / steps;
  __syncthreads();
  c0 = ticks();
  for (int i = 0; i < steps; i++) x = fmax(x, __shfl_xor(x, 1 + (i & 15), 64));
  c1 = ticks();
  if (t == 0) out[3] = (double)(c1 - c0) / steps;
  __syncthreads();
  c0 = ticks();
  for (int i = 0; i < steps; i++) {
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), i & 63);
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), i & 63);
    x = __hiloint2double(hi, lo) + b;
  }
  c1 = ticks();
  if (t == 0) out[4] = (double)(c1 - c0) / steps;
  __syncthreads();
  c0 = ticks();
  for (int i = 0; i < steps; i++) {
    lds[(t + i) & 1023] = x;
    __builtin_amdgcn_s_waitcnt(0);
    x = lds[(t + i) & 1023] + b;
  }
  c1 = ticks();
  if (t == 0) out[5] = (double)(c1 - c0) / steps;
  __syncthreads();
  c0 = ticks();
  for (int i = 0; i < steps; i++) {
    lds[t] = x;
    __syncthreads();
    x = lds[(t + 64) & (blockDim.x - 1)] + b;
    __syncthreads();
  }
  c1 = ticks();
  if (t == 0) out[6] = (double)(c1 - c0) / steps;
  double x1 = x, x2 = x + 1.0, x3 = x + 2.0, x4 = x + 3.0;
  __syncthreads();
  c0 = ticks();
  for (int i = 0; i < steps; i++) {
    x1 = fma(x1, a, b);
    x2 = fma(x2, a, b);
    x3 = fma(x3, a, b);
    x4 = fma(x4, a, b);
  }
  c1 = ticks();
  if (t == 0) out[7] = (double)(c1 - c0) / steps;
  // keep every chain live
  if (x + e + x1 + x2 + x3 + x4 == 12345.0) out[8] = x;
}

}  // namespace
}  // namespace ddqd

using namespace ddqd;

extern "C" int ddqd_latency_probe(double* out, int threads, int steps, void* stream) {
  clear_error();
  if (!out || (threads != 64 && threads != 256 && threads != 1024) || steps < 1 ||
      steps > (1 << 20))
    return set_error(DDQD_E_ARG, "latency probe: out, threads (64/256/1024) or steps invalid");
  int rc;
  if ((rc = check_device())) return rc;
  hipLaunchKernelGGL(latency_kernel, dim3(1), dim3(threads), 0, (hipStream_t)stream, out,
                     0.999999, 1e-7, steps);
  return check_launch("latency_kernel");
}
