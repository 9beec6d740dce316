// DD matrix-product kernels on FP64 FMA: Simple and Block (the paper's
// Sec. 2: Eq. 1, and its blocked form C_ij = sum_K A_iK B_Kj).
//
// Block kernel.  A 256-thread workgroup owns a 64x64 tile of C; each thread
// a 4x4 register micro-tile.  K advances in steps of 16: the hi and lo planes
// of the A tile (stored k-major, so a thread reads its 4 rows with two 16-byte
// LDS reads per plane) and of the B tile are double-buffered in LDS while the
// next step is prefetched into registers.  A 32x32 tile (2x2 per thread)
// gives small products four times as many workgroups; every entry of C sees
// the same operations in the same order with either tile, so the two results
// are bit-identical.
//
// Per multiply-add (a_h + a_l)(b_h + b_l) the kernel forms the product's
// leading part p = fl(a_h b_h) and its tail q = err(a_h b_h) + a_h b_l +
// a_l b_h with three FMAs (the a_l b_l term is below 2^-106 relative and is
// dropped), adds p into a running FP64 sum s with TwoSum, and adds the TwoSum
// error and q into a correction e: 12 FP64 operations.  After every K step
// (s, e) is renormalised by TwoSum, which keeps the accumulated rounding of e
// at most about 16 l u^2 times sum |a||b| (u = 2^-53), inside 2^-100 l.
#include "common.hpp"
#include "eft.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

constexpr int kBK = 16, kThreads = 256;
constexpr int kPad = 2;  // keeps 16-byte rows, spreads banks

template <int BM>
using TileBuf = double[2][2][kBK][BM + kPad];

// One BM x BM tile (tm, tn) of problem b of the batch g.  Shared by the
// batched and the grouped kernels, so a product computed inside a group is
// bit-identical to the same product launched on its own.
template <int BM>
__device__ __forceinline__ void dd_block_tile(const GemmBatch& g, int64_t b, int64_t tm,
                                              int64_t tn, TileBuf<BM>& As, TileBuf<BM>& Bs) {
  constexpr int kBN = BM, kTM = BM / 16, kTN = BM / 16;
  static_assert((BM / kTM) * (kBN / kTN) == kThreads, "16 x 16 threads per tile");
  const int64_t row0 = tm * BM, col0 = tn * kBN;

  const double* Ab = g.A.p + b * g.A.bstride;
  const double* Bb = g.B.p + b * g.B.bstride;
  double* Cb = g.C.p + b * g.C.bstride;

  const int tid = threadIdx.x;
  const int tx = tid % (kBN / kTN), ty = tid / (kBN / kTN);

  double s[kTM][kTN], e[kTM][kTN];
  const double sa = (double)g.alpha;
#pragma unroll
  for (int r = 0; r < kTM; r++)
#pragma unroll
    for (int c = 0; c < kTN; c++) {
      s[r][c] = 0.0;
      e[r][c] = 0.0;
      int64_t i = row0 + ty * kTM + r, j = col0 + tx * kTN + c;
      if (g.beta && i < g.m && j < g.n) {
        // start from alpha*C so the result alpha*(alpha*C + AB) = C + alpha*AB
        s[r][c] = sa * Cb[i * g.C.ld + j];
        e[r][c] = sa * Cb[g.C.ps + i * g.C.ld + j];
      }
    }

  // global -> register staging: 4 elements per plane per operand per thread
  constexpr int kPer = BM * kBK / kThreads;  // 4 (64x64) or 2 (32x32)
  double ra[2][kPer], rb[2][kPer];
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < kPer; q++) {
      int el = tid + q * kThreads;
      int rr = el / kBK, kk = el % kBK;
      int64_t i = row0 + rr, k = k0 + kk;
      bool ok = i < g.m && k < g.l;
      ra[0][q] = ok ? Ab[i * g.A.ld + k] : 0.0;
      ra[1][q] = ok ? Ab[g.A.ps + i * g.A.ld + k] : 0.0;
      int kb = el / kBN, cc = el % kBN;
      int64_t kg = k0 + kb, j = col0 + cc;
      bool okb = kg < g.l && j < g.n;
      rb[0][q] = okb ? Bb[kg * g.B.ld + j] : 0.0;
      rb[1][q] = okb ? Bb[g.B.ps + kg * g.B.ld + j] : 0.0;
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int q = 0; q < kPer; q++) {
      int el = tid + q * kThreads;
      int rr = el / kBK, kk = el % kBK;
      As[buf][0][kk][rr] = ra[0][q];
      As[buf][1][kk][rr] = ra[1][q];
      int kb = el / kBN, cc = el % kBN;
      Bs[buf][0][kb][cc] = rb[0][q];
      Bs[buf][1][kb][cc] = rb[1][q];
    }
  };

  const int64_t ksteps = (g.l + kBK - 1) / kBK;
  if (ksteps > 0) {
    load_tiles(0);
    store_tiles(0);
  }
  __syncthreads();
  for (int64_t ks = 0; ks < ksteps; ks++) {
    const int buf = (int)(ks & 1);
    if (ks + 1 < ksteps) load_tiles((ks + 1) * kBK);
#pragma unroll 4
    for (int kk = 0; kk < kBK; kk++) {
      double ah[kTM], al[kTM], bh[kTN], bl[kTN];
      const double2* pah = reinterpret_cast<const double2*>(&As[buf][0][kk][ty * kTM]);
      const double2* pal = reinterpret_cast<const double2*>(&As[buf][1][kk][ty * kTM]);
      const double2* pbh = reinterpret_cast<const double2*>(&Bs[buf][0][kk][tx * kTN]);
      const double2* pbl = reinterpret_cast<const double2*>(&Bs[buf][1][kk][tx * kTN]);
#pragma unroll
      for (int v = 0; v < kTM / 2; v++) {
        double2 x = pah[v], y = pal[v];
        ah[2 * v] = x.x;
        ah[2 * v + 1] = x.y;
        al[2 * v] = y.x;
        al[2 * v + 1] = y.y;
      }
#pragma unroll
      for (int v = 0; v < kTN / 2; v++) {
        double2 x = pbh[v], y = pbl[v];
        bh[2 * v] = x.x;
        bh[2 * v + 1] = x.y;
        bl[2 * v] = y.x;
        bl[2 * v + 1] = y.y;
      }
#pragma unroll
      for (int r = 0; r < kTM; r++)
#pragma unroll
        for (int c = 0; c < kTN; c++) dd_mac(s[r][c], e[r][c], ah[r], al[r], bh[c], bl[c]);
    }
#pragma unroll
    for (int r = 0; r < kTM; r++)
#pragma unroll
      for (int c = 0; c < kTN; c++) two_sum(s[r][c], e[r][c], s[r][c], e[r][c]);
    if (ks + 1 < ksteps) store_tiles(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int r = 0; r < kTM; r++)
#pragma unroll
    for (int c = 0; c < kTN; c++) {
      int64_t i = row0 + ty * kTM + r, j = col0 + tx * kTN + c;
      if (i < g.m && j < g.n) {
        double h, lo;
        two_sum(s[r][c], e[r][c], h, lo);
        Cb[i * g.C.ld + j] = sa * h;
        Cb[g.C.ps + i * g.C.ld + j] = sa * lo;
      }
    }
}

template <int BM>
__global__ __launch_bounds__(kThreads) void dd_gemm_block_kernel(GemmBatch g, int64_t tiles_m,
                                                                 int64_t tiles_n) {
  __shared__ __attribute__((aligned(16))) TileBuf<BM> As, Bs;
  const int64_t t = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
  const int64_t per = tiles_m * tiles_n;
  dd_block_tile<BM>(g, t / per, (t % per) / tiles_n, (t % per) % tiles_n, As, Bs);
}

// Grouped: up to kMaxGroup unrelated problems of any shapes in one
// persistent launch; workgroup w takes tiles w, w + grid, w + 2 grid, ... of
// the concatenated tile list (a fixed order: results do not depend on the
// grid size or on the other problems).
__global__ __launch_bounds__(kThreads) void dd_gemm_grouped_kernel(GroupArgs ga) {
  __shared__ __attribute__((aligned(16))) TileBuf<64> As, Bs;
  for (int64_t t = blockIdx.x; t < ga.start[ga.count]; t += gridDim.x) {
    int p = 0;
    while (t >= ga.start[p + 1]) p++;
    const int64_t r = t - ga.start[p];
    const int64_t tn_count = (ga.g[p].n + 63) / 64;
    dd_block_tile<64>(ga.g[p], 0, r / tn_count, r % tn_count, As, Bs);
    __syncthreads();
  }
}

// Simple: one thread per c_ij, k ascending, each step a DD product and an
// accurate DD sum (the paper's Eq. 1 with DD operators).
__global__ __launch_bounds__(256) void dd_gemm_simple_kernel(GemmBatch g) {
  const int64_t j = (int64_t)blockIdx.x * 16 + threadIdx.x % 16;
  const int64_t i = (int64_t)blockIdx.y * 16 + threadIdx.x / 16;
  const int64_t b = blockIdx.z;
  if (i >= g.m || j >= g.n) return;
  const double* Ab = g.A.p + b * g.A.bstride;
  const double* Bb = g.B.p + b * g.B.bstride;
  double* Cb = g.C.p + b * g.C.bstride;
  dd_t acc{0.0, 0.0};
  for (int64_t k = 0; k < g.l; k++) {
    dd_t a{Ab[i * g.A.ld + k], Ab[g.A.ps + i * g.A.ld + k]};
    dd_t bb{Bb[k * g.B.ld + j], Bb[g.B.ps + k * g.B.ld + j]};
    acc = dd_add(acc, dd_mul(a, bb));
  }
  if (g.alpha < 0) acc = dd_neg(acc);
  if (g.beta) acc = dd_add(dd_t{Cb[i * g.C.ld + j], Cb[g.C.ps + i * g.C.ld + j]}, acc);
  Cb[i * g.C.ld + j] = acc.hi;
  Cb[g.C.ps + i * g.C.ld + j] = acc.lo;
}

}  // namespace

int launch_dd_block(const GemmBatch& g, int tile, hipStream_t stream) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return 0;
  if (tile != 64 && tile != 32) return set_error(1 /*DDQD_E_ARG*/, "tile must be 64 or 32");
  int64_t tm = (g.m + tile - 1) / tile, tn = (g.n + tile - 1) / tile;
  int64_t nblk = tm * tn * g.batch;
  if (nblk > INT32_MAX) return set_error(4 /*DDQD_E_UNSUPPORTED*/, "grid too large");
  if (tile == 64)
    launch_timed("dd_gemm_block_kernel", dd_gemm_block_kernel<64>, dim3((unsigned)nblk),
                 dim3(kThreads), 0, stream, g, tm, tn);
  else
    launch_timed("dd_gemm_block_kernel<32>", dd_gemm_block_kernel<32>, dim3((unsigned)nblk),
                 dim3(kThreads), 0, stream, g, tm, tn);
  return check_launch("dd_gemm_block_kernel");
}

int64_t dd_block_tiles(int64_t m, int64_t n) { return ((m + 63) / 64) * ((n + 63) / 64); }

int launch_dd_grouped(const GroupArgs& ga, int grid, hipStream_t stream) {
  if (ga.count <= 0 || ga.start[ga.count] <= 0) return 0;
  prof_begin(stream);
  hipLaunchKernelGGL(dd_gemm_grouped_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, ga);
  prof_record("dd_gemm_grouped_kernel", stream);
  return check_launch("dd_gemm_grouped_kernel");
}

int launch_dd_simple(const GemmBatch& g, hipStream_t stream) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return 0;
  dim3 grid((unsigned)((g.n + 15) / 16), (unsigned)((g.m + 15) / 16), (unsigned)g.batch);
  if (grid.y > 65535 || grid.z > 65535) return set_error(4, "grid too large");
  prof_begin(stream);
  hipLaunchKernelGGL(dd_gemm_simple_kernel, grid, dim3(256), 0, stream, g);
  prof_record("dd_gemm_simple_kernel", stream);
  return check_launch("dd_gemm_simple_kernel");
}

}  // namespace ddqd
