// QD matrix-product kernels on FP64 FMA: Simple and Block (Sec. 2 of the
// paper, in the quad-double precision of its Table 2).
//
// Block kernel.  A 256-thread workgroup owns a 32x32 tile of C, each thread a
// 2x2 micro-tile held as four order buckets per entry (see qd_mac); the
// 16x16 variant (one entry per thread) gives small products four times the
// workgroups.  K moves in steps of 16 with the four planes of the A tile
// (k-major) and B tile double-buffered in LDS.  The buckets are renormalised
// after every K step.  Every entry sees the same operations in the same order
// in both variants, so their results are identical.  About 113 FP64
// operations per QD multiply-add make the kernel VALU-bound; LDS traffic is
// 16 doubles per 4 multiply-adds (32x32).
#include "common.hpp"
#include "qd.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

constexpr int kBK = 16, kThreads = 256;
constexpr int kPad = 2;

// kT x kT micro-tiles per thread, tile edge 16 kT
template <int kT>
__global__ __launch_bounds__(kThreads) void qd_gemm_block_kernel(GemmBatch g, int64_t tiles_m,
                                                                 int64_t tiles_n) {
  constexpr int kBM = 16 * kT, kBN = 16 * kT, kTM = kT, kTN = kT;
  __shared__ __attribute__((aligned(16))) double As[2][4][kBK][kBM + kPad];
  __shared__ __attribute__((aligned(16))) double Bs[2][4][kBK][kBN + kPad];

  const int64_t t = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
  const int64_t per = tiles_m * tiles_n;
  const int64_t b = t / per;
  const int64_t tm = (t % per) / tiles_n, tn = (t % per) % tiles_n;
  const int64_t row0 = tm * kBM, col0 = tn * kBN;
  const double* Ab = g.A.p + b * g.A.bstride;
  const double* Bb = g.B.p + b * g.B.bstride;
  double* Cb = g.C.p + b * g.C.bstride;

  const int tid = threadIdx.x;
  const int tx = tid % (kBN / kTN), ty = tid / (kBN / kTN);
  const double sa = (double)g.alpha;

  qd_acc acc[kTM][kTN];
#pragma unroll
  for (int r = 0; r < kTM; r++)
#pragma unroll
    for (int c = 0; c < kTN; c++) {
      acc[r][c] = qd_acc{0.0, 0.0, 0.0, 0.0};
      int64_t i = row0 + ty * kTM + r, j = col0 + tx * kTN + c;
      if (g.beta && i < g.m && j < g.n) {
        const int64_t o = i * g.C.ld + j;
        acc[r][c] = qd_acc{sa * Cb[o], sa * Cb[g.C.ps + o], sa * Cb[2 * g.C.ps + o],
                           sa * Cb[3 * g.C.ps + o]};
      }
    }

  constexpr int kPer = (kBM * kBK + kThreads - 1) / kThreads;  // 2 (32x32) or 1 (16x16)
  double ra[4][kPer], rb[4][kPer];
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < kPer; q++) {
      int el = tid + q * kThreads;
      int rr = el / kBK, kk = el % kBK;
      int64_t i = row0 + rr, k = k0 + kk;
      bool ok = i < g.m && k < g.l;
      int kb = el / kBN, cc = el % kBN;
      int64_t kg = k0 + kb, j = col0 + cc;
      bool okb = kg < g.l && j < g.n;
#pragma unroll
      for (int c = 0; c < 4; c++) {
        ra[c][q] = ok ? Ab[c * g.A.ps + i * g.A.ld + k] : 0.0;
        rb[c][q] = okb ? Bb[c * g.B.ps + kg * g.B.ld + j] : 0.0;
      }
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int q = 0; q < kPer; q++) {
      int el = tid + q * kThreads;
      int rr = el / kBK, kk = el % kBK;
      int kb = el / kBN, cc = el % kBN;
#pragma unroll
      for (int c = 0; c < 4; c++) {
        As[buf][c][kk][rr] = ra[c][q];
        Bs[buf][c][kb][cc] = rb[c][q];
      }
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
#pragma unroll 2
    for (int kk = 0; kk < kBK; kk++) {
      double a[kTM][4], bv[kTN][4];
#pragma unroll
      for (int c = 0; c < 4; c++) {
        if constexpr (kT == 2) {
          double2 x = *reinterpret_cast<const double2*>(&As[buf][c][kk][ty * kTM]);
          double2 y = *reinterpret_cast<const double2*>(&Bs[buf][c][kk][tx * kTN]);
          a[0][c] = x.x;
          a[1][c] = x.y;
          bv[0][c] = y.x;
          bv[1][c] = y.y;
        } else {
#pragma unroll
          for (int r = 0; r < kT; r++) {
            a[r][c] = As[buf][c][kk][ty * kTM + r];
            bv[r][c] = Bs[buf][c][kk][tx * kTN + r];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kTM; r++)
#pragma unroll
        for (int c = 0; c < kTN; c++) qd_mac(acc[r][c], a[r], bv[c]);
    }
#pragma unroll
    for (int r = 0; r < kTM; r++)
#pragma unroll
      for (int c = 0; c < kTN; c++)
        qd_renorm(acc[r][c].s0, acc[r][c].s1, acc[r][c].s2, acc[r][c].s3);
    if (ks + 1 < ksteps) store_tiles(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int r = 0; r < kTM; r++)
#pragma unroll
    for (int c = 0; c < kTN; c++) {
      int64_t i = row0 + ty * kTM + r, j = col0 + tx * kTN + c;
      if (i < g.m && j < g.n) {
        qd_acc v = acc[r][c];
        qd_renorm(v.s0, v.s1, v.s2, v.s3);
        const int64_t o = i * g.C.ld + j;
        Cb[o] = sa * v.s0;
        Cb[g.C.ps + o] = sa * v.s1;
        Cb[2 * g.C.ps + o] = sa * v.s2;
        Cb[3 * g.C.ps + o] = sa * v.s3;
      }
    }
}

// Simple: one thread per c_ij, k ascending, acc := acc + a_ik * b_kj with QD
// operators.
__global__ __launch_bounds__(256) void qd_gemm_simple_kernel(GemmBatch g) {
  const int64_t j = (int64_t)blockIdx.x * 16 + threadIdx.x % 16;
  const int64_t i = (int64_t)blockIdx.y * 16 + threadIdx.x / 16;
  const int64_t b = blockIdx.z;
  if (i >= g.m || j >= g.n) return;
  const double* Ab = g.A.p + b * g.A.bstride;
  const double* Bb = g.B.p + b * g.B.bstride;
  double* Cb = g.C.p + b * g.C.bstride;
  qd_t acc{{0.0, 0.0, 0.0, 0.0}};
  for (int64_t k = 0; k < g.l; k++) {
    qd_t a = QDNum::load(Ab, g.A.ps, i * g.A.ld + k);
    qd_t bb = QDNum::load(Bb, g.B.ps, k * g.B.ld + j);
    acc = qd_add(acc, qd_mul(a, bb));
  }
  if (g.alpha < 0) acc = qd_neg(acc);
  if (g.beta) acc = qd_add(QDNum::load(Cb, g.C.ps, i * g.C.ld + j), acc);
  QDNum::store(Cb, g.C.ps, i * g.C.ld + j, acc);
}

}  // namespace

// tile: 32 or 16 (the same results), 0 = 32
int launch_qd_block(const GemmBatch& g, int tile, hipStream_t stream) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return 0;
  if (tile == 0) tile = 32;
  if (tile != 32 && tile != 16) return set_error(1 /*DDQD_E_ARG*/, "QD tile must be 32 or 16");
  int64_t tm = (g.m + tile - 1) / tile, tn = (g.n + tile - 1) / tile;
  int64_t nblk = tm * tn * g.batch;
  if (nblk > INT32_MAX) return set_error(4, "grid too large");
  if (tile == 32)
    launch_timed("qd_gemm_block_kernel", qd_gemm_block_kernel<2>, dim3((unsigned)nblk),
                 dim3(kThreads), 0, stream, g, tm, tn);
  else
    launch_timed("qd_gemm_block_kernel<16>", qd_gemm_block_kernel<1>, dim3((unsigned)nblk),
                 dim3(kThreads), 0, stream, g, tm, tn);
  return check_launch("qd_gemm_block_kernel");
}

int launch_qd_simple(const GemmBatch& g, hipStream_t stream) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return 0;
  dim3 grid((unsigned)((g.n + 15) / 16), (unsigned)((g.m + 15) / 16), (unsigned)g.batch);
  if (grid.y > 65535 || grid.z > 65535) return set_error(4, "grid too large");
  prof_begin(stream);
  hipLaunchKernelGGL(qd_gemm_simple_kernel, grid, dim3(256), 0, stream, g);
  prof_record("qd_gemm_simple_kernel", stream);
  return check_launch("qd_gemm_simple_kernel");
}

}  // namespace ddqd
