// QD matrix product on INT8 matrix cores by the Ozaki-style split of the DD
// form, carried to S (default 31) digits per operand.  A base kernel for the
// leaves of Sec. 2's algorithms in QD (Sec. 3, Table 2's precision); not in
// the paper, which predates it.
//
// 1. Scale: the DD form's row exponents of A and column exponents of B (from
//    the leading components), a'_ik = a_ik 2^-e_i, b'_kj = b_kj 2^-f_j.
// 2. Slice: each scaled QD value is written as sum_{t=1..S} d_t 2^-7t + r,
//    d_t = rint(2^7 r_{t-1}) in [-64, 64].  The remainder stays an exact
//    four-term expansion: after a digit is taken from the leading term, one
//    bottom-up TwoSum pass (error-free) renormalises the four terms, so the
//    leading term is the remainder to within a few ulps and the next digit
//    is its nearest integer.  The digits are stored as INT8 in the fragment
//    order of the 32x32x32 MFMA (lane l: line l % 32, k = 16 (l / 32) + 0..15).
// 3. Products: P_d = sum_{t+u=d} A_t B_u for d = 0..S-1, exact INT32 sums
//    (|P_d| <= S 64^2 l < 2^31 for K chunks of 2^14 and S <= 31).  S 32x32
//    INT32 accumulators (16 S registers a lane) do not fit one wave, so the
//    four waves of a workgroup share one 32x32 block of C and split the
//    diagonals into four contiguous ranges of about S(S+1)/8 products each;
//    the 2S fragments of a K block are staged once in LDS by direct loads
//    (double-buffered) and each wave reads the ones its range needs.
// 4. Recombine: each wave folds its diagonals in groups of four exactly into
//    FP64 (2^21 P_d + 2^14 P_d+1 + 2^7 P_d+2 + P_d+3 < 2^53); the group values
//    of all waves meet in LDS and their sum is formed as a QD by VecSum passes,
//    scaled by 2^(e_i + f_j); then C := beta C + alpha value in QD.
//
// Error: the slicing remainders and the dropped diagonals d >= S contribute at
// most about l (S + 3) 2^(-7S-2) 2^(e_i + f_j) to entry (i, j); with S = 31
// that is below 2^-213 l max|a_i.| max|b_.j| -- QD's accuracy class.
#include "ddqd.h"
#include "common.hpp"
#include "eft.hpp"
#include "qd.hpp"

#pragma clang fp contract(off)

namespace ddqd {

int launch_oz_exponents(const GemmBatch& g, int64_t rows_pad, int64_t cols_pad, int* ea, int* fb,
                        hipStream_t s);

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kFrag = 1024;          // bytes of one 32x32 INT8 fragment block
constexpr int64_t kKChunk = 16384;   // K per exact INT32 accumulation
constexpr int kMinS = 28, kMaxS = 31;

struct OzqLayout {
  int64_t m, n, l;
  int64_t rb, cb, kb;  // 32-blocks: rows of A, columns of B, K
  int S;
  int64_t a_bytes, b_bytes;  // per batch entry
};

OzqLayout ozq_layout(int64_t m, int64_t n, int64_t l, int S) {
  OzqLayout o;
  o.m = m;
  o.n = n;
  o.l = l;
  o.S = S;
  o.rb = (m + 31) / 32;
  o.cb = (n + 31) / 32;
  o.kb = (l + 31) / 32;
  o.a_bytes = o.rb * o.kb * S * (int64_t)kFrag;
  o.b_bytes = o.cb * o.kb * S * (int64_t)kFrag;
  return o;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---- the split of the diagonals over the four waves -------------------------

constexpr int tri(int d) { return d * (d + 1) / 2; }  // products of the diagonals < d
constexpr int iabs(int x) { return x < 0 ? -x : x; }

// First diagonal of wave w's range: the d whose product count before it is
// nearest to w/4 of all S(S+1)/2 products.
constexpr int cut(int S, int w) {
  int best = 0;
  for (int d = 0; d <= S; d++)
    if (iabs(4 * tri(d) - w * tri(S)) < iabs(4 * tri(best) - w * tri(S))) best = d;
  return best;
}
constexpr int ngroups(int S, int w) { return (cut(S, w + 1) - cut(S, w) + 3) / 4; }
constexpr int slot0(int S, int w) {
  int s = 0;
  for (int v = 0; v < w; v++) s += ngroups(S, v);
  return s;
}
constexpr int nslots(int S) { return slot0(S, 4); }

// ---- slicing ----------------------------------------------------------------

// A workgroup takes 32 lines (rows of A or columns of B) by 64 k (two 32-k
// blocks): the four planes are read with coalesced loads into LDS; wave w
// then slices k block w / 2, half w % 2 of every lane's 16-k fragment slot
// (8 values of one line per lane, 8 bytes per digit).
constexpr int kSliceK = 64;

template <int S>
__global__ __launch_bounds__(256) void ozq_slice_kernel(CMat A, CMat B, int64_t m, int64_t n,
                                                        int64_t l, OzqLayout o, const int* ea,
                                                        const int* fb, signed char* Asl,
                                                        signed char* Bsl) {
  __shared__ double tile[4][32][kSliceK + 1];
  const int side = blockIdx.y;
  const int64_t b = blockIdx.z;
  const int64_t nblk32 = side == 0 ? o.rb : o.cb;
  const int64_t kgroups = (o.kb + 1) / 2;
  if ((int64_t)blockIdx.x >= nblk32 * kgroups) return;  // uniform per workgroup
  const int64_t blk = blockIdx.x / kgroups, kg = blockIdx.x % kgroups;
  const int64_t line0 = blk * 32, kbase = kg * kSliceK;
  const CMat X = side == 0 ? A : B;
  const int64_t lines_live = side == 0 ? m : n;
  const double* base = X.p + b * X.bstride;
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int e = t + 256 * j;
      const int ln = side == 0 ? e / kSliceK : e % 32;
      const int kk = side == 0 ? e % kSliceK : e / 32;
      const int64_t line = line0 + ln, k = kbase + kk;
      const bool in = line < lines_live && k < l;
      const int64_t idx = in ? (side == 0 ? line * X.ld + k : k * X.ld + line) : 0;
      v[j] = in ? base[c * X.ps + idx] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int e = t + 256 * j;
      const int ln = side == 0 ? e / kSliceK : e % 32;
      const int kk = side == 0 ? e % kSliceK : e / 32;
      tile[c][ln][kk] = v[j];
    }
  }
  __syncthreads();
  const int w = t / 64, lane = t % 64;
  const int64_t kb = kg * 2 + w / 2;
  if (kb >= o.kb) return;
  const int half = w % 2;
  const int ln = lane % 32, k0 = (w / 2) * 32 + 16 * (lane / 32) + 8 * half;
  const int ex = (side == 0 ? ea : fb)[b * (nblk32 * 32) + line0 + ln];
  double r0[8], r1[8], r2[8], r3[8];
#pragma unroll
  for (int q = 0; q < 8; q++) {
    r0[q] = ldexp(tile[0][ln][k0 + q], -ex);
    r1[q] = ldexp(tile[1][ln][k0 + q], -ex);
    r2[q] = ldexp(tile[2][ln][k0 + q], -ex);
    r3[q] = ldexp(tile[3][ln][k0 + q], -ex);
  }
  signed char* dst = (side == 0 ? Asl + b * o.a_bytes : Bsl + b * o.b_bytes) +
                     (blk * o.kb + kb) * S * (int64_t)kFrag + lane * 16 + 8 * half;
#pragma unroll 1
  for (int s = 0; s < S; s++) {
    uint32_t x[2] = {0u, 0u};
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const double h = r0[q] * 128.0;
      const double d = rint(h);
      x[q / 4] |= (uint32_t)(uint8_t)(signed char)(int)d << (8 * (q % 4));
      // remainder (h - d) + 128 (r1 + r2 + r3), all terms exact; one
      // bottom-up TwoSum pass keeps the sum and brings it to the front
      double a2, a3, a1, b2, a0, b1;
      two_sum(r2[q] * 128.0, r3[q] * 128.0, a2, a3);
      two_sum(r1[q] * 128.0, a2, a1, b2);
      two_sum(h - d, a1, a0, b1);
      r0[q] = a0;
      r1[q] = b1;
      r2[q] = b2;
      r3[q] = a3;
    }
    *reinterpret_cast<uint2*>(dst + s * (int64_t)kFrag) = uint2{x[0], x[1]};
  }
}

// ---- products ---------------------------------------------------------------

template <int S>
struct Stage {
  v4i (*lds)[2 * S][64];
  const signed char* asrc;  // this workgroup's A row block, lane offset applied
  const signed char* bsrc;  // its B column block

  // wave W's share (fragments W, W + 4, ...) of the 2S fragments of K block
  // kb into buffer st
  template <int W>
  __device__ __forceinline__ void load(int st, int64_t kb) const {
#pragma unroll
    for (int f = W; f < 2 * S; f += 4) {
      const signed char* src = f < S ? asrc + (kb * S + f) * (int64_t)kFrag
                                     : bsrc + (kb * S + f - S) * (int64_t)kFrag;
      __builtin_amdgcn_global_load_lds(
          (const void*)src, (__attribute__((address_space(3))) void*)&lds[st][f][0], 16, 0, 0);
    }
  }
};

// Wave with diagonals [D0, D1): rows t of the product triangle from the last
// down to 0, each row's slices u ascending, so every row brings in one new A
// and one new B fragment (prefetched during the row before) and consecutive
// uses of one accumulator are at least a row apart.  Afterwards the
// diagonals go to LDS as FP64 group values (slots from SL0).
template <int S, int W>
__device__ __forceinline__ void ozq_wave(const Stage<S>& stage, int lane, int64_t kc0,
                                         int64_t kc1, double (*red)[32][32]) {
  constexpr int D0 = cut(S, W), D1 = cut(S, W + 1), SL0 = slot0(S, W);
  constexpr int ND = D1 - D0;
  v16i acc[ND];
#pragma unroll
  for (int d = 0; d < ND; d++)
#pragma unroll
    for (int q = 0; q < 16; q++) acc[d][q] = 0;
  for (int64_t kb = kc0; kb < kc1; kb++) {
    const int st = (int)((kb - kc0) & 1);
    // block kb has landed in buffer st, every wave is done with buffer st ^ 1
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (kb + 1 < kc1) stage.template load<W>(st ^ 1, kb + 1);
    const v4i(*L)[64] = stage.lds[st];
    v4i fb[S];
    constexpr int t_hi = D1 - 1;  // D1 <= S
    v4i fa_cur = L[t_hi][lane];
    fb[0] = L[S + 0][lane];
#pragma unroll
    for (int t = t_hi; t >= 0; t--) {
      const int ulo = D0 - t > 0 ? D0 - t : 0, uhi = D1 - 1 - t;
      v4i fa_next = fa_cur;
      if (t > 0) {
        fa_next = L[t - 1][lane];
        fb[D1 - t] = L[S + D1 - t][lane];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = ulo; u <= uhi; u++)
        acc[t + u - D0] =
            __builtin_amdgcn_mfma_i32_32x32x32_i8(fa_cur, fb[u], acc[t + u - D0], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      fa_cur = fa_next;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();  // staging buffers are free: red aliases them
  // lane's outputs: column lane % 32, rows 8 (q / 4) + 4 (lane / 32) + q % 4
  const int col = lane % 32, rb2 = 4 * (lane / 32);
#pragma unroll
  for (int gi = 0; gi < (ND + 3) / 4; gi++) {
    const int dfirst = D0 + 4 * gi;
    const int dlast = dfirst + 3 < D1 - 1 ? dfirst + 3 : D1 - 1;
#pragma unroll
    for (int q = 0; q < 16; q++) {
      double G = 0.0;  // exact: integers < 2^53
#pragma unroll
      for (int d = dfirst; d <= dlast; d++) G = __builtin_fma(G, 128.0, (double)acc[d - D0][q]);
      red[SL0 + gi][8 * (q / 4) + rb2 + q % 4][col] = ldexp(G, -7 * (dlast + 2));
    }
  }
}

template <int S>
__global__ __launch_bounds__(256) void ozq_gemm_kernel(GemmBatch g, OzqLayout o,
                                                       const signed char* Asl,
                                                       const signed char* Bsl, const int* ea,
                                                       const int* fb, int64_t kc0, int64_t kc1,
                                                       int beta) {
  __shared__ v4i lds[2][2 * S][64];
  static_assert(nslots(S) * 32 * 32 * sizeof(double) <= sizeof(lds), "epilogue LDS");
  static_assert(cut(S, 1) <= 16, "wave 0 keeps at most 16 accumulators");

  const int64_t t = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
  const int64_t per = o.rb * o.cb;
  const int64_t b = t / per;
  const int64_t rbi = (t % per) / o.cb, cbi = (t % per) % o.cb;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wu = __builtin_amdgcn_readfirstlane(w);

  Stage<S> stage{lds, Asl + b * o.a_bytes + rbi * o.kb * S * (int64_t)kFrag + lane * 16,
                 Bsl + b * o.b_bytes + cbi * o.kb * S * (int64_t)kFrag + lane * 16};
  double(*red)[32][32] = reinterpret_cast<double(*)[32][32]>(&lds[0][0][0]);
  if (wu == 0) {
    stage.template load<0>(0, kc0);
    ozq_wave<S, 0>(stage, lane, kc0, kc1, red);
  } else if (wu == 1) {
    stage.template load<1>(0, kc0);
    ozq_wave<S, 1>(stage, lane, kc0, kc1, red);
  } else if (wu == 2) {
    stage.template load<2>(0, kc0);
    ozq_wave<S, 2>(stage, lane, kc0, kc1, red);
  } else {
    stage.template load<3>(0, kc0);
    ozq_wave<S, 3>(stage, lane, kc0, kc1, red);
  }
  __syncthreads();

  // sum of the group values (largest first) as a QD by VecSum passes, then
  // the exponent scaling and C := beta C + alpha value
  constexpr int NS = nslots(S);
  const int c = threadIdx.x % 32;
  const int64_t col = cbi * 32 + c;
  if (col >= g.n) return;
  const int fexp = fb[b * (o.cb * 32) + col];
  const double* Cb_ro = g.C.p + b * g.C.bstride;
  double* Cb = g.C.p + b * g.C.bstride;
#pragma unroll 1
  for (int z = 0; z < 4; z++) {
    const int r = threadIdx.x / 32 + 8 * z;
    const int64_t row = rbi * 32 + r;
    if (row >= g.m) break;
    double v[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) v[k] = red[k][r][c];
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
      for (int i = NS - 1; i > k; i--) two_sum(v[i - 1], v[i], v[i - 1], v[i]);
    double tail = 0.0;
#pragma unroll
    for (int k = NS - 1; k >= 4; k--) tail += v[k];
    qd_t x{{v[0], v[1], v[2], v[3] + tail}};
    qd_renorm(x.c[0], x.c[1], x.c[2], x.c[3]);
    const int sc = ea[b * (o.rb * 32) + row] + fexp;
#pragma unroll
    for (int k = 0; k < 4; k++) x.c[k] = ldexp(x.c[k], sc);
    if (g.alpha < 0) x = qd_neg(x);
    const int64_t off = row * g.C.ld + col;
    if (beta)
      x = qd_add(qd_t{{Cb_ro[off], Cb_ro[g.C.ps + off], Cb_ro[2 * g.C.ps + off],
                       Cb_ro[3 * g.C.ps + off]}},
                 x);
#pragma unroll
    for (int k = 0; k < 4; k++) Cb[k * g.C.ps + off] = x.c[k];
  }
}

template <int S>
int run_ozaki_qd(const GemmBatch& g, char* ws, hipStream_t s) {
  OzqLayout o = ozq_layout(g.m, g.n, g.l, S);
  signed char* Asl = (signed char*)ws;
  signed char* Bsl = (signed char*)(ws + align256(o.a_bytes * g.batch));
  int* ea = (int*)(ws + align256(o.a_bytes * g.batch) + align256(o.b_bytes * g.batch));
  int* fb = ea + g.batch * o.rb * 32;
  if (g.batch > 65535) return set_error(DDQD_E_UNSUPPORTED, "batch too large");
  const int64_t sblocks = (o.rb > o.cb ? o.rb : o.cb) * ((o.kb + 1) / 2);
  if (sblocks > INT32_MAX || o.kb > 65535)
    return set_error(DDQD_E_UNSUPPORTED, "matrix too large for one Ozaki launch");
  int rc = launch_oz_exponents(g, o.rb * 32, o.cb * 32, ea, fb, s);
  if (rc) return rc;
  prof_begin(s);
  hipLaunchKernelGGL(ozq_slice_kernel<S>, dim3((unsigned)sblocks, 2, (unsigned)g.batch),
                     dim3(256), 0, s, g.A, g.B, g.m, g.n, g.l, o, (const int*)ea, (const int*)fb,
                     Asl, Bsl);
  prof_record("ozq_slice_kernel", s);
  if ((rc = check_launch("ozq_slice_kernel"))) return rc;
  const int64_t nblk = o.rb * o.cb * g.batch;
  if (nblk > INT32_MAX) return set_error(DDQD_E_UNSUPPORTED, "grid too large");
  for (int64_t kc0 = 0; kc0 < o.kb; kc0 += kKChunk / 32) {
    const int64_t kc1 = kc0 + kKChunk / 32 < o.kb ? kc0 + kKChunk / 32 : o.kb;
    prof_begin(s);
    hipLaunchKernelGGL(ozq_gemm_kernel<S>, dim3((unsigned)nblk), dim3(256), 0, s, g, o,
                       (const signed char*)Asl, (const signed char*)Bsl, (const int*)ea,
                       (const int*)fb, kc0, kc1, kc0 == 0 ? g.beta : 1);
    prof_record("ozq_gemm_kernel", s);
    if ((rc = check_launch("ozq_gemm_kernel"))) return rc;
  }
  return DDQD_OK;
}

}  // namespace

int ozaki_qd_default_slices() { return 31; }

size_t ozaki_qd_workspace(int64_t m, int64_t n, int64_t l, int64_t batch, int slices) {
  const int S = slices == 0 ? ozaki_qd_default_slices() : slices;
  if (S < kMinS || S > kMaxS || m <= 0 || n <= 0 || l <= 0) return 0;
  OzqLayout o = ozq_layout(m, n, l, S);
  return align256(o.a_bytes * batch) + align256(o.b_bytes * batch) +
         align256(sizeof(int) * (size_t)(batch * (o.rb + o.cb) * 32));
}

int launch_ozaki_qd(const GemmBatch& g, int slices, void* ws, size_t ws_bytes, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return DDQD_OK;
  const int S = slices == 0 ? ozaki_qd_default_slices() : slices;
  if (S < kMinS || S > kMaxS)
    return set_error(DDQD_E_UNSUPPORTED, "QD Ozaki slices must be in %d..%d", kMinS, kMaxS);
  if (ozaki_qd_workspace(g.m, g.n, g.l, g.batch, S) > ws_bytes)
    return set_error(DDQD_E_WORKSPACE, "Ozaki workspace too small");
  char* w = (char*)ws;
  switch (S) {
    case 28: return run_ozaki_qd<28>(g, w, s);
    case 29: return run_ozaki_qd<29>(g, w, s);
    case 30: return run_ozaki_qd<30>(g, w, s);
    case 31: return run_ozaki_qd<31>(g, w, s);
  }
  return set_error(DDQD_E_UNSUPPORTED, "slices");
}

}  // namespace ddqd
