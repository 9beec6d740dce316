// QD matrix product on INT8 matrix cores by the Ozaki-style split of the DD
// form, carried to S (default 31) digits per operand.  A base kernel for the
// leaves of Sec. 2's algorithms in QD (Sec. 3, Table 2's precision); not in
// the paper, which predates it.  Steps 1 and 2 run in ozaki_split.hip,
// steps 3 and 4 here.
//
// 1. Scale: the DD form's row exponents of A and column exponents of B (from
//    the leading components), a'_ik = a_ik 2^-e_i, b'_kj = b_kj 2^-f_j.
// 2. Slice: each scaled QD value is written as sum_{t=1..S} d_t 2^-7t + r,
//    d_t in [-64, 64].  The remainder stays an exact four-term expansion:
//    runs of six digits d = rint(2^7 r0), r0 := 2^7 r0 - d are taken from the
//    leading term alone (exact steps; the lower terms stand for themselves
//    times 2^(7j)), then the lower terms are scaled by 2^42 and one
//    bottom-up TwoSum pass (error-free) renormalises the four terms, leaving
//    the rest within about an ulp of the leading term.  Inside a run the
//    ignored part is below 2^-12 of a digit unit, so digits stay in
//    [-64, 64].  The digits are stored as INT8 in the fragment order of the
//    32x32x32 MFMA (lane l: line l % 32, k = 16 (l / 32) + 0..15).
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
// most about l (S + 3) 2^(-7S-2) 2^(e_i + f_j) to entry (i, j).  Since
// max|a_i.| >= 2^(e_i - 2) and max|b_.j| >= 2^(f_j - 2), 2^(e_i + f_j) is at
// most 16 max|a_i.| max|b_.j|; with S = 31 the bound is below
// 2^-209 l max|a_i.| max|b_.j| -- QD's accuracy class.
#include "ddqd.h"
#include "common.hpp"
#include "eft.hpp"
#include "qd.hpp"
#include "ozaki.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kFrag = kOzFrag;
constexpr int64_t kKChunk = 16384;   // K per exact INT32 accumulation
constexpr int kMinS = 28, kMaxS = 31;

size_t align256(size_t x) { return oz_align256(x); }

// ---- the split of the slice products over the four waves -------------------
//
// Products are numbered along the diagonals: product (t, u) of diagonal
// d = t + u has index tri(d) + t.  Wave 0 takes the whole diagonals [0, c),
// c the diagonal whose product count before it is nearest a quarter of all
// (so it keeps at most 16 accumulators); waves 1-3 split the remaining
// indices into three ranges of equal size, so a diagonal may be shared by two
// waves: each accumulates its part exactly and the epilogue adds all parts.

constexpr int tri(int d) { return d * (d + 1) / 2; }  // products of the diagonals < d
constexpr int iabs(int x) { return x < 0 ? -x : x; }

constexpr int first_cut(int S) {
  int best = 0;
  for (int d = 0; d <= S; d++)
    if (iabs(4 * tri(d) - tri(S)) < iabs(4 * tri(best) - tri(S))) best = d;
  return best;
}
// first product index of wave w (w = 4: one past the last)
constexpr int qstart(int S, int w) {
  if (w == 0) return 0;
  if (w >= 4) return tri(S);
  const int q1 = tri(first_cut(S));
  return q1 + (2 * (tri(S) - q1) * (w - 1) + 3) / 6;
}
constexpr int diag_of(int idx) {
  int d = 0;
  while (tri(d + 1) <= idx) d++;
  return d;
}
constexpr int dlo(int S, int w) { return diag_of(qstart(S, w)); }
constexpr int dhi(int S, int w) { return diag_of(qstart(S, w + 1) - 1); }
constexpr int ngroups(int S, int w) { return (dhi(S, w) - dlo(S, w) + 1 + 3) / 4; }
constexpr int slot0(int S, int w) {
  int s = 0;
  for (int v = 0; v < w; v++) s += ngroups(S, v);
  return s;
}
constexpr int nslots(int S) { return slot0(S, 4); }

// Row t of wave w's part of the product triangle: slices u in [ulo, uhi].
struct Rows {
  int ulo[32], uhi[32];
  int pre[32];  // products in the rows above t (the wave walks t downwards)
  int tmax;
};
constexpr Rows rows_of(int S, int w) {
  Rows r{};
  r.tmax = -1;
  const int a = qstart(S, w), b = qstart(S, w + 1);
  for (int t = 0; t < 32; t++) {
    r.ulo[t] = 1;
    r.uhi[t] = 0;
    int lo = -1, hi = -1;
    for (int u = 0; t + u < S; u++) {
      const int idx = tri(t + u) + t;
      if (idx >= a && idx < b) {
        if (lo < 0) lo = u;
        hi = u;
      }
    }
    if (lo >= 0) {
      r.ulo[t] = lo;
      r.uhi[t] = hi;
      r.tmax = t;
    }
  }
  int n = 0;
  for (int t = 31; t >= 0; t--) {
    r.pre[t] = n;
    if (r.ulo[t] <= r.uhi[t]) n += r.uhi[t] - r.ulo[t] + 1;
  }
  return r;
}
// every row up to tmax holds products and the windows only move up as t
// falls: then each B fragment is read once, when it first enters the window
constexpr bool rows_ok(int S, int w) {
  const Rows r = rows_of(S, w);
  if (r.tmax < 0) return false;
  for (int t = 0; t <= r.tmax; t++) {
    if (r.ulo[t] > r.uhi[t]) return false;
    if (t > 0 && (r.ulo[t - 1] < r.ulo[t] || r.uhi[t - 1] < r.uhi[t])) return false;
  }
  return true;
}

// ---- products ---------------------------------------------------------------

template <int S>
struct Stage {
  v4i (*lds)[2 * S][64];
  const signed char* asrc;  // this workgroup's A row block, lane offset applied
  const signed char* bsrc;  // its B column block

  // the j-th of wave W's fragments (W + 4 j) of K block kb into buffer st
  template <int W>
  __device__ __forceinline__ void load_one(int st, int64_t kb, int j) const {
    const int f = W + 4 * j;
    const signed char* src = f < S ? asrc + (kb * S + f) * (int64_t)kFrag
                                   : bsrc + (kb * S + f - S) * (int64_t)kFrag;
    __builtin_amdgcn_global_load_lds(
        (const void*)src, (__attribute__((address_space(3))) void*)&lds[st][f][0], 16, 0, 0);
  }
  // how many of the 2S fragments are wave W's
  template <int W>
  static constexpr int count() { return (2 * S - W + 3) / 4; }
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

// Wave W's part of the products: rows t from the last down to 0, each row's
// slices u ascending, so every row brings in one new A fragment and the B
// fragments entering its window (read two rows ahead), and
// consecutive uses of one accumulator are at least a row apart.  Afterwards
// its diagonals [D0, D1) go to LDS as FP64 group values (slots from SL0).
template <int S, int W>
__device__ __forceinline__ void ozq_wave(const Stage<S>& stage, int lane, int64_t kc0,
                                         int64_t kc1, double (*red)[32][32]) {
  constexpr int D0 = dlo(S, W), D1 = dhi(S, W) + 1, SL0 = slot0(S, W);
  constexpr int ND = D1 - D0;
  constexpr Rows R = rows_of(S, W);
  constexpr int TM = R.tmax;
  static_assert(rows_ok(S, W), "wave rows");
  v16i acc[ND];
#pragma unroll
  for (int d = 0; d < ND; d++)
#pragma unroll
    for (int q = 0; q < 16; q++) acc[d][q] = 0;
  constexpr int NDMA = Stage<S>::template count<W>();
  static_assert(NDMA <= tri(S), "one DMA load per MFMA");
  for (int64_t kb = kc0; kb < kc1; kb++) {
    const int st = (int)((kb - kc0) & 1);
    // block kb has landed in buffer st, every wave is done with buffer st ^ 1
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // block kb + 1 goes into buffer st ^ 1, one fragment after each of the
    // first MFMAs, so the DMA issue hides behind the matrix cores.  In the
    // last iteration the last block is loaded again (buffer st ^ 1 is not
    // read any more, and the loads have landed before the epilogue reuses
    // LDS), which keeps the MFMA stream free of branches.
    const int64_t kn = kb + 1 < kc1 ? kb + 1 : kc1 - 1;
    const v4i(*L)[64] = stage.lds[st];
    // fragments are read two rows ahead (short rows would not cover the LDS
    // latency with one)
    v4i fa[S], fb[S];
    fa[TM] = L[TM][lane];
#pragma unroll
    for (int u = R.ulo[TM]; u <= R.uhi[TM]; u++) fb[u] = L[S + u][lane];
    if (TM > 0) {
      fa[TM - 1] = L[TM - 1][lane];
#pragma unroll
      for (int u = R.uhi[TM] + 1; u <= R.uhi[TM > 0 ? TM - 1 : 0]; u++) fb[u] = L[S + u][lane];
    }
#pragma unroll
    for (int t = TM; t >= 0; t--) {
      if (t > 1) {
        fa[t - 2] = L[t - 2][lane];
#pragma unroll
        for (int u = R.uhi[t - 1] + 1; u <= R.uhi[t - 2]; u++) fb[u] = L[S + u][lane];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = R.ulo[t]; u <= R.uhi[t]; u++) {
        acc[t + u - D0] =
            __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[t], fb[u], acc[t + u - D0], 0, 0, 0);
        const int m = R.pre[t] + u - R.ulo[t];
        if (m < NDMA) {
          stage.template load_one<W>(st ^ 1, kn, m);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
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
__global__ __launch_bounds__(256) void ozq_gemm_kernel(GemmBatch g, OzLayout o,
                                                       const signed char* Asl,
                                                       const signed char* Bsl, const int* ea,
                                                       const int* fb, int64_t kc0, int64_t kc1,
                                                       int beta, int band) {
  __shared__ v4i lds[2][2 * S][64];
  static_assert(nslots(S) * 32 * 32 * sizeof(double) <= sizeof(lds), "epilogue LDS");
  static_assert(first_cut(S) <= 16, "wave 0 keeps at most 16 accumulators");

  const int64_t t = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
  const int64_t per = o.rb * o.cb;
  const int64_t b = t / per;
  int64_t rbi, cbi;
  banded_tile(t % per, o.rb, o.cb, band, rbi, cbi);
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
int run_ozaki_qd(const GemmBatch& g, char* ws, hipStream_t s, int band) {
  OzLayout o = oz_layout(4, g.m, g.n, g.l, S);
  const OzWs w = oz_ws(ws, o, g.batch);
  signed char *Asl = w.Asl, *Bsl = w.Bsl;
  const int *ea = w.ea, *fb = w.fb;
  int rc = launch_oz_exponents(g, o, w, s);
  if (rc) return rc;
  if ((rc = launch_oz_slice(4, g, o, w, s))) return rc;
  const int64_t nblk = o.rb * o.cb * g.batch;
  if (nblk > INT32_MAX) return set_error(DDQD_E_UNSUPPORTED, "grid too large");
  for (int64_t kc0 = 0; kc0 < o.kb; kc0 += kKChunk / 32) {
    const int64_t kc1 = kc0 + kKChunk / 32 < o.kb ? kc0 + kKChunk / 32 : o.kb;
    launch_timed("ozq_gemm_kernel", ozq_gemm_kernel<S>, dim3((unsigned)nblk), dim3(256), 0, s, g,
                 o, (const signed char*)Asl, (const signed char*)Bsl, (const int*)ea,
                 (const int*)fb, kc0, kc1, kc0 == 0 ? g.beta : 1, band);
    if ((rc = check_launch("ozq_gemm_kernel"))) return rc;
  }
  return DDQD_OK;
}

}  // namespace

int ozaki_qd_default_slices() { return 31; }

size_t ozaki_qd_workspace(int64_t m, int64_t n, int64_t l, int64_t batch, int slices) {
  const int S = slices == 0 ? ozaki_qd_default_slices() : slices;
  if (S < kMinS || S > kMaxS || m <= 0 || n <= 0 || l <= 0) return 0;
  OzLayout o = oz_layout(4, m, n, l, S);
  return oz_workspace_bytes(o, batch);
}

int launch_ozaki_qd(const GemmBatch& g, int slices, void* ws, size_t ws_bytes, hipStream_t s,
                    int band) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return DDQD_OK;
  const int S = slices == 0 ? ozaki_qd_default_slices() : slices;
  if (S < kMinS || S > kMaxS)
    return set_error(DDQD_E_UNSUPPORTED, "QD Ozaki slices must be in %d..%d", kMinS, kMaxS);
  if (ozaki_qd_workspace(g.m, g.n, g.l, g.batch, S) > ws_bytes)
    return set_error(DDQD_E_WORKSPACE, "Ozaki workspace too small");
  char* w = (char*)ws;
  switch (S) {
    case 28: return run_ozaki_qd<28>(g, w, s, band ? band : 4);
    case 29: return run_ozaki_qd<29>(g, w, s, band ? band : 4);
    case 30: return run_ozaki_qd<30>(g, w, s, band ? band : 4);
    case 31: return run_ozaki_qd<31>(g, w, s, band ? band : 4);
  }
  return set_error(DDQD_E_UNSUPPORTED, "slices");
}

}  // namespace ddqd
