// DD matrix product on INT8 matrix cores by an Ozaki-style split
// (a base kernel for the leaves of Sec. 2's algorithms; not in the paper,
// which predates it).  Steps 1 and 2 run in ozaki_split.hip, steps 3 and 4
// here.
//
// 1. Scale.  For row i of A take e_i with max_k |a_ik| < 2^(e_i - 1) (from the
//    leading components), for column j of B likewise f_j; a'_ik = a_ik 2^-e_i
//    and b'_kj = b_kj 2^-f_j lie in (-1/2, 1/2) exactly.
// 2. Slice.  Each scaled DD value is written as sum_{t=1..S} d_t 2^-7t + r
//    with signed digits d_t in [-64, 64] (round to nearest of 2^7 times the
//    remainder, which is then formed exactly in DD), |r| <= 2^(-7S-1).  The
//    digits are stored as INT8 in the fragment order of the 32x32x32 MFMA:
//    for a 32-row (or 32-column) by 32-k block, lane l's 16 bytes are row
//    (column) l % 32, k = 16 (l / 32) + 0..15.
// 3. Products.  For every diagonal d = t + u <= S + 1 the INT32 sum
//    P_d = sum_{t+u=d} A_t B_u is accumulated exactly on
//    v_mfma_i32_32x32x32_i8 (|P_d| <= S l 65^2 < 2^31 for K chunks of at
//    most 2^14).  A wave owns a 32x32 block of C and keeps all S diagonal
//    accumulators (16 S registers) live, so each K step loads the 2S
//    fragments once and issues S(S+1)/2 MFMAs on them.
// 4. Recombine (epilogue of the same kernel).  Four consecutive diagonals
//    combine exactly in FP64 (2^21 P_d + 2^14 P_d+1 + 2^7 P_d+2 + P_d+3 <
//    2^53); the four group values, scaled by 2^(e_i + f_j - 7(d+3)), are
//    summed by TwoSum into a DD, then C := beta C + alpha value.
//
// Error: slicing and the dropped diagonals d > S + 1 contribute at most about
// l (S + 3) 2^(-7S-2) 2^(e_i + f_j) to entry (i, j); as 2^(e_i + f_j) <= 16
// max|a_i.| max|b_.j|, with S = 16 that is below 2^-105 l max|a_i.| max|b_.j|
// -- the same accuracy class as the FMA kernel.
#include "ddqd.h"
#include "common.hpp"
#include "eft.hpp"
#include "ozaki.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kFrag = kOzFrag;
constexpr int64_t kKChunk = 16384;   // K per exact INT32 accumulation
constexpr int kMinS = 8, kMaxS = 20;

size_t align256(size_t x) { return oz_align256(x); }

// The product kernel: 4 waves (2x2) per 64x64 tile of C, one 32x32 block per
// wave with S INT32 diagonal accumulators (16 S accumulator registers).
// Fragments move global -> LDS by direct loads (global_load_lds_dwordx4, no
// registers): per K block the workgroup stages 4 S fragments of 1 KB (the S
// slices of its two row blocks of A and two column blocks of B; wave w loads
// group w), double-buffered.  Each wave then holds its S B fragments in
// registers and reads one A fragment at a time from LDS.
// Tile (tm, tn) of batch entry b (the kernels below pick the tile).
template <int S>
__device__ __forceinline__ void oz_gemm_tile(const GemmBatch& g, const OzLayout& o,
                                             const signed char* Asl, const signed char* Bsl,
                                             const int* ea, const int* fb, int64_t b,
                                             int64_t tm, int64_t tn, int64_t kc0, int64_t kc1,
                                             int beta, v4i (&lds)[2][4 * S][64]) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wr = w / 2, wc = w % 2;
  const int64_t rb = 2 * tm + wr, cb = 2 * tn + wc;

  // fragment group this wave stages: 0, 1 = A row blocks 2tm, 2tm+1; 2, 3 = B column blocks
  const signed char* src =
      w < 2 ? Asl + b * o.a_bytes + (2 * tm + w) * o.kb * S * (int64_t)kFrag
            : Bsl + b * o.b_bytes + (2 * tn + (w - 2)) * o.kb * S * (int64_t)kFrag;
  src += lane * 16;
  // the wave index as a scalar, so LDS destinations are scalar arithmetic
  const int wu = __builtin_amdgcn_readfirstlane(w);
  auto stage_one = [&](int st, int64_t kb, int s) {
    __builtin_amdgcn_global_load_lds(
        (const void*)(src + (kb * S + s) * (int64_t)kFrag),
        (__attribute__((address_space(3))) void*)&lds[st][wu * S + s][0], 16, 0, 0);
  };
  auto stage = [&](int st, int64_t kb) {
#pragma unroll
    for (int s = 0; s < S; s++) stage_one(st, kb, s);
  };

  // this lane's 16 outputs: column cb*32 + lane % 32, rows 8 (q / 4) + 4 (lane / 32) + q % 4
  const double* Cb_ro = g.C.p + b * g.C.bstride;
  double* Cb = g.C.p + b * g.C.bstride;

  // K blocks [kc0, kc1): one exact INT32 accumulation (the host splits
  // longer K into chunks and accumulates them into C with beta = 1).
  // Pipeline: registers hold all 2S fragments of block kb while its MFMAs
  // run; A slice ta and B slice S-1-ta are dead after row ta of the triangle,
  // and are reloaded there from LDS with block kb+1's fragments.  LDS buffer
  // kb % 2 is refilled by DMA with block kb+2 once every wave has read it.
  {
    v16i acc[S];
#pragma unroll
    for (int d = 0; d < S; d++)
#pragma unroll
      for (int q = 0; q < 16; q++) acc[d][q] = 0;
    v4i fa[S], fbv[S];
    stage(0, kc0);
    if (kc0 + 1 < kc1) stage(1, kc0 + 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < S; s2++) {
      fa[s2] = lds[0][wr * S + s2][lane];
      fbv[s2] = lds[0][2 * S + wc * S + s2][lane];
    }
    for (int64_t kb = kc0; kb < kc1; kb++) {
      const int st = (int)((kb - kc0) & 1);
      // all waves have read buffer st (block kb) and block kb+1 has landed
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      // block kb+2 goes into buffer st, one slice after each MFMA of the
      // first row, so the DMA issue hides behind the matrix cores.  Near the
      // end the last block is loaded again (harmless: buffer st is not read
      // before it is refilled), which keeps the MFMA stream free of branches.
      const int64_t kn = kb + 2 < kc1 ? kb + 2 : kc1 - 1;
      // The reloads are unconditional (after the last block they read a
      // stale buffer and are never used), which keeps the MFMA stream free
      // of branches.  A slice is reloaded one row after its last use, so the
      // LDS write into its registers never waits on the MFMA still reading
      // them: fa[ta] (last used by the final MFMA of row ta) after row ta+1,
      // fbv[S-1-ta] (last used by the first MFMA of row ta) after row ta.
#pragma unroll
      for (int ta = 0; ta < S; ta++) {
#pragma unroll
        for (int ub = S - 1 - ta; ub >= 0; ub--) {
          acc[ta + ub] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[ta], fbv[ub], acc[ta + ub], 0,
                                                               0, 0);
          if (ta == 0) {
            stage_one(st, kn, S - 1 - ub);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if (ta > 0) fa[ta - 1] = lds[st ^ 1][wr * S + ta - 1][lane];
        fbv[S - 1 - ta] = lds[st ^ 1][2 * S + wc * S + (S - 1 - ta)][lane];
        __builtin_amdgcn_sched_barrier(0);
      }
      fa[S - 1] = lds[st ^ 1][wr * S + S - 1][lane];
    }
    __builtin_amdgcn_s_waitcnt(0);  // the last blocks' loads land before LDS is released
    // recombine: value = 2^(e_i + f_j) sum_d 2^(-7 (d + 2)) P_d, d = 0..S-1,
    // four outputs at a time (scheduling barriers keep the temporaries of
    // only those four live).
    // Opaque copy of the lane index: the epilogue's row and address arithmetic
    // derives from it, so none of it is hoisted into (and kept live through)
    // the MFMA loop.
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int rb2 = 4 * (ln / 32);
    const int64_t col = cb * 32 + ln % 32;
    const int fexp = col < g.n ? fb[b * (o.cb * 32) + col] : 0;
    // all sixteen row exponents in flight at once (the fragment registers
    // are free by now), not one group's latency after another
    int eaq[16];
#pragma unroll
    for (int q = 0; q < 16; q++) {
      const int64_t r = rb * 32 + 8 * (q / 4) + rb2 + q % 4;
      eaq[q] = r < g.m ? ea[b * (o.rb * 32) + r] : 0;
    }
#pragma unroll
    for (int q4 = 0; q4 < 4; q4++) {
      __builtin_amdgcn_sched_barrier(0);
      int sc[4];
      int64_t row[4];
#pragma unroll
      for (int z = 0; z < 4; z++) {
        row[z] = rb * 32 + 8 * q4 + rb2 + z;
        sc[z] = row[z] < g.m ? eaq[4 * q4 + z] + fexp : 0;
      }
      double sh[4], sl[4];
#pragma unroll
      for (int gi = 0; gi < (S + 3) / 4; gi++) {
        double G[4] = {0.0, 0.0, 0.0, 0.0};
        int last = 0;
#pragma unroll
        for (int zz = 0; zz < 4; zz++) {
          const int d = 4 * gi + zz;
          if (d < S) {
#pragma unroll
            for (int z = 0; z < 4; z++)  // exact: integers < 2^53
              G[z] = __builtin_fma(G[z], 128.0, (double)acc[d][4 * q4 + z]);
            last = d;
          }
        }
#pragma unroll
        for (int z = 0; z < 4; z++) {
          const double part = ldexp(G[z], sc[z] - 7 * (last + 2));
          if (gi == 0) {
            sh[z] = part;
            sl[z] = 0.0;
          } else {
            double err;
            two_sum(sh[z], part, sh[z], err);
            sl[z] += err;
          }
        }
      }
#pragma unroll
      for (int z = 0; z < 4; z++) {
        if (row[z] >= g.m || col >= g.n) continue;
        dd_t v;
        two_sum(sh[z], sl[z], v.hi, v.lo);
        if (g.alpha < 0) v = dd_neg(v);
        const int64_t off = row[z] * g.C.ld + col;
        if (beta) v = dd_add(dd_t{Cb_ro[off], Cb_ro[g.C.ps + off]}, v);
        Cb[off] = v.hi;
        Cb[g.C.ps + off] = v.lo;
      }
    }
  }
}

template <int S>
__global__ __launch_bounds__(256) void oz_gemm_kernel(GemmBatch g, OzLayout o,
                                                      const signed char* Asl,
                                                      const signed char* Bsl, const int* ea,
                                                      const int* fb, int64_t tiles_m,
                                                      int64_t tiles_n, int64_t kc0, int64_t kc1,
                                                      int beta, int band) {
  __shared__ v4i lds[2][4 * S][64];
  const int64_t t = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
  const int64_t per = tiles_m * tiles_n;
  int64_t tm, tn;
  banded_tile(t % per, tiles_m, tiles_n, band, tm, tn);
  oz_gemm_tile<S>(g, o, Asl, Bsl, ea, fb, t / per, tm, tn, kc0, kc1, beta, lds);
}

// The products of a group: problem q owns tiles [ga.tile[q], ga.tile[q+1])
// of the concatenated list, each computed exactly as by oz_gemm_kernel (one
// K chunk: every problem of a group has l <= 16384).
template <int S>
__global__ __launch_bounds__(256) void oz_gemm_grouped_kernel(OzGroupArgs ga) {
  __shared__ v4i lds[2][4 * S][64];
  const int64_t t = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
  const int q = oz_group_find(ga.tile, ga.count, t);
  const OzProb& p = ga.p[q];
  const int64_t tiles_m = p.o.rb / 2, tiles_n = p.o.cb / 2;
  int64_t tm, tn;
  banded_tile(t - ga.tile[q], tiles_m, tiles_n, 4, tm, tn);
  oz_gemm_tile<S>(p.g, p.o, p.w.Asl, p.w.Bsl, p.w.ea, p.w.fb, 0, tm, tn, 0, p.o.kb, p.g.beta,
                  lds);
}

template <int S>
int run_ozaki_grouped(const OzGroupArgs& ga, hipStream_t s) {
  int rc;
  if ((rc = launch_oz_exponents_grouped(ga, s))) return rc;
  if ((rc = launch_oz_slice_grouped(ga, S, s))) return rc;
  const int64_t nblk = ga.tile[ga.count];
  if (nblk <= 0) return DDQD_OK;
  if (nblk > INT32_MAX) return set_error(DDQD_E_UNSUPPORTED, "group too large");
  prof_begin(s);
  hipLaunchKernelGGL(oz_gemm_grouped_kernel<S>, dim3((unsigned)nblk), dim3(256), 0, s, ga);
  prof_record("oz_gemm_grouped_kernel", s);
  return check_launch("oz_gemm_grouped_kernel");
}

template <int S>
int run_ozaki(const GemmBatch& g, char* ws, hipStream_t s, int band) {
  OzLayout o = oz_layout(2, g.m, g.n, g.l, S);
  const OzWs w = oz_ws(ws, o, g.batch);
  signed char *Asl = w.Asl, *Bsl = w.Bsl;
  const int *ea = w.ea, *fb = w.fb;
  int rc = launch_oz_exponents(g, o, w, s);
  if (rc) return rc;
  if ((rc = launch_oz_slice(2, g, o, w, s))) return rc;
  const int64_t tm = o.rb / 2, tn = o.cb / 2;
  const int64_t nblk = tm * tn * g.batch;
  if (nblk > INT32_MAX) return set_error(DDQD_E_UNSUPPORTED, "grid too large");
  for (int64_t kc0 = 0; kc0 < o.kb; kc0 += kKChunk / 32) {
    const int64_t kc1 = kc0 + kKChunk / 32 < o.kb ? kc0 + kKChunk / 32 : o.kb;
    launch_timed("oz_gemm_kernel", oz_gemm_kernel<S>, dim3((unsigned)nblk), dim3(256), 0, s, g, o,
                 (const signed char*)Asl, (const signed char*)Bsl, (const int*)ea,
                 (const int*)fb, tm, tn, kc0, kc1, kc0 == 0 ? g.beta : 1, band);
    if ((rc = check_launch("oz_gemm_kernel"))) return rc;
  }
  return DDQD_OK;
}

}  // namespace

int ozaki_qd_default_slices();
size_t ozaki_qd_workspace(int64_t m, int64_t n, int64_t l, int64_t batch, int slices);
int launch_ozaki_qd(const GemmBatch& g, int slices, void* ws, size_t ws_bytes, hipStream_t s,
                    int band);

int ozaki_default_slices(int P) { return P == 4 ? ozaki_qd_default_slices() : 16; }

bool ozaki_slices_ok(int P, int slices) {
  if (slices == 0) return true;
  return P == 4 ? ozaki_qd_workspace(1, 1, 1, 1, slices) != 0 : slices >= kMinS && slices <= kMaxS;
}

static size_t ozaki_dd_workspace(int64_t m, int64_t n, int64_t l, int64_t batch, int slices) {
  const int S = slices == 0 ? ozaki_default_slices(2) : slices;
  if (S < kMinS || S > kMaxS || m <= 0 || n <= 0 || l <= 0) return 0;
  OzLayout o = oz_layout(2, m, n, l, S);
  return oz_workspace_bytes(o, batch);
}

size_t ozaki_workspace(int P, int64_t m, int64_t n, int64_t l, int64_t batch, int slices) {
  return P == 4 ? ozaki_qd_workspace(m, n, l, batch, slices)
                : ozaki_dd_workspace(m, n, l, batch, slices);
}

// Workspace of the grouped form for one problem (DD, one K chunk) at S slices.
size_t ozaki_grouped_bytes(const GemmBatch& g, int S) {
  return oz_align256(oz_workspace_bytes(oz_layout(2, g.m, g.n, g.l, S), 1));
}

// Unrelated DD products (batch = 1 each, 0 < l <= 16384) at S slices in
// launches of up to kOzGroup problems: one exponent, one slicing and one
// product launch per group.  ws holds ozaki_grouped_bytes of every problem,
// in order.
int launch_ozaki_grouped(const GemmBatch* probs, int count, int S, char* ws, size_t ws_bytes,
                         hipStream_t s) {
  if (S < kMinS || S > kMaxS)
    return set_error(DDQD_E_UNSUPPORTED, "Ozaki slices must be in %d..%d", kMinS, kMaxS);
  size_t off = 0;
  for (int c0 = 0; c0 < count; c0 += kOzGroup) {
    OzGroupArgs ga;
    ga.count = 0;
    ga.wg[0] = ga.chunk[0] = ga.tile[0] = 0;
    for (int i = c0; i < count && i < c0 + kOzGroup; i++) {
      const GemmBatch& g = probs[i];
      if (g.l > kKChunk) return set_error(DDQD_E_UNSUPPORTED, "grouped Ozaki product with l > %lld",
                                          (long long)kKChunk);
      OzProb& p = ga.p[ga.count];
      p.g = g;
      p.o = oz_layout(2, g.m, g.n, g.l, S);
      const size_t need = ozaki_grouped_bytes(g, S);
      if (off + need > ws_bytes) return set_error(DDQD_E_WORKSPACE, "grouped Ozaki workspace");
      p.w = oz_ws((char*)ws + off, p.o, 1);
      off += need;
      const int c = ga.count++;
      ga.wg[c + 1] = ga.wg[c] + oz_exp_wgs(p.o);
      ga.chunk[c + 1] = ga.chunk[c] + oz_slice_chunks(p.o, 2);
      ga.tile[c + 1] = ga.tile[c] + (p.o.rb / 2) * (p.o.cb / 2);
    }
    if (ga.count == 0) continue;
    int rc;
    switch (S) {
      case 8: rc = run_ozaki_grouped<8>(ga, s); break;
      case 9: rc = run_ozaki_grouped<9>(ga, s); break;
      case 10: rc = run_ozaki_grouped<10>(ga, s); break;
      case 11: rc = run_ozaki_grouped<11>(ga, s); break;
      case 12: rc = run_ozaki_grouped<12>(ga, s); break;
      case 13: rc = run_ozaki_grouped<13>(ga, s); break;
      case 14: rc = run_ozaki_grouped<14>(ga, s); break;
      case 15: rc = run_ozaki_grouped<15>(ga, s); break;
      case 16: rc = run_ozaki_grouped<16>(ga, s); break;
      case 17: rc = run_ozaki_grouped<17>(ga, s); break;
      case 18: rc = run_ozaki_grouped<18>(ga, s); break;
      case 19: rc = run_ozaki_grouped<19>(ga, s); break;
      default: rc = run_ozaki_grouped<20>(ga, s); break;
    }
    if (rc) return rc;
  }
  return DDQD_OK;
}

// band: tile rows per band of the product's tile order (0 = 4); the order
// changes only which workgroups share L2, never a result bit.
int launch_ozaki(int P, const GemmBatch& g, int slices, void* ws, size_t ws_bytes,
                 hipStream_t s, int band) {
  if (P == 4) return launch_ozaki_qd(g, slices, ws, ws_bytes, s, band);
  if (band == 0) band = 4;
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return DDQD_OK;
  const int S = slices == 0 ? ozaki_default_slices(2) : slices;
  if (S < kMinS || S > kMaxS)
    return set_error(DDQD_E_UNSUPPORTED, "Ozaki slices must be in %d..%d", kMinS, kMaxS);
  if (ozaki_dd_workspace(g.m, g.n, g.l, g.batch, S) > ws_bytes)
    return set_error(DDQD_E_WORKSPACE, "Ozaki workspace too small");
  char* w = (char*)ws;
  switch (S) {
    case 8: return run_ozaki<8>(g, w, s, band);
    case 9: return run_ozaki<9>(g, w, s, band);
    case 10: return run_ozaki<10>(g, w, s, band);
    case 11: return run_ozaki<11>(g, w, s, band);
    case 12: return run_ozaki<12>(g, w, s, band);
    case 13: return run_ozaki<13>(g, w, s, band);
    case 14: return run_ozaki<14>(g, w, s, band);
    case 15: return run_ozaki<15>(g, w, s, band);
    case 16: return run_ozaki<16>(g, w, s, band);
    case 17: return run_ozaki<17>(g, w, s, band);
    case 18: return run_ozaki<18>(g, w, s, band);
    case 19: return run_ozaki<19>(g, w, s, band);
    case 20: return run_ozaki<20>(g, w, s, band);
  }
  return set_error(DDQD_E_UNSUPPORTED, "slices");
}

}  // namespace ddqd
