// Preparation of the Ozaki-split products (DD and QD): the scaling exponents
// of A's rows and B's columns, and the slicing of every scaled entry into S
// signed 7-bit digits stored as INT8 in MFMA fragment order.  The products
// themselves are in ozaki.hip (DD) and ozaki_qd.hip (QD).
#include <algorithm>
#include <type_traits>

#include "ddqd.h"
#include "common.hpp"
#include "eft.hpp"
#include "ozaki.hpp"

#pragma clang fp contract(off)

namespace ddqd {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// Exponents e with max |leading component| < 2^(e-1), in one launch:
// workgroups [0, nrow) take four rows of A each (one wave per row, all of a
// lane's loads in flight before the reduction; padded rows get 1); the others
// take 64 columns by one 32-row slab of B and store the exponent of each
// column's slab maximum (kNoExp for an all-zero slab).  Exponents are
// monotone in |x|, so the maximum over slabs of these is the exponent of the
// column maximum; the slicing kernel reduces them.
constexpr int kNoExp = -(1 << 20);

// Workgroup `bid` of the exponent pass of batch entry b (see oz_exp_kernel).
__device__ __forceinline__ void oz_exp_body(const CMat& A, const CMat& B, int64_t m, int64_t n,
                                            int64_t l, const OzLayout& o, int64_t nrow, int* ea,
                                            int* part, int64_t b, int64_t bid,
                                            double (&red)[4][64]) {
  const int lane = threadIdx.x % 64;
  if (bid < nrow) {
    const int64_t rows_pad = o.rb * 32;
    const int64_t r = bid * 4 + threadIdx.x / 64;
    if (r >= rows_pad) return;
    double mx = 0.0;
    if (r < m) {
      const double* p = A.p + b * A.bstride + r * A.ld;
      int64_t k = lane;
      for (; k + 960 < l; k += 1024) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; q++) v[q] = p[k + 64 * q];
#pragma unroll
        for (int q = 0; q < 16; q++) mx = fmax(mx, fabs(v[q]));
      }
      for (; k < l; k += 64) mx = fmax(mx, fabs(p[k]));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) {
      int ex = 0;
      if (mx > 0.0) frexp(mx, &ex);
      ea[b * rows_pad + r] = ex + 1;
    }
    return;
  }
  const int64_t cols_pad = o.cb * 32;
  const int64_t ncb = (cols_pad + 63) / 64;
  const int64_t jb = bid - nrow;
  const int64_t slab = jb / ncb;
  const int c_in = threadIdx.x % 64, r = threadIdx.x / 64;
  const int64_t c = (jb % ncb) * 64 + c_in;
  const int64_t k0 = slab * 32 + r * 8;
  double mx = 0.0;
  if (c < n) {
    const double* p = B.p + b * B.bstride + c;
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; q++) v[q] = k0 + q < l ? p[(k0 + q) * B.ld] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; q++) mx = fmax(mx, fabs(v[q]));
  }
  red[r][c_in] = mx;
  __syncthreads();
  if (r == 0 && c < cols_pad) {
    mx = fmax(fmax(red[0][c_in], red[1][c_in]), fmax(red[2][c_in], red[3][c_in]));
    int ex = kNoExp;
    if (mx > 0.0) {
      frexp(mx, &ex);
      ex += 1;
    }
    part[(b * o.kb + slab) * cols_pad + c] = ex;
  }
}

__global__ __launch_bounds__(256) void oz_exp_kernel(CMat A, CMat B, int64_t m, int64_t n,
                                                     int64_t l, OzLayout o, int64_t nrow,
                                                     int* ea, int* part) {
  __shared__ double red[4][64];
  oz_exp_body(A, B, m, n, l, o, nrow, ea, part, blockIdx.y, blockIdx.x, red);
}

// The exponent passes of a group's problems: problem q takes workgroups
// [ga.wg[q], ga.wg[q+1]).
__global__ __launch_bounds__(256) void oz_exp_grouped_kernel(OzGroupArgs ga) {
  __shared__ double red[4][64];
  const int q = oz_group_find(ga.wg, ga.count, blockIdx.x);
  const OzProb& p = ga.p[q];
  oz_exp_body(p.g.A, p.g.B, p.g.m, p.g.n, p.g.l, p.o, (p.o.rb * 32 + 3) / 4, p.w.ea, p.w.part,
              0, (int64_t)blockIdx.x - ga.wg[q], red);
}

// Column exponents of B's 32 columns line0.. of batch entry b: the maximum of
// the slab exponents, into xc[32]; the workgroup with write_fb also stores
// them for the product kernel.  All 256 threads take part.
__device__ __forceinline__ void col_exponents(const OzLayout& o, const int* part, int* fb,
                                              int64_t b, int64_t line0, bool write_fb,
                                              int* xc /* __shared__ [8][32] */) {
  const int64_t cols_pad = o.cb * 32;
  const int c = threadIdx.x % 32, r = threadIdx.x / 32;
  int ex = kNoExp;
  for (int64_t sl = r; sl < o.kb; sl += 8) {
    const int v = part[(b * o.kb + sl) * cols_pad + line0 + c];
    ex = v > ex ? v : ex;
  }
  xc[r * 32 + c] = ex;
  __syncthreads();
  if (r == 0) {
#pragma unroll
    for (int q = 1; q < 8; q++) ex = xc[q * 32 + c] > ex ? xc[q * 32 + c] : ex;
    xc[c] = ex;
    if (write_fb) fb[b * cols_pad + line0 + c] = ex;
  }
  __syncthreads();
}

// The work is cut into chunks of 32 lines (rows of A or columns of B) by KB
// 32-k blocks (DD: 4, QD: 2), A's chunks first, then B's; workgroup g takes
// chunks g, g + G, g + 2G, ... (G workgroups per batch entry).  A chunk's P
// planes are read with coalesced loads into registers (along k for A, along
// the columns for B) while the workgroup still slices the previous chunk,
// then pass through LDS.  DD: wave w slices k block w, every lane its whole
// 16-k fragment slot (16 bytes per digit: each store instruction writes a
// whole 1 KB fragment); QD: wave w slices k block w / 2, half w % 2 of the
// slot (8 values, 8 bytes per digit).
//
// Digits of a scaled value r (|r| < 1/2) held as an expansion r0 + r1 (+ r2
// + r3): runs of kRun digits are taken from the leading term alone, then the
// lower terms are scaled by 2^(7 kRun) and merged: DD by FastTwoSum(r0, r1)
// (r0 is 0 or a multiple of 2^(7 kRun) ulp(r0 at the run's start) >= 2 |r1|,
// its precondition), QD by one bottom-up TwoSum pass, which leaves the rest
// within about an ulp of the leading term.  Inside a run the part a digit
// ignores is below 2^(7 kRun - 54) <= 2^-12 of a digit unit, so digits stay in
// [-64, 64] and the remainder after S digits stays below (1/2 + 2^-12) 2^-7S.
//
// Within a run, N_j = rint(2^(7j) r0) is read from t_j = r0 + 1.5 2^(52-7j):
// that sum lies in a binade whose ulp is 2^(-7j), so it is r0 rounded to a
// multiple of 2^(-7j) (nearest, ties to even), and the low 32 bits of its
// encoding are N_j modulo 2^32.  Digit j is N_j - 2^7 N_(j-1) (N_0 = 0), the
// same digit as rint(2^7 x) of the remainder x left by digits 1..j-1 (shifting
// by the even integer 2^7 N_(j-1) keeps ties to even), and |digit| <= 64.
// After kRun digits the remainder 2^(7 kRun) (r0 - (t_kRun - 1.5 2^(52 - 7 kRun)))
// is exact (Sterbenz for the subtraction, a power of two for the scaling).
constexpr int kRun = 6;       // digits per run from the leading term alone
static_assert(kRun == 6, "the merge scales by 2^42 = 2^(7 kRun)");
constexpr int kSliceWgs = 512;  // workgroups of one slicing launch (two per CU)
// 1.5 2^(52 - 7j), j = 1..kRun: r0 + kMagic[j - 1] rounds r0 to a multiple of 2^(-7j)
constexpr double kMagic[kRun] = {0x1.8p45, 0x1.8p38, 0x1.8p31, 0x1.8p24, 0x1.8p17, 0x1.8p10};

struct SliceChunk {
  int side;            // 0: rows of A, 1: columns of B
  int64_t blk, kg;     // 32-line block, group of KB k blocks
};

__device__ __forceinline__ SliceChunk slice_chunk(const OzLayout& o, int64_t ch, int64_t kgroups) {
  const int64_t na = o.rb * kgroups;
  SliceChunk c;
  c.side = ch < na ? 0 : 1;
  const int64_t x = c.side == 0 ? ch : ch - na;
  c.blk = x / kgroups;
  c.kg = x % kgroups;
  return c;
}

// Issues the loads of one chunk's 32 x 32 KB values (4 KB per thread and
// plane), every load in flight before the first use; values outside the
// matrix read as zero.
template <int P, int KB>
__device__ __forceinline__ void slice_load(const CMat& A, const CMat& B, int64_t m, int64_t n,
                                           int64_t l, int64_t b, const SliceChunk& c,
                                           double (&v)[P][4 * KB]) {
  constexpr int K = 32 * KB;
  const CMat X = c.side == 0 ? A : B;
  const int64_t lines_live = c.side == 0 ? m : n;
  const double* base = X.p + b * X.bstride;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4 * KB; j++) {
    const int e = t + 256 * j;
    const int ln = c.side == 0 ? e / K : e % 32;
    const int kk = c.side == 0 ? e % K : e / 32;
    const int64_t line = c.blk * 32 + ln, k = c.kg * K + kk;
    const bool in = line < lines_live && k < l;
    const int64_t idx = in ? (c.side == 0 ? line * X.ld + k : k * X.ld + line) : 0;
#pragma unroll
    for (int q = 0; q < P; q++) v[q][j] = in ? base[q * X.ps + idx] : 0.0;
  }
}

// The digits of chunk `cur` of batch entry b, whose values (unscaled) are in
// `tile`; xc is scratch for B's column exponents.  All 256 threads take part.
template <int P, int S, int KB>
__device__ __forceinline__ void slice_digits(const OzLayout& o, const int* ea, const int* part,
                                             int* fb, signed char* Asl, signed char* Bsl,
                                             int64_t b, const SliceChunk& cur,
                                             double (&tile)[P][32][32 * KB + 1], int* xc) {
  constexpr int V = 4 * KB;  // values per lane: the whole 16-k slot (KB = 4) or half of it
  static_assert(KB == 4 || KB == 2, "four waves cover KB k blocks");
  using Word = typename std::conditional<V == 16, uint4, uint2>::type;
  const int t = threadIdx.x, w = t / 64, lane = t % 64;
  const int64_t line0 = cur.blk * 32;
  // uniform per workgroup
  if (cur.side == 1) col_exponents(o, part, fb, b, line0, cur.kg == 0, xc);
  const int wk = KB == 4 ? w : w / 2, half = KB == 4 ? 0 : w % 2;
  const int64_t kb = cur.kg * KB + wk;
  if (kb >= o.kb) return;  // past the last K block (no barrier follows in this pass)
  const int ln = lane % 32, k0 = wk * 32 + 16 * (lane / 32) + 8 * half;
  const int ex = cur.side == 0 ? ea[b * (o.rb * 32) + line0 + ln] : xc[ln];
  double r[P][V];
#pragma unroll
  for (int q = 0; q < V; q++)
#pragma unroll
    for (int p = 0; p < P; p++) r[p][q] = ldexp(tile[p][ln][k0 + q], -ex);
  // an input whose terms overlap is brought into shape first (exact)
#pragma unroll
  for (int q = 0; q < V; q++) {
    if constexpr (P == 2) {
      two_sum(r[0][q], r[1][q], r[0][q], r[1][q]);
    } else {
      double a2, a3, a1, b2, a0, b1;
      two_sum(r[2][q], r[3][q], a2, a3);
      two_sum(r[1][q], a2, a1, b2);
      two_sum(r[0][q], a1, a0, b1);
      r[0][q] = a0;
      r[1][q] = b1;
      r[2][q] = b2;
      r[3][q] = a3;
    }
  }
  signed char* dst = (cur.side == 0 ? Asl + b * o.a_bytes : Bsl + b * o.b_bytes) +
                     (cur.blk * o.kb + kb) * S * (int64_t)kOzFrag + lane * 16 + 8 * half;
#pragma unroll 1
  for (int s0 = 0; s0 < S; s0 += kRun) {
    uint32_t prev[V];
    double tl[V];  // t_j of the run's last digit
#pragma unroll
    for (int q = 0; q < V; q++) prev[q] = 0u;
#pragma unroll
    for (int j = 0; j < kRun; j++) {
      if (s0 + j < S) {
        const double magic = kMagic[j];
        uint32_t x[V / 4];
#pragma unroll
        for (int q = 0; q < V / 4; q++) x[q] = 0u;
#pragma unroll
        for (int q = 0; q < V; q++) {
          const double tq = r[0][q] + magic;
          const uint32_t nj = (uint32_t)__builtin_bit_cast(uint64_t, tq);
          const uint32_t d = nj - (prev[q] << 7);
          prev[q] = nj;
          tl[q] = tq;
          x[q / 4] |= (d & 0xffu) << (8 * (q % 4));
        }
        *reinterpret_cast<Word*>(dst + (s0 + j) * (int64_t)kOzFrag) = __builtin_bit_cast(Word, x);
      }
    }
    if (s0 + kRun >= S) break;  // no digits left: the remainder is not needed
#pragma unroll
    for (int q = 0; q < V; q++) {
      const double rem = (r[0][q] - (tl[q] - kMagic[kRun - 1])) * 0x1p42;
      if constexpr (P == 2) {
        fast_two_sum(rem, r[1][q] * 0x1p42, r[0][q], r[1][q]);
      } else {
        // remainder rem + 2^42 (r1 + r2 + r3), all terms exact; one bottom-up
        // TwoSum pass keeps the sum and brings it to the front
        double a2, a3, a1, b2, a0, b1;
        two_sum(r[2][q] * 0x1p42, r[3][q] * 0x1p42, a2, a3);
        two_sum(r[1][q] * 0x1p42, a2, a1, b2);
        two_sum(rem, a1, a0, b1);
        r[0][q] = a0;
        r[1][q] = b1;
        r[2][q] = b2;
        r[3][q] = a3;
      }
    }
  }
}

// The loaded values of a chunk into the LDS tile (after a barrier that every
// reader of the previous chunk has passed).
template <int P, int KB>
__device__ __forceinline__ void slice_to_tile(const SliceChunk& c, const double (&v)[P][4 * KB],
                                              double (&tile)[P][32][32 * KB + 1]) {
  constexpr int K = 32 * KB;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4 * KB; j++) {
    const int e = t + 256 * j;
    const int ln = c.side == 0 ? e / K : e % 32;
    const int kk = c.side == 0 ? e % K : e / 32;
#pragma unroll
    for (int q = 0; q < P; q++) tile[q][ln][kk] = v[q][j];
  }
}

template <int P, int S>
__global__ __launch_bounds__(256) void oz_slice_kernel(CMat A, CMat B, int64_t m, int64_t n,
                                                       int64_t l, OzLayout o, const int* ea,
                                                       const int* part, int* fb,
                                                       signed char* Asl, signed char* Bsl) {
  constexpr int KB = oz_slice_kb(P);
  __shared__ double tile[P][32][32 * KB + 1];
  __shared__ int xc[8 * 32];
  const int64_t b = blockIdx.z;
  const int64_t kgroups = (o.kb + KB - 1) / KB;
  const int64_t nchunks = (o.rb + o.cb) * kgroups;
  int64_t ch = blockIdx.x;
  if (ch >= nchunks) return;  // uniform per workgroup
  double v[P][4 * KB];
  SliceChunk c = slice_chunk(o, ch, kgroups);
  slice_load<P, KB>(A, B, m, n, l, b, c, v);
  for (; ch < nchunks; ch += gridDim.x) {
    __syncthreads();  // the previous chunk's readers of tile and xc are done
    slice_to_tile<P, KB>(c, v, tile);
    __syncthreads();
    const SliceChunk cur = c;
    if (ch + gridDim.x < nchunks) {  // the next chunk's loads fly during the slicing
      c = slice_chunk(o, ch + gridDim.x, kgroups);
      slice_load<P, KB>(A, B, m, n, l, b, c, v);
    }
    slice_digits<P, S, KB>(o, ea, part, fb, Asl, Bsl, b, cur, tile, xc);
  }
}

// The slicing of a group's problems (DD): one persistent grid over the
// concatenated chunk lists, problem q owning chunks [ga.chunk[q],
// ga.chunk[q+1]); the same digits as the single product's launch.
template <int S>
__global__ __launch_bounds__(256) void oz_slice_grouped_kernel(OzGroupArgs ga) {
  constexpr int KB = oz_slice_kb(2);
  __shared__ double tile[2][32][32 * KB + 1];
  __shared__ int xc[8 * 32];
  const int64_t total = ga.chunk[ga.count];
  int64_t G = blockIdx.x;
  if (G >= total) return;  // uniform per workgroup
  double v[2][4 * KB];
  int q = oz_group_find(ga.chunk, ga.count, G);
  SliceChunk c = slice_chunk(ga.p[q].o, G - ga.chunk[q], (ga.p[q].o.kb + KB - 1) / KB);
  {
    const GemmBatch& g = ga.p[q].g;
    slice_load<2, KB>(g.A, g.B, g.m, g.n, g.l, 0, c, v);
  }
  for (; G < total; G += gridDim.x) {
    __syncthreads();
    slice_to_tile<2, KB>(c, v, tile);
    __syncthreads();
    const SliceChunk cur = c;
    const int qc = q;
    if (G + gridDim.x < total) {
      q = oz_group_find(ga.chunk, ga.count, G + gridDim.x);
      c = slice_chunk(ga.p[q].o, G + gridDim.x - ga.chunk[q], (ga.p[q].o.kb + KB - 1) / KB);
      const GemmBatch& g = ga.p[q].g;
      slice_load<2, KB>(g.A, g.B, g.m, g.n, g.l, 0, c, v);
    }
    const OzProb& p = ga.p[qc];
    slice_digits<2, S, KB>(p.o, p.w.ea, p.w.part, p.w.fb, p.w.Asl, p.w.Bsl, 0, cur, tile, xc);
  }
}

}  // namespace

int launch_oz_exponents(const GemmBatch& g, const OzLayout& o, const OzWs& w, hipStream_t s) {
  const int64_t nrow = (o.rb * 32 + 3) / 4;
  const int64_t ncol = ((o.cb * 32 + 63) / 64) * o.kb;
  if (nrow + ncol > INT32_MAX || g.batch > 65535)
    return set_error(DDQD_E_UNSUPPORTED, "matrix too large for one Ozaki launch");
  launch_timed("oz_exp_kernel", oz_exp_kernel, dim3((unsigned)(nrow + ncol), (unsigned)g.batch),
               dim3(256), 0, s, g.A, g.B, g.m, g.n, g.l, o, nrow, w.ea, w.part);
  return check_launch("oz_exp_kernel");
}

namespace {

// Workgroups per batch entry: kSliceWgs over the batch, at most one per chunk.
inline int64_t slice_grid(int P, const GemmBatch& g, const OzLayout& o) {
  const int64_t nchunks = oz_slice_chunks(o, P);
  const int64_t per = std::max<int64_t>(1, kSliceWgs / std::max<int64_t>(1, g.batch));
  return std::min(nchunks, per);
}

template <int S>
int slice_dd(const GemmBatch& g, const OzLayout& o, const OzWs& w, hipStream_t s) {
  const int64_t grid = slice_grid(2, g, o);
  launch_timed("oz_slice_kernel", oz_slice_kernel<2, S>, dim3((unsigned)grid, 1, (unsigned)g.batch),
               dim3(256), 0, s, g.A, g.B, g.m, g.n, g.l, o, (const int*)w.ea, (const int*)w.part,
               w.fb, w.Asl, w.Bsl);
  return check_launch("oz_slice_kernel");
}

template <int S>
int slice_qd(const GemmBatch& g, const OzLayout& o, const OzWs& w, hipStream_t s) {
  const int64_t grid = slice_grid(4, g, o);
  launch_timed("oz_slice_kernel", oz_slice_kernel<4, S>, dim3((unsigned)grid, 1, (unsigned)g.batch),
               dim3(256), 0, s, g.A, g.B, g.m, g.n, g.l, o, (const int*)w.ea, (const int*)w.part,
               w.fb, w.Asl, w.Bsl);
  return check_launch("oz_slice_kernel");
}

template <int S>
int slice_grouped(const OzGroupArgs& ga, hipStream_t s) {
  const int64_t grid = std::min<int64_t>(ga.chunk[ga.count], kSliceWgs);
  prof_begin(s);
  hipLaunchKernelGGL((oz_slice_grouped_kernel<S>), dim3((unsigned)grid), dim3(256), 0, s, ga);
  prof_record("oz_slice_grouped_kernel", s);
  return check_launch("oz_slice_grouped_kernel");
}

}  // namespace

int launch_oz_exponents_grouped(const OzGroupArgs& ga, hipStream_t s) {
  const int64_t grid = ga.wg[ga.count];
  if (grid <= 0) return DDQD_OK;
  if (grid > INT32_MAX) return set_error(DDQD_E_UNSUPPORTED, "group too large");
  prof_begin(s);
  hipLaunchKernelGGL(oz_exp_grouped_kernel, dim3((unsigned)grid), dim3(256), 0, s, ga);
  prof_record("oz_exp_grouped_kernel", s);
  return check_launch("oz_exp_grouped_kernel");
}

int launch_oz_slice_grouped(const OzGroupArgs& ga, int S, hipStream_t s) {
  if (ga.chunk[ga.count] <= 0) return DDQD_OK;
  switch (S) {
    case 8: return slice_grouped<8>(ga, s);
    case 9: return slice_grouped<9>(ga, s);
    case 10: return slice_grouped<10>(ga, s);
    case 11: return slice_grouped<11>(ga, s);
    case 12: return slice_grouped<12>(ga, s);
    case 13: return slice_grouped<13>(ga, s);
    case 14: return slice_grouped<14>(ga, s);
    case 15: return slice_grouped<15>(ga, s);
    case 16: return slice_grouped<16>(ga, s);
    case 17: return slice_grouped<17>(ga, s);
    case 18: return slice_grouped<18>(ga, s);
    case 19: return slice_grouped<19>(ga, s);
    case 20: return slice_grouped<20>(ga, s);
  }
  return set_error(DDQD_E_UNSUPPORTED, "slices");
}

int launch_oz_slice(int P, const GemmBatch& g, const OzLayout& o, const OzWs& w, hipStream_t s) {
  if (P == 2) {
    switch (o.S) {
      case 8: return slice_dd<8>(g, o, w, s);
      case 9: return slice_dd<9>(g, o, w, s);
      case 10: return slice_dd<10>(g, o, w, s);
      case 11: return slice_dd<11>(g, o, w, s);
      case 12: return slice_dd<12>(g, o, w, s);
      case 13: return slice_dd<13>(g, o, w, s);
      case 14: return slice_dd<14>(g, o, w, s);
      case 15: return slice_dd<15>(g, o, w, s);
      case 16: return slice_dd<16>(g, o, w, s);
      case 17: return slice_dd<17>(g, o, w, s);
      case 18: return slice_dd<18>(g, o, w, s);
      case 19: return slice_dd<19>(g, o, w, s);
      case 20: return slice_dd<20>(g, o, w, s);
    }
  } else {
    switch (o.S) {
      case 28: return slice_qd<28>(g, o, w, s);
      case 29: return slice_qd<29>(g, o, w, s);
      case 30: return slice_qd<30>(g, o, w, s);
      case 31: return slice_qd<31>(g, o, w, s);
    }
  }
  return set_error(DDQD_E_UNSUPPORTED, "slices");
}

}  // namespace ddqd
