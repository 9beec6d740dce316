// DD matrix product on INT8 matrix cores by modular integer arithmetic (a
// base kernel for the leaves of Sec. 2's algorithms, like the Ozaki split in
// ozaki.hip; not in the paper, which predates both).  Where the split takes
// every product of S digit slices (S(S+1)/2 INT8 products), this form takes
// one INT8 product per modulus of a set of N pairwise coprime moduli and
// rebuilds the exact integer product by the Chinese remainder theorem.
//
// 1. Scale (ozaki_split.hip's exponent pass): e_i with max_k |a_ik| < 2^(e_i-1)
//    for row i of A, f_j likewise for column j of B.
// 2. Integers.  A'_ik = a_ik 2^(P1 - e_i) rounded to an integer (|A'| <= 2^P1;
//    2^(P1-1) for normalised DD input), B' likewise; the rounding moves each
//    by at most 1.
// 3. Residues.  For every modulus m_s the symmetric residue of A' (and B')
//    modulo m_s, |r| <= m_s / 2 <= 128, stored as INT8 in the fragment order
//    of the 32x32x32 MFMA (lane l: line l % 32, k = 16 (l / 32) + 0..15).
// 4. Products.  C_s = A'_s B'_s exactly in INT32 on v_mfma_i32_32x32x32_i8
//    (|C_s| <= kc 2^14 <= 2^30 for K chunks kc <= 2^16), reduced to a
//    symmetric residue c_s of m_s and stored as INT8.
// 5. Rebuild.  X = A' B' is the integer with X = c_s (mod m_s) for every s and
//    |X| < M / 2, M = prod m_s (N is chosen so that M > 2 kc 2^(2 P1)):
//    X / M = frac(sum_s c_s y_s / m_s), y_s = (M / m_s)^-1 mod m_s.  Each term
//    is taken as c_s Z_s, Z_s = floor(y_s 2^160 / m_s), in 160-bit fixed
//    point (the sum mod 2^160; error below |c_s| units of 2^-160 a term), and
//    the signed fraction times M gives X; C_ij = X 2^(e_i + f_j - 2 P1) in DD.
//
// Error: the integers move each operand by at most 2^(e_i - P1) (A) and
// 2^(f_j - P1) (B), so entry (i, j) moves by at most about
// kc 2^(e_i + f_j - P1) <= kc 2^(4 - P1) max|a_i.| max|b_.j| (P1 = 107:
// 2^-103 kc max|a_i.| max|b_.j|); the rebuild adds at most 2^12 M 2^-160
// <= 2^86 units of X (2^(e_i + f_j - 128)) and the DD rounding of the result.
//
// QD.  The integers are T = a 2^(2 P1 + 1 - e) rounded (|T| <= 2^214), split
// T = H 2^108 + L with |H| <= 2^106 and |L| <= 2^107 (1 + 2^-35) (the low
// limbs balanced).  Then
//   A'B' 2^-(430 - e - f) = H_a H_b 2^216 + (H_a L_b + L_a H_b) 2^108 + L_a L_b,
// the last term dropped (at most kc 2^(e + f - 216)).  Both products run on
// one set of N moduli (M > kc 2^215 (1 + 2^-35), the cross term's bound; the
// cross product is one product over 2 K, [H_a L_a] by [L_b; H_b]): the
// residues of H and L sit in alternate K blocks (A: H then L, B: L then H),
// so the cross product reads every block and H_a H_b every other one.  The
// rebuild takes F_hh in 270-bit fixed point (X_hh exact to far below one
// unit) and F_x in 162-bit (X_x within 2^77 units, needed within 2^106), the
// latter taken signed and added 108 bits down (6-bit digits make that a
// whole number of digits), and C = M (F_hh + F_x 2^-108) 2^(e + f - 214)
// from one QD fraction.
// Error: the dropped term and the roundings of the integers, each at most
// about kc 2^(e + f - 216) (in all kc 2^(e + f - 215) <= kc 2^-211 max|a_i.|
// max|b_.j|), and the QD roundings of the rebuild.
#include "ddqd.h"
#include "common.hpp"
#include "eft.hpp"
#include "ozaki.hpp"
#include "qd.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>

#pragma clang fp contract(off)

namespace ddqd {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kCrtMaxN = 32;
constexpr int kP1 = 107;              // |A'| <= 2^107
constexpr int64_t kChunk = 65536;     // K per exact INT32 product
// A product workgroup's tile is TB x TB blocks of 32 (TB = 4: 128 x 128, each
// wave 2 x 2 blocks; TB = 8: 256 x 256, each wave 4 x 4 blocks).

// The moduli: pairwise coprime, largest first (each <= 256, so residues fit
// INT8); the first N are used.
constexpr int kModuli[kCrtMaxN] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223,
                                   217, 211, 199, 197, 193, 191, 181, 179, 173, 167, 163,
                                   157, 151, 149, 139, 137, 131, 127, 113, 109, 107};

// Residue constants (kernel argument): m_s, 1 / m_s rounded, 2^36 and 2^72
// modulo m_s.
struct CrtResidue {
  int N;
  double m[kCrtMaxN], inv[kCrtMaxN], t36[kCrtMaxN], t72[kCrtMaxN];
};

// Rebuild constants (kernel argument): Z_s = floor(y_s 2^160 / m_s) in 7-bit
// digits, laid out as the rebuild's MFMA A operand, and M 2^-160 as a DD.
constexpr int kDigitBits = 7;  // digits of the 160-bit fixed point: 23 of 7 bits (161 bits)
constexpr int kDigits = 23;
struct CrtRebuild {
  int N;
  // the rebuild's MFMA operand: lane L holds digit L % 32 of Z_s for
  // s = 16 (L / 32) + 0..15 (one byte each; zero past N and past kDigits)
  uint32_t zd[64][4];
  double mhi, mlo;
};

// QD rebuild constants: Z_s = floor(y_s 2^270 / m_s) in 6-bit digits (45;
// digits 18..44 are floor(y_s 2^162 / m_s), the cross term's) as MFMA A
// operands laid out like CrtRebuild's: digits 0..31 (zh0), 32..44 (zh1),
// 18..44 (zx, as digits 0..26), and M 2^-256 as a QD.
constexpr int kDigitsQ = 45;  // 270-bit fixed point
constexpr int kDigitsX = 27;  // 162-bit (the cross term, 108 bits = 18 digits lower)
struct CrtRebuildQ {
  int N;
  uint32_t zh0[64][4], zh1[64][4], zx[64][4];
  double mq[4];
};

// Product kernel launch description.  Logical K block kb of a line is stored
// block kb kst + koa (A) or kb kst + kob (B); NS residue sets are stored per
// batch entry, of which the first N are multiplied.
struct CrtProd {
  const signed char *Ares, *Bres;
  signed char* Cres;
  int N, NS;
  double m[kCrtMaxN], inv[kCrtMaxN];
  int64_t kst, koa, kob;
  int64_t RB, CB, KB;        // 32-blocks of rows, columns, stored K blocks
  int64_t tiles_m, tiles_n;  // workgroup tiles
  int64_t kb0, kb1;          // K blocks of this chunk (a multiple of 4)
  int64_t batch;
};

// ---- host: constants -------------------------------------------------------

struct Consts {
  CrtResidue res;
  CrtRebuild reb;
  CrtRebuildQ rq;
  double bits;  // log2 M
};

int64_t inv_mod(int64_t a, int64_t m) {  // a^-1 mod m, gcd(a, m) = 1
  int64_t t = 0, nt = 1, r = m, nr = a % m;
  while (nr) {
    const int64_t q = r / nr, tt = t - q * nt, rr = r - q * nr;
    t = nt;
    nt = tt;
    r = nr;
    nr = rr;
  }
  return t < 0 ? t + m : t;
}

Consts make_consts(int N) {
  Consts c{};
  c.res.N = c.reb.N = c.rq.N = N;
  c.bits = 0;
  // M as 32-bit words (at most 256 bits for 32 moduli)
  uint32_t M[9] = {1};
  for (int s = 0; s < N; s++) {
    const int64_t m = kModuli[s];
    c.bits += std::log2((double)m);
    c.res.m[s] = (double)m;
    c.res.inv[s] = 1.0 / (double)m;
    int64_t p36 = 1, p72;
    for (int b = 0; b < 36; b++) p36 = p36 * 2 % m;
    p72 = p36 * p36 % m;
    c.res.t36[s] = (double)p36;
    c.res.t72[s] = (double)p72;
    // y_s = (M / m_s)^-1 mod m_s
    int64_t q = 1;
    for (int t = 0; t < N; t++)
      if (t != s) q = q * (kModuli[t] % m) % m;
    const int64_t y = inv_mod(q, m);
    // Z_s = floor(y 2^160 / m): long division of y 2^160 (32-bit words; the
    // quotient is below 2^160 as y < m)
    uint32_t num[6] = {0, 0, 0, 0, 0, (uint32_t)y}, quo[6];
    uint64_t rem = 0;
    for (int w = 5; w >= 0; w--) {
      const uint64_t cur = (rem << 32) | num[w];
      quo[w] = (uint32_t)(cur / (uint64_t)m);
      rem = cur % (uint64_t)m;
    }
    for (int d = 0; d < kDigits; d++) {
      uint32_t v = 0;
      for (int b = 0; b < kDigitBits; b++) {
        const int i = kDigitBits * d + b;
        if (i < 160) v |= ((quo[i / 32] >> (i % 32)) & 1u) << b;
      }
      const int L = d + 32 * (s / 16), j = s % 16;
      c.reb.zd[L][j / 4] |= v << (8 * (j % 4));
    }
    // Z_s = floor(y 2^270 / m) likewise (QD; y 2^270 = (y 2^14) 2^256)
    uint32_t numq[9] = {0, 0, 0, 0, 0, 0, 0, 0, (uint32_t)y << 14}, quoq[9];
    rem = 0;
    for (int w = 8; w >= 0; w--) {
      const uint64_t cur = (rem << 32) | numq[w];
      quoq[w] = (uint32_t)(cur / (uint64_t)m);
      rem = cur % (uint64_t)m;
    }
    for (int d = 0; d < kDigitsQ; d++) {
      uint32_t v = 0;
      for (int b = 0; b < 6; b++) {
        const int i = 6 * d + b;
        v |= ((quoq[i / 32] >> (i % 32)) & 1u) << b;
      }
      const int j = s % 16, sh = 8 * (j % 4);
      const int L0 = 32 * (s / 16);
      if (d < 32) c.rq.zh0[L0 + d][j / 4] |= v << sh;
      else c.rq.zh1[L0 + d - 32][j / 4] |= v << sh;
      if (d >= kDigitsQ - kDigitsX) c.rq.zx[L0 + d - (kDigitsQ - kDigitsX)][j / 4] |= v << sh;
    }
    // M *= m
    uint64_t carry = 0;
    for (int w = 0; w < 9; w++) {
      const uint64_t v = (uint64_t)M[w] * (uint64_t)m + carry;
      M[w] = (uint32_t)v;
      carry = v >> 32;
    }
  }
  // M 2^-160 as a DD: its leading 53 bits, then the next 53 (truncated)
  auto bit = [&](int i) -> uint64_t { return i < 0 ? 0u : (M[i / 32] >> (i % 32)) & 1u; };
  int top = 9 * 32 - 1;
  while (top > 0 && !bit(top)) top--;
  uint64_t h = 0, lw = 0;
  for (int i = 0; i < 53; i++) h = (h << 1) | bit(top - i);
  for (int i = 53; i < 106; i++) lw = (lw << 1) | bit(top - i);
  const double hi = std::ldexp((double)h, top - 52 - 160);
  const double lo = std::ldexp((double)lw, top - 105 - 160);
  c.reb.mhi = hi;
  c.reb.mlo = lo;
  // M 2^-256 as a QD: four consecutive 53-bit pieces of M (truncated:
  // relative error below 2^-211), each below an ulp of the one before
  for (int p = 0; p < 4; p++) {
    uint64_t w = 0;
    for (int i = 53 * p; i < 53 * p + 53; i++) w = (w << 1) | bit(top - i);
    c.rq.mq[p] = std::ldexp((double)w, top - 53 * p - 52 - 256);
  }
  return c;
}

const Consts& consts(int N) {
  static Consts table[kCrtMaxN + 1];
  static std::once_flag once;
  std::call_once(once, [] {
    for (int n = 1; n <= kCrtMaxN; n++) table[n] = make_consts(n);
  });
  return table[N];
}

int moduli_for_bits(double need) {
  for (int n = 1; n <= kCrtMaxN; n++)
    if (consts(n).bits >= need) return n;
  return 0;
}

// Moduli for K chunks of kc: M > 2 kc 2^(2 P1) (|A'|, |B'| <= 2^P1); QD:
// M > kc 2^215 (1 + 2^-35), the cross term's bound.
int moduli_for(int P, int64_t kc) {
  const double lk = std::log2((double)(kc < 1 ? 1 : kc));
  return moduli_for_bits(P == 4 ? 215.0 + lk + 0.01 : 2.0 * kP1 + lk + 1.0 + 0.01);
}

// ---- layout and workspace ---------------------------------------------------

struct CrtLayout {
  int64_t m, n, l, batch;
  int P, N, TB;
  int64_t RB, CB;  // 32-blocks of rows and columns (multiples of TB)
  int64_t KBo;     // 32-blocks of K (a multiple of 4)
  int64_t KB;      // stored K blocks a line: KBo (DD), 2 KBo (QD: H and L)
  int64_t kc;      // K chunk
  size_t a_bytes, b_bytes, c_bytes;  // residues, all batch entries (c: per product)
};

// 128 x 128 unless `tile` asks for 256 x 256 (the tuner's other candidate):
// the fragments' path from L2 to LDS, not LDS reads or register reuse, bounds
// both (the larger tile moves half the bytes a multiply-add but runs one
// workgroup a compute unit), and the smaller measured faster at n = 1024 and
// 2048.
int crt_tile_blocks(int64_t m, int64_t n, int tile) {
  (void)m;
  (void)n;
  return tile == 256 ? 8 : 4;
}

// K per chunk: the INT32 sums of one product cover kChunk (QD: the cross
// product runs over twice the chunk)
int64_t chunk_k(int P) { return P == 4 ? kChunk / 2 : kChunk; }

CrtLayout crt_layout(int P, int64_t m, int64_t n, int64_t l, int64_t batch, int TB) {
  CrtLayout L;
  L.m = m;
  L.n = n;
  L.l = l;
  L.batch = batch;
  L.P = P;
  L.TB = TB;
  L.RB = (m + 32 * TB - 1) / (32 * TB) * TB;
  L.CB = (n + 32 * TB - 1) / (32 * TB) * TB;
  L.KBo = ((l + 31) / 32 + 3) / 4 * 4;  // two steps of up to two blocks
  L.KB = P == 4 ? 2 * L.KBo : L.KBo;
  L.kc = l < chunk_k(P) ? l : chunk_k(P);
  L.N = moduli_for(P, L.kc);
  L.a_bytes = (size_t)batch * L.N * L.RB * L.KB * kOzFrag;
  L.b_bytes = (size_t)batch * L.N * L.CB * L.KB * kOzFrag;
  L.c_bytes = (size_t)batch * L.N * L.RB * L.CB * kOzFrag;
  return L;
}

// The exponent pass's layout (ozaki_split.hip): rows and columns padded to
// the residues' blocks.
OzLayout exp_layout(const CrtLayout& L) {
  OzLayout o{};
  o.m = L.m;
  o.n = L.n;
  o.l = L.l;
  o.rb = L.RB;
  o.cb = L.CB;
  o.kb = (L.l + 31) / 32;
  o.S = 1;
  return o;
}

struct CrtWs {
  signed char *Ares, *Bres, *Cres, *Cx;  // Cx: QD's cross product
  OzWs e;  // exponents (Asl / Bsl unused)
};

size_t crt_ws_bytes(const CrtLayout& L) {
  const OzLayout o = exp_layout(L);
  return oz_align256(L.a_bytes) + oz_align256(L.b_bytes) +
         (L.P == 4 ? 2 : 1) * oz_align256(L.c_bytes) +
         oz_align256(sizeof(int) * (size_t)(L.batch * (o.rb + o.cb) * 32)) +
         oz_align256(sizeof(int) * (size_t)(L.batch * o.kb * o.cb * 32));
}

CrtWs crt_ws(char* ws, const CrtLayout& L) {
  CrtWs w;
  w.Ares = (signed char*)ws;
  ws += oz_align256(L.a_bytes);
  w.Bres = (signed char*)ws;
  ws += oz_align256(L.b_bytes);
  w.Cres = (signed char*)ws;
  ws += oz_align256(L.c_bytes);
  w.Cx = nullptr;
  if (L.P == 4) {
    w.Cx = (signed char*)ws;
    ws += oz_align256(L.c_bytes);
  }
  const OzLayout o = exp_layout(L);
  w.e.Asl = w.e.Bsl = nullptr;
  w.e.ea = (int*)ws;
  w.e.fb = w.e.ea + L.batch * o.rb * 32;
  ws += oz_align256(sizeof(int) * (size_t)(L.batch * (o.rb + o.cb) * 32));
  w.e.part = (int*)ws;
  return w;
}

// ---- residues ---------------------------------------------------------------
// Workgroup = 32 lines (rows of A or columns of B) by 64 k (two K blocks) of
// one batch entry; A's chunks first, then B's.  Thread t takes line t % 32
// and k = 8 (t / 32) + 0..7: it forms the 8 integers, then for each modulus
// their 8 residues (8 bytes of its line's 16-byte fragment slot; a wave's
// stores cover half a fragment, 512 contiguous bytes).  QD: H and L each, in
// the line's stored blocks 2 kb and 2 kb + 1 (A: H first, B: L first).
template <int P>
__global__ __launch_bounds__(256) void crt_residue_kernel(CMat A, CMat B, int64_t m, int64_t n,
                                                          int64_t l, int64_t RB, int64_t CB,
                                                          int64_t KBo, int64_t KB, int64_t kbe,
                                                          const int* ea, const int* part,
                                                          int* fb, CrtResidue cr,
                                                          signed char* Ares, signed char* Bres) {
  __shared__ int xc[8][32];
  const int64_t b = blockIdx.y;
  const int64_t kchunks = KBo / 2;
  const int64_t ch = blockIdx.x;
  const int side = ch < RB * kchunks ? 0 : 1;
  const int64_t x = side == 0 ? ch : ch - RB * kchunks;
  const int64_t lb = x / kchunks, kc = x % kchunks;
  const int t = threadIdx.x, ln = t % 32, g = t / 32;
  const int64_t line = lb * 32 + ln;
  // the 8 values (loaded first: their latency overlaps the exponent's)
  const CMat X = side == 0 ? A : B;
  const int64_t live = side == 0 ? m : n;
  const double* base = X.p + b * X.bstride;
  const int64_t k0 = kc * 64 + 8 * g;
  double v[P][8];
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const int64_t k = k0 + q;
    const bool in = line < live && k < l;
    const int64_t idx = in ? (side == 0 ? line * X.ld + k : k * X.ld + line) : 0;
#pragma unroll
    for (int c = 0; c < P; c++) v[c][q] = in ? base[c * X.ps + idx] : 0.0;
  }
  // exponent of this line (B: the maximum of the column's slab exponents,
  // four independent loads a pass)
  int ex;
  if (side == 0) {
    ex = ea[b * RB * 32 + line];
  } else {
    const int c = t % 32, r = t / 32;
    int e = -(1 << 20);
    for (int64_t s0 = r; s0 < kbe; s0 += 32) {
      int pv[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int64_t sl = s0 + 8 * u;
        pv[u] = sl < kbe ? part[(b * kbe + sl) * (CB * 32) + lb * 32 + c] : -(1 << 20);
      }
#pragma unroll
      for (int u = 0; u < 4; u++) e = pv[u] > e ? pv[u] : e;
    }
    xc[r][c] = e;
    __syncthreads();
    if (r == 0) {
#pragma unroll
      for (int q = 1; q < 8; q++) e = xc[q][c] > e ? xc[q][c] : e;
      xc[0][c] = e;
      if (kc == 0) fb[b * CB * 32 + lb * 32 + c] = e;
    }
    __syncthreads();
    ex = xc[0][ln];
  }
  // limbs of 36 bits (all exact): DD, A' = d0 + d1 2^36 + d2 2^72; QD,
  // T = sum_j d_j 2^(36 j), H = d3 + d4 2^36 + d5 2^72, L = d0 + d1 2^36 + d2 2^72
  constexpr int NLB = P == 4 ? 6 : 3;
  double d[NLB][8];
  if constexpr (P == 2) {
    const int sh = kP1 - ex;
#pragma unroll
    for (int q = 0; q < 8; q++) {
      double s, e;
      two_sum(v[0][q], v[1][q], s, e);  // normalised (exact)
      const double hs = ldexp(s, sh), h = rint(hs);
      const double lo = rint(ldexp(e, sh) + (hs - h));
      const double c2 = trunc(h * 0x1p-72);
      const double h1 = __builtin_fma(-c2, 0x1p72, h);
      const double c1 = trunc(h1 * 0x1p-36);
      const double c0 = __builtin_fma(-c1, 0x1p36, h1);
      const double l1 = trunc(lo * 0x1p-36);
      const double l0 = __builtin_fma(-l1, 0x1p36, lo);
      d[0][q] = c0 + l0;
      d[1][q] = c1 + l1;
      d[2][q] = c2;
    }
  } else {
    // T = a 2^(2 P1 + 1 - e) rounded: each component rounded with the
    // previous one's fraction carried in (that sum is exact or of terms
    // below 1), then cut into six limbs (|d_j| < 2^38 summed)
    const int sh = 2 * kP1 + 1 - ex;
#pragma unroll
    for (int q = 0; q < 8; q++) {
#pragma unroll
      for (int j = 0; j < 6; j++) d[j][q] = 0.0;
      double f = 0.0;
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const double xs = ldexp(v[c][q], sh) + f;
        double r = rint(xs);
        f = xs - r;
        constexpr double up[6] = {1.0, 0x1p36, 0x1p72, 0x1p108, 0x1p144, 0x1p180};
        constexpr double dn[6] = {1.0, 0x1p-36, 0x1p-72, 0x1p-108, 0x1p-144, 0x1p-180};
#pragma unroll
        for (int j = 5; j >= 1; j--) {
          const double cj = trunc(r * dn[j]);
          r = __builtin_fma(-cj, up[j], r);
          d[j][q] += cj;
        }
        d[0][q] += r;
      }
      // balance the low limbs (|d_j| <= 2^35, j < 3), so |L| <= 2^107 (1 + 2^-35)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        const double cy = rint(d[j][q] * 0x1p-36);
        d[j][q] = __builtin_fma(-cy, 0x1p36, d[j][q]);
        d[j + 1][q] += cy;
      }
    }
  }
  // fragment slot of (line, k0): K block, half and byte offset
  const int64_t kb = kc * 2 + g / 4;
  const int half = (g % 4) / 2, off = 8 * (g % 2);
  signed char* dst = side == 0 ? Ares : Bres;
  const int64_t lines = side == 0 ? RB : CB;
  const int64_t slot = (ln + 32 * half) * 16 + off;
  for (int s = 0; s < cr.N; s++) {
    const double mm = cr.m[s], iv = cr.inv[s], t1 = cr.t36[s], t2 = cr.t72[s];
    const int64_t line0 = ((b * cr.N + s) * lines + lb) * KB;
#pragma unroll
    for (int part3 = 0; part3 < NLB / 3; part3++) {  // DD: A'; QD: L, then H
      uint32_t w[2] = {0u, 0u};
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const double xr = __builtin_fma(d[3 * part3 + 2][q], t2,
                                        __builtin_fma(d[3 * part3 + 1][q], t1,
                                                      d[3 * part3][q]));  // exact
        const double r = __builtin_fma(-rint(xr * iv), mm, xr);  // |r| <= m / 2
        w[q / 4] |= ((uint32_t)(int)r & 0xFFu) << (8 * (q % 4));
      }
      // DD: block kb; QD: L to 2 kb + 1 (A) or 2 kb (B), H to the other
      const int64_t sb = P == 2 ? kb : 2 * kb + ((part3 == 0) == (side == 0) ? 1 : 0);
      *(uint2*)(dst + (line0 + sb) * kOzFrag + slot) = make_uint2(w[0], w[1]);
    }
  }
}

// ---- products ---------------------------------------------------------------
// Workgroup = one tile of C (TB x TB blocks of 32) for one modulus and batch
// entry; 4 waves (2 x 2), each WB x WB blocks (WB = TB / 2; 16 WB^2
// accumulator registers).  K advances G blocks a step (one barrier a step).
// Fragments move global -> LDS by direct loads into a ring of ST steps' G
// blocks (each wave loads WB of a block's 2 TB fragments): once every wave
// holds step x's fragments in registers, its slot takes step x + ST; near the
// end the last block is loaded again into slots no one reads, so every wait
// is the same.  A wave reads step x + 1's fragments from LDS while step x's
// MFMAs run.
template <int TB, int ST, int G, int KST>
__global__ __launch_bounds__(256) void crt_gemm_kernel(CrtProd a) {
  constexpr int WB = TB / 2;
  __shared__ v4i lds[ST][G][2 * TB][64];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wr = w / 2, wc = w % 2;
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const int64_t per = a.tiles_m * a.tiles_n;
  const int64_t t = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x);
  const int64_t bs = t / per;  // batch entry and modulus
  const int s = (int)(bs % a.N);
  const int64_t b = bs / a.N;
  int64_t tm, tn;
  banded_tile(t % per, a.tiles_m, a.tiles_n, 2, tm, tn);

  // wave w stages fragments w, w + 4, ... of the 2 TB (A row blocks, then B
  // column blocks) of each K block
  const signed char* src[WB];
#pragma unroll
  for (int f = 0; f < WB; f++) {
    const int x = wu + 4 * f;
    src[f] = x < TB ? a.Ares + (((b * a.NS + s) * a.RB + TB * tm + x) * a.KB + a.koa) * kOzFrag +
                          lane * 16
                    : a.Bres +
                          (((b * a.NS + s) * a.CB + TB * tn + (x - TB)) * a.KB + a.kob) * kOzFrag +
                          lane * 16;
  }
  constexpr int64_t kstep = KST * kOzFrag;  // bytes between logical K blocks (a.kst)
  const int64_t kb0 = a.kb0, kb1 = a.kb1;
  const int64_t steps = (kb1 - kb0) / G;
  auto stage = [&](int64_t x) {  // the G blocks of step x
    const int st = (int)(x % ST);
#pragma unroll
    for (int gg = 0; gg < G; gg++) {
      const int64_t kb = kb0 + x * G + gg;
      const int64_t kr = kb < kb1 ? kb : kb1 - 1;  // past the end: the last block again
#pragma unroll
      for (int f = 0; f < WB; f++)
        __builtin_amdgcn_global_load_lds(
            (const void*)(src[f] + kr * kstep),
            (__attribute__((address_space(3))) void*)&lds[st][gg][wu + 4 * f][0], 16, 0, 0);
    }
  };
  auto frags = [&](int64_t x, v4i (&fa)[G][WB], v4i (&fb)[G][WB]) {
    const int st = (int)(x % ST);
#pragma unroll
    for (int gg = 0; gg < G; gg++) {
#pragma unroll
      for (int i = 0; i < WB; i++) fa[gg][i] = lds[st][gg][WB * wr + i][lane];
#pragma unroll
      for (int j = 0; j < WB; j++) fb[gg][j] = lds[st][gg][TB + WB * wc + j][lane];
    }
  };
  // s_waitcnt with vmcnt = WB G (ST - 2) (the loads of the ST - 2 steps after
  // the next one may stay in flight) and lgkmcnt = 0; gfx9 encoding: vmcnt in
  // bits 3:0 and 15:14, expcnt 6:4 (7: no wait), lgkmcnt 11:8
  constexpr int kV = WB * G * (ST - 2);
  static_assert(kV < 64, "vmcnt has six bits");
  constexpr int kWait = (kV & 15) | ((kV >> 4) << 14) | 0x70;
  auto sync = [&]() {
    __builtin_amdgcn_sched_barrier(0);  // the previous step's MFMAs stay before the wait
    __builtin_amdgcn_s_waitcnt(kWait);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();  // (no fence: it would wait for every load in flight)
    asm volatile("" ::: "memory");
  };

  v16i acc[WB][WB];
#pragma unroll
  for (int i = 0; i < WB; i++)
#pragma unroll
    for (int j = 0; j < WB; j++)
#pragma unroll
      for (int q = 0; q < 16; q++) acc[i][j][q] = 0;
#pragma unroll
  for (int d = 0; d < ST; d++) stage(d);  // the whole ring
  // two register sets of fragments, taken in turn (the loop runs two steps a
  // pass, the step count being even, so each set is named statically)
  v4i fa0[G][WB], fb0[G][WB], fa1[G][WB], fb1[G][WB];
  // one step: step x + 1 landed for every wave and every wave's reads of
  // step x are done (lgkmcnt 0), so step x's slot may be refilled
  auto step = [&](int64_t x, v4i (&ua)[G][WB], v4i (&ub)[G][WB], v4i (&na)[G][WB],
                  v4i (&nb)[G][WB]) {
    sync();
    stage(x + ST);  // into the slot of step x (== x + ST modulo ST)
    if (x + 1 < steps) frags(x + 1, na, nb);
#pragma unroll
    for (int gg = 0; gg < G; gg++)
#pragma unroll
      for (int i = 0; i < WB; i++)
#pragma unroll
        for (int j = 0; j < WB; j++)
          acc[i][j] =
              __builtin_amdgcn_mfma_i32_32x32x32_i8(ua[gg][i], ub[gg][j], acc[i][j], 0, 0, 0);
  };
  // steps 0 and 1 in LDS (the ST - 2 later ones may be in flight), step 0
  // in registers
  sync();
  frags(0, fa0, fb0);
  for (int64_t x = 0; x < steps; x += 2) {
    step(x, fa0, fb0, fa1, fb1);
    step(x + 1, fa1, fb1, fa0, fb0);
  }
  // residues of C_s: per block, quarter h of every lane's 16 outputs (the
  // MFMA output order, q = 4 h .. 4 h + 3) at bytes 256 h + 4 lane
  const double mm = a.m[s], iv = a.inv[s];
#pragma unroll
  for (int i = 0; i < WB; i++)
#pragma unroll
    for (int j = 0; j < WB; j++) {
      uint32_t wd[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int q = 0; q < 16; q++) {
        const double c = (double)acc[i][j][q];
        const double r = __builtin_fma(-rint(c * iv), mm, c);  // |r| <= m / 2
        wd[q / 4] |= ((uint32_t)(int)r & 0xFFu) << (8 * (q % 4));
      }
      const int64_t rb = TB * tm + WB * wr + i, cb = TB * tn + WB * wc + j;
      const int64_t blk = ((b * a.N + s) * a.RB + rb) * a.CB + cb;
#pragma unroll
      for (int h = 0; h < 4; h++) *(uint32_t*)(a.Cres + blk * kOzFrag + 256 * h + 4 * lane) = wd[h];
    }
}

// ---- rebuild ----------------------------------------------------------------
// 4 x 4 byte transpose: y[q] byte j = x[j] byte q.
__device__ __forceinline__ void transpose4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                           uint32_t (&y)[4]) {
  const uint32_t a = __builtin_amdgcn_perm(x1, x0, 0x05010400u);  // x0.0 x1.0 x0.1 x1.1
  const uint32_t b = __builtin_amdgcn_perm(x1, x0, 0x07030602u);  // x0.2 x1.2 x0.3 x1.3
  const uint32_t c = __builtin_amdgcn_perm(x3, x2, 0x05010400u);
  const uint32_t d = __builtin_amdgcn_perm(x3, x2, 0x07030602u);
  y[0] = __builtin_amdgcn_perm(c, a, 0x05040100u);
  y[1] = __builtin_amdgcn_perm(c, a, 0x07060302u);
  y[2] = __builtin_amdgcn_perm(d, b, 0x05040100u);
  y[3] = __builtin_amdgcn_perm(d, b, 0x07060302u);
}

// A wave's residues of one product as MFMA B operands, half u of its rows:
// op[q] holds, for the output in row 8 h + 4 u + q and column L % 32 of the
// block, its residues of moduli 16 (L / 32) + 0..15 (lane L; zero past N),
// the layout of the B operand (column L % 32, k = 16 (L / 32) + 0..15) of
// v_mfma_i32_32x32x32_i8 with the outputs of one row as columns.  Modulus
// s's residues of the quarter sit at src + s stride: lane l's four outputs
// (rows 8 h + 4 (l / 32) + 0..3, column l % 32) at bytes 4 l; lane L reads
// those of lane L % 32 + 32 u (32-bit loads, each lane half's covering 128
// contiguous bytes), then a 4 x 4 byte transpose per four moduli.
__device__ __forceinline__ void crt_residue_operands(const signed char* src, int64_t stride,
                                                     int N, int u, v4i (&op)[4]) {
  const int lane = threadIdx.x % 64, s0 = 16 * (lane / 32);
  const signed char* p = src + 4 * (lane % 32 + 32 * u);
  uint32_t w[16];
#pragma unroll
  for (int j = 0; j < 16; j++)
    w[j] = s0 + j < N ? *(const uint32_t*)(p + (int64_t)(s0 + j) * stride) : 0u;
#pragma unroll
  for (int g = 0; g < 4; g++) {
    uint32_t y[4];
    transpose4(w[4 * g], w[4 * g + 1], w[4 * g + 2], w[4 * g + 3], y);
#pragma unroll
    for (int q = 0; q < 4; q++) op[q][g] = (int)y[q];
  }
}

// Two MFMA results (outputs of rows t and t + 1 as columns, digits as rows:
// lane L, register r holds digit 8 (r / 4) + 4 (L / 32) + r % 4 of column
// L % 32) traded between the lane halves so that lane L holds every digit of
// one output (lanes 0-31: row t, lanes 32-63: row t + 1): digit d is then
// da[4 (d / 8) + d % 4] for (d / 4) even, db[...] for (d / 4) odd.
__device__ __forceinline__ void crt_gather_digits(v16i& da, v16i& db) {
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const auto x = __builtin_amdgcn_permlane32_swap(da[r], db[r], false, false);
    da[r] = (int)x[0];
    db[r] = (int)x[1];
  }
}
__device__ __forceinline__ int crt_digit(const v16i& da, const v16i& db, int d) {
  return ((d / 4) % 2 == 0 ? da : db)[4 * (d / 8) + d % 4];
}

// Workgroup = one 32 x 32 block of C; wave 2 h + u takes its rows 8 h + 4 u
// .. 8 h + 4 u + 3 (the residues' quarter h, half u).  The sums G_d =
// sum_s c_s Zd_s,d (Zd: Z's 7-bit digits, |G_d| < 2^19) run on the matrix
// cores, one MFMA per 32 outputs; lane L then carries the digits of its
// outputs (rows 8 h + 2 p + L / 32, column L % 32, p = 2 u, 2 u + 1) into
// the 160-bit fraction F (mod 2^160, signed), and X = F M 2^-160 in DD.
__global__ __launch_bounds__(512) void crt_rebuild_kernel(Mat C, int64_t m, int64_t n,
                                                          int64_t RB, int64_t CB,
                                                          const signed char* Cres,
                                                          const int* ea, const int* fb,
                                                          int alpha, int beta, CrtRebuild cb_,
                                                          int64_t blocks) {
  // 8 waves: wave 2 h + u takes rows 8 h + 4 u .. 8 h + 4 u + 3
  const int h = threadIdx.x / 128, u = (threadIdx.x / 64) % 2, lane = threadIdx.x % 64;
  const int64_t blk = blockIdx.x;
  if (blk >= blocks) return;
  const int64_t per = RB * CB;
  const int64_t b = blk / per, rb = (blk % per) / CB, cbk = blk % CB;
  const signed char* src = Cres + ((b * cb_.N) * per + rb * CB + cbk) * kOzFrag + 256 * h;
  v4i za;
#pragma unroll
  for (int g = 0; g < 4; g++) za[g] = (int)cb_.zd[lane][g];
  const int64_t col = cbk * 32 + lane % 32;
  const bool live = col < n;
  const int fexp = live ? fb[b * CB * 32 + col] : 0;
  double* Cb = C.p + b * C.bstride;
  const v16i zero = {};
  v4i op[4];
  crt_residue_operands(src, per * kOzFrag, cb_.N, u, op);
#pragma unroll
  for (int pp = 0; pp < 2; pp++) {
    const int p = 2 * u + pp;
    v16i da = __builtin_amdgcn_mfma_i32_32x32x32_i8(za, op[2 * pp], zero, 0, 0, 0);
    v16i db = __builtin_amdgcn_mfma_i32_32x32x32_i8(za, op[2 * pp + 1], zero, 0, 0, 0);
    crt_gather_digits(da, db);
    const int64_t row = rb * 32 + 8 * h + 2 * p + lane / 32;
    if (!live || row >= m) continue;
    // carries: 7-bit digits, bits from 160 up dropped (the sum mod 2^160)
    uint32_t wd[5] = {0u, 0u, 0u, 0u, 0u};
    int carry = 0;
#pragma unroll
    for (int d = 0; d < kDigits; d++) {
      const int x = crt_digit(da, db, d) + carry;
      const uint32_t dig = (uint32_t)x & ((1u << kDigitBits) - 1u);
      carry = x >> kDigitBits;  // arithmetic
      const int bit = kDigitBits * d, w = bit / 32, o = bit % 32;
      if (w < 5) wd[w] |= dig << o;
      if (o > 32 - kDigitBits && w + 1 < 5) wd[w + 1] |= dig >> (32 - o);
    }
    // the signed fraction F (units of 2^-160) from five 32-bit words, as a DD
    double hi = ldexp((double)(int32_t)wd[4], 128), lo = 0.0;
#pragma unroll
    for (int j = 3; j >= 0; j--) {
      double e;
      two_sum(hi, ldexp((double)wd[j], 32 * j), hi, e);
      lo += e;
    }
    fast_two_sum(hi, lo, hi, lo);
    dd_t x = dd_mul(dd_t{hi, lo}, dd_t{cb_.mhi, cb_.mlo});  // X = F M 2^-160
    const int sc = ea[b * RB * 32 + row] + fexp - 2 * kP1;
    x.hi = ldexp(x.hi, sc);
    x.lo = ldexp(x.lo, sc);
    if (alpha < 0) x = dd_neg(x);
    const int64_t off = row * C.ld + col;
    if (beta) x = dd_add(dd_t{Cb[off], Cb[C.ps + off]}, x);
    Cb[off] = x.hi;
    Cb[C.ps + off] = x.lo;
  }
}

// QD rebuild.  Workgroup and waves as in crt_rebuild_kernel; per pair of
// rows three MFMA sums each: the cross product's digits against zx, and
// H_a H_b's against zh0 and zh1.  Lane L's outputs: F_x (mod 2^162) made
// signed by the carry-out and sign bit of its own carry pass (F_x 2^-108
// sits on the low 27 digits of the 270-bit frame, 2^162 on digit 27), its
// digit sums and H_a H_b's carried together mod 2^270; the magnitude (two's
// complement when the sign bit is set) cut at its leading one into four
// 53-bit pieces, a QD; C = M 2^-256 F 2^(e + f + 42).
// (eight waves a workgroup, one half of a quarter's rows each: 143
// registers, three waves a SIMD)
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3))) void
crt_rebuild_qd_kernel(Mat C, int64_t m, int64_t n, int64_t RB, int64_t CB, const signed char* Chh,
                      const signed char* Cx, const int* ea, const int* fb, int alpha, int beta,
                      CrtRebuildQ k, int64_t blocks) {
  // 8 waves: wave 2 h + u takes rows 8 h + 4 u .. 8 h + 4 u + 3
  const int h = threadIdx.x / 128, u = (threadIdx.x / 64) % 2, lane = threadIdx.x % 64;
  const int64_t blk = blockIdx.x;
  if (blk >= blocks) return;
  const int64_t per = RB * CB;
  const int64_t b = blk / per, rb = (blk % per) / CB, cbk = blk % CB;
  const int64_t off0 = ((b * k.N) * per + rb * CB + cbk) * kOzFrag + 256 * h;
  v4i zx, zh0, zh1;
#pragma unroll
  for (int g = 0; g < 4; g++) {
    zx[g] = (int)k.zx[lane][g];
    zh0[g] = (int)k.zh0[lane][g];
    zh1[g] = (int)k.zh1[lane][g];
  }
  const int64_t col = cbk * 32 + lane % 32;
  const bool live = col < n;
  const int fexp = live ? fb[b * CB * 32 + col] : 0;
  double* Cb = C.p + b * C.bstride;
  const qd_t mq{{k.mq[0], k.mq[1], k.mq[2], k.mq[3]}};
  const v16i zero = {};
  v4i ox[4], oh[4];
  crt_residue_operands(Cx + off0, per * kOzFrag, k.N, u, ox);
  crt_residue_operands(Chh + off0, per * kOzFrag, k.N, u, oh);
#pragma unroll
  for (int pp = 0; pp < 2; pp++) {
    const int p = 2 * u + pp, t = 2 * pp;
    // F_x = sum_d Gx_d 2^(6 d) (mod 2^162) taken signed: the raw sum less
    // (q_x + s_x) 2^162, q_x its carry out of 27 digits and s_x the sign bit
    // of what remains; in the 270-bit frame F_x 2^-108 sits on digits 0..26
    // and 2^162 is digit 27
    v16i xa = __builtin_amdgcn_mfma_i32_32x32x32_i8(zx, ox[t], zero, 0, 0, 0);
    v16i xb = __builtin_amdgcn_mfma_i32_32x32x32_i8(zx, ox[t + 1], zero, 0, 0, 0);
    crt_gather_digits(xa, xb);
    int fix;
    {
      int carry = 0, top = 0;
#pragma unroll
      for (int d = 0; d < kDigitsX; d++) {
        top = crt_digit(xa, xb, d) + carry;
        carry = top >> 6;
      }
      fix = -(carry + ((top >> 5) & 1));
    }
    // the frame: H_a H_b's digit sums plus F_x's (and the fix), carried
    // mod 2^270 into 36-bit pieces (six digits; the last three)
    constexpr int NP = (kDigitsQ + 5) / 6;
    uint64_t pc[NP];
#pragma unroll
    for (int q = 0; q < NP; q++) pc[q] = 0u;
    int carry = 0;
    auto put = [&](int d, int x) {
      x += carry;
      carry = x >> 6;
      pc[d / 6] |= (uint64_t)(x & 63) << (6 * (d % 6));
    };
    __builtin_amdgcn_sched_barrier(0);
    {
      v16i ha = __builtin_amdgcn_mfma_i32_32x32x32_i8(zh0, oh[t], zero, 0, 0, 0);
      v16i hb = __builtin_amdgcn_mfma_i32_32x32x32_i8(zh0, oh[t + 1], zero, 0, 0, 0);
      crt_gather_digits(ha, hb);
#pragma unroll
      for (int d = 0; d < 32; d++)
        put(d, crt_digit(ha, hb, d) + (d < kDigitsX ? crt_digit(xa, xb, d) : 0) +
                   (d == kDigitsX ? fix : 0));
    }
    __builtin_amdgcn_sched_barrier(0);
    {
      v16i ga = __builtin_amdgcn_mfma_i32_32x32x32_i8(zh1, oh[t], zero, 0, 0, 0);
      v16i gb = __builtin_amdgcn_mfma_i32_32x32x32_i8(zh1, oh[t + 1], zero, 0, 0, 0);
      crt_gather_digits(ga, gb);
#pragma unroll
      for (int d = 32; d < kDigitsQ; d++) put(d, crt_digit(ga, gb, d - 32));
    }
    const int64_t row = rb * 32 + 8 * h + 2 * p + lane / 32;
    if (!live || row >= m) continue;
    // a negative F as its magnitude (two's complement over the pieces)
    constexpr int topbits = 6 * (kDigitsQ - 6 * (NP - 1));
    const bool neg = ((pc[NP - 1] >> (topbits - 1)) & 1u) != 0;
    if (neg) {
      uint64_t cy = 1u;
#pragma unroll
      for (int q = 0; q < NP; q++) {
        const uint64_t mask = q < NP - 1 ? (1ull << 36) - 1 : (1ull << topbits) - 1;
        const uint64_t x = (mask - pc[q]) + cy;
        pc[q] = x & mask;
        cy = x >> (q < NP - 1 ? 36 : topbits);
      }
    }
    // the magnitude's leading 212 bits as four 53-bit pieces: the 270 bits in
    // 64-bit words, moved up until the leading one is bit 63 of the top word,
    // then cut (the truncation is below 2^-211 of F); the pieces do not
    // overlap, each below an ulp of the one before
    uint64_t W[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < NP; q++) {
      const int bit = 36 * q, w = bit / 64, o = bit % 64;
      W[w] |= pc[q] << o;
      if (o + 36 > 64 && w + 1 < 5) W[w + 1] |= pc[q] >> (64 - o);
    }
    int e = 320;  // the top word's bit 63 is bit e - 1 of the integer
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const bool z = W[4] == 0u;
      W[4] = z ? W[3] : W[4];
      W[3] = z ? W[2] : W[3];
      W[2] = z ? W[1] : W[2];
      W[1] = z ? W[0] : W[1];
      W[0] = z ? 0u : W[0];
      e -= z ? 64 : 0;
    }
    qd_t f{{0.0, 0.0, 0.0, 0.0}};
    if (W[4] != 0u) {
      const int lz = __builtin_clzll(W[4]);
      if (lz) {
        W[4] = (W[4] << lz) | (W[3] >> (64 - lz));
        W[3] = (W[3] << lz) | (W[2] >> (64 - lz));
        W[2] = (W[2] << lz) | (W[1] >> (64 - lz));
        W[1] = (W[1] << lz) | (W[0] >> (64 - lz));
      }
      e -= lz;
      const uint64_t c0 = W[4] >> 11;
      const uint64_t c1 = ((W[4] & 0x7FFull) << 42) | (W[3] >> 22);
      const uint64_t c2 = ((W[3] & 0x3FFFFFull) << 31) | (W[2] >> 33);
      const uint64_t c3 = ((W[2] & 0x1FFFFFFFFull) << 20) | (W[1] >> 44);
      const int u0 = e - 53 - 6 * kDigitsQ;  // c0's unit (F in units of 2^-270)
      f.c[0] = ldexp((double)c0, u0);
      f.c[1] = ldexp((double)c1, u0 - 53);
      f.c[2] = ldexp((double)c2, u0 - 106);
      f.c[3] = ldexp((double)c3, u0 - 159);
    }
    if (neg) f = qd_neg(f);
    qd_t x = qd_mul(f, mq);
    const int sc = ea[b * RB * 32 + row] + fexp + 42;
#pragma unroll
    for (int c = 0; c < 4; c++) x.c[c] = ldexp(x.c[c], sc);
    if (alpha < 0) x = qd_neg(x);
    const int64_t off = row * C.ld + col;
    if (beta)
      x = qd_add(qd_t{{Cb[off], Cb[C.ps + off], Cb[2 * C.ps + off], Cb[3 * C.ps + off]}}, x);
#pragma unroll
    for (int c = 0; c < 4; c++) Cb[c * C.ps + off] = x.c[c];
  }
}

int run_crt(int P, const GemmBatch& g, char* ws, hipStream_t s, int tile) {
  const CrtLayout L = crt_layout(P, g.m, g.n, g.l, g.batch, crt_tile_blocks(g.m, g.n, tile));
  if (L.N == 0) return set_error(DDQD_E_UNSUPPORTED, "no modulus set covers K = %lld",
                                 (long long)g.l);
  const CrtWs w = crt_ws(ws, L);
  const OzLayout o = exp_layout(L);
  int rc = launch_oz_exponents(g, o, w.e, s);
  if (rc) return rc;
  const Consts& k = consts(L.N);
  // residues
  const int64_t chunks = (L.RB + L.CB) * (L.KBo / 2);
  if (chunks > INT32_MAX || g.batch > 65535)
    return set_error(DDQD_E_UNSUPPORTED, "residue grid too large");
  if (P == 4)
    launch_timed("crt_residue_kernel", crt_residue_kernel<4>,
                 dim3((unsigned)chunks, (unsigned)g.batch), dim3(256), 0, s, g.A, g.B, g.m, g.n,
                 g.l, L.RB, L.CB, L.KBo, L.KB, o.kb, (const int*)w.e.ea, (const int*)w.e.part,
                 w.e.fb, k.res, w.Ares, w.Bres);
  else
    launch_timed("crt_residue_kernel", crt_residue_kernel<2>,
                 dim3((unsigned)chunks, (unsigned)g.batch), dim3(256), 0, s, g.A, g.B, g.m, g.n,
                 g.l, L.RB, L.CB, L.KBo, L.KB, o.kb, (const int*)w.e.ea, (const int*)w.e.part,
                 w.e.fb, k.res, w.Ares, w.Bres);
  if ((rc = check_launch("crt_residue_kernel"))) return rc;
  // products and rebuild, K chunk by K chunk
  CrtProd p{};
  p.Ares = w.Ares;
  p.Bres = w.Bres;
  p.N = p.NS = L.N;
  for (int q = 0; q < L.N; q++) {
    p.m[q] = k.res.m[q];
    p.inv[q] = k.res.inv[q];
  }
  p.RB = L.RB;
  p.CB = L.CB;
  p.KB = L.KB;
  p.tiles_m = L.RB / L.TB;
  p.tiles_n = L.CB / L.TB;
  p.batch = g.batch;
  const int64_t nblk = p.tiles_m * p.tiles_n * L.N * g.batch;
  const int64_t blocks = L.RB * L.CB * g.batch;
  if (nblk > INT32_MAX || blocks > INT32_MAX)
    return set_error(DDQD_E_UNSUPPORTED, "grid too large");
  auto product = [&](signed char* out, int64_t kst, int64_t koa, int64_t kob, int64_t kb0,
                     int64_t kb1) {
    p.Cres = out;
    p.kst = kst;
    p.koa = koa;
    p.kob = kob;
    p.kb0 = kb0;
    p.kb1 = kb1;
    const dim3 grid((unsigned)nblk);
    if (L.TB == 8 && kst == 2)
      launch_timed("crt_gemm_kernel", crt_gemm_kernel<8, 5, 2, 2>, grid, dim3(256), 0, s, p);
    else if (L.TB == 8)
      launch_timed("crt_gemm_kernel", crt_gemm_kernel<8, 5, 2, 1>, grid, dim3(256), 0, s, p);
    else if (kst == 2)
      launch_timed("crt_gemm_kernel", crt_gemm_kernel<4, 4, 1, 2>, grid, dim3(256), 0, s, p);
    else
      launch_timed("crt_gemm_kernel", crt_gemm_kernel<4, 4, 1, 1>, grid, dim3(256), 0, s, p);
    return check_launch("crt_gemm_kernel");
  };
  // K blocks per chunk: all of them when l fits one chunk (the padding
  // blocks hold zeros), else the chunk's
  const int64_t kcb = g.l <= chunk_k(P) ? L.KBo : chunk_k(P) / 32;
  for (int64_t kb0 = 0; kb0 < L.KBo; kb0 += kcb) {
    const int64_t kb1 = kb0 + kcb < L.KBo ? kb0 + kcb : L.KBo;
    const int bt = kb0 == 0 ? g.beta : 1;
    if (P == 4) {
      // H_a H_b: A's even blocks by B's odd ones; the cross product: all
      if ((rc = product(w.Cres, 2, 0, 1, kb0, kb1))) return rc;
      if ((rc = product(w.Cx, 1, 0, 0, 2 * kb0, 2 * kb1))) return rc;
      launch_timed("crt_rebuild_qd_kernel", crt_rebuild_qd_kernel, dim3((unsigned)blocks),
                   dim3(512), 0, s, g.C, g.m, g.n, L.RB, L.CB, (const signed char*)w.Cres,
                   (const signed char*)w.Cx, (const int*)w.e.ea, (const int*)w.e.fb, g.alpha, bt,
                   k.rq, blocks);
      if ((rc = check_launch("crt_rebuild_qd_kernel"))) return rc;
    } else {
      if ((rc = product(w.Cres, 1, 0, 0, kb0, kb1))) return rc;
      launch_timed("crt_rebuild_kernel", crt_rebuild_kernel, dim3((unsigned)blocks), dim3(512),
                   0, s, g.C, g.m, g.n, L.RB, L.CB, (const signed char*)w.Cres,
                   (const int*)w.e.ea, (const int*)w.e.fb, g.alpha, bt, k.reb, blocks);
      if ((rc = check_launch("crt_rebuild_kernel"))) return rc;
    }
  }
  return DDQD_OK;
}

}  // namespace

// enough for either tile (the tuner tries both on one workspace)
size_t crt_workspace(int P, int64_t m, int64_t n, int64_t l, int64_t batch) {
  if ((P != 2 && P != 4) || m <= 0 || n <= 0 || l <= 0 || batch <= 0) return 0;
  const CrtLayout L4 = crt_layout(P, m, n, l, batch, 4), L8 = crt_layout(P, m, n, l, batch, 8);
  if (L4.N == 0) return 0;
  return std::max(crt_ws_bytes(L4), crt_ws_bytes(L8));
}

// tile: 0 (by shape), 128 or 256
int launch_crt(int P, const GemmBatch& g, void* ws, size_t ws_bytes, hipStream_t s, int tile) {
  if (P != 2 && P != 4) return set_error(DDQD_E_UNSUPPORTED, "the modular INT8 base is DD or QD");
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return DDQD_OK;
  if (g.l <= 0) return set_error(DDQD_E_ARG, "empty K reached the modular base");
  const size_t need = crt_workspace(P, g.m, g.n, g.l, g.batch);
  if (need == 0 || need > ws_bytes || !ws)
    return set_error(DDQD_E_WORKSPACE, "modular base: workspace of %zu bytes needed, %zu given",
                     need, ws_bytes);
  return run_crt(P, g, (char*)ws, s, tile);
}

}  // namespace ddqd

extern "C" int ddqd_crt_moduli(int precision, int64_t l, int* out, int cap) {
  using namespace ddqd;
  if ((precision != 2 && precision != 4) || l <= 0 || cap < 0 || (cap > 0 && !out)) return -1;
  const int64_t kc = l < chunk_k(precision) ? l : chunk_k(precision);
  const int N = moduli_for(precision, kc);
  for (int s = 0; s < N && s < cap; s++) out[s] = kModuli[s];
  return N;
}
