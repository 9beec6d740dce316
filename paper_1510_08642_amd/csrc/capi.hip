// C ABI of libddqd: argument validation, workspace planning and the
// breadth-first Strassen / Winograd driver (declarations in include/ddqd.h).
//
// Recursion plan.  Level j (1..L) of the recursion has 7^j subproblems, all of
// the same shape m_j x l_j x n_j with m_j = floor(m_{j-1}/2) (likewise l, n).
// Instead of recursing depth-first (the paper runs the seven products of a
// level as parallel OpenMP sections), the driver walks the tree breadth-first
// so every step is one launch over all subproblems of a level:
//   scaling    exponents for an exact power-of-two equilibration of A's rows
//              and B's columns, applied as the top level reads A and B and
//              undone as it writes C (sums then mix rows of equal scale),
//   pre-adds   level 1..L: one kernel per side writes the 7 operands of every
//              child into workspace (strided batches),
//   leaves     one batched launch computes all 7^L leaf products,
//   post-adds  level L..1: one kernel combines 7 products into each parent,
//              the top level applying C := beta*C + alpha*result,
//   peeling    where an order is not a multiple of 2^L and is cut down, the
//              few k beyond the core (a rank-r update of C), the last rows
//              and the last columns of C are products of their own: Simple
//              for the short K, the thin kernels (K spread over waves) for
//              the few rows and columns.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "ddqd.h"
#include "common.hpp"
#include "qd.hpp"

namespace ddqd {

int launch_dd_block(const GemmBatch& g, int tile, hipStream_t stream);
int launch_dd_simple(const GemmBatch& g, hipStream_t stream);
int64_t dd_block_tiles(int64_t m, int64_t n);
bool thin_shape(const GemmBatch& g);
int launch_thin(int P, const GemmBatch& g, hipStream_t stream);
// autotuning (tune.hip)
void auto_choice(int P, int64_t m, int64_t n, int64_t l, int base, int slices, int* algo,
                 int* levels, int* tile, int* band);
size_t auto_workspace(int P, int64_t m, int64_t n, int64_t l, int base, int slices);
int launch_dd_grouped(const GroupArgs& ga, int grid, hipStream_t stream);
int launch_qd_block(const GemmBatch& g, int tile, hipStream_t stream);
int launch_qd_simple(const GemmBatch& g, hipStream_t stream);
template <class N>
int launch_preadd(CMat src, Mat dst, int64_t rows, int64_t cols, int64_t src_rows,
                  int64_t src_cols, int64_t parents, int algo, int side, const int* expo,
                  hipStream_t stream);
template <class N>
int launch_postadd(CMat prod, Mat dst, int64_t rows, int64_t cols, int64_t dst_rows,
                   int64_t dst_cols, int64_t parents, int algo, int alpha, int beta,
                   const int* ea, const int* fb, hipStream_t stream);
int launch_exponents(CMat A, CMat B, int64_t m, int64_t n, int64_t l, int* ea, int* fb,
                     hipStream_t stream);
size_t ozaki_workspace(int P, int64_t m, int64_t n, int64_t l, int64_t batch, int slices);
int ozaki_default_slices(int P);
size_t ozaki_grouped_bytes(const GemmBatch& g, int S);
int launch_ozaki_grouped(const GemmBatch* probs, int count, int S, char* ws, size_t ws_bytes,
                         hipStream_t s);
int launch_ozaki(int P, const GemmBatch& g, int slices, void* ws, size_t ws_bytes,
                 hipStream_t stream, int band = 0);
bool ozaki_slices_ok(int P, int slices);
size_t crt_workspace(int P, int64_t m, int64_t n, int64_t l, int64_t batch);
int launch_crt(int P, const GemmBatch& g, void* ws, size_t ws_bytes, hipStream_t s, int tile);

static thread_local char g_msg[512];

int set_error(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  return status;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(DDQD_E_HIP, "%s: %s", what, hipGetErrorString(e));
  return DDQD_OK;
}

// ---- per-kernel timing ----------------------------------------------------
namespace {
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::atomic<int> g_prof{0};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof_recs;
thread_local hipEvent_t g_prof_pending = nullptr;
}  // namespace

void prof_begin(hipStream_t s) {
  if (!g_prof.load(std::memory_order_relaxed)) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  if (hipEventRecord(e, s) != hipSuccess) {
    (void)hipEventDestroy(e);
    return;
  }
  g_prof_pending = e;
}

ProfEvents prof_events(hipStream_t s) {
  ProfEvents e;
  if (!g_prof.load(std::memory_order_relaxed)) return e;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return e;
  if (hipEventCreate(&e.start) != hipSuccess) {
    e.start = nullptr;
    return e;
  }
  if (hipEventCreate(&e.stop) != hipSuccess) {
    (void)hipEventDestroy(e.start);
    e.start = e.stop = nullptr;
  }
  return e;
}

void prof_commit(const char* kernel, const ProfEvents& e) {
  if (!e.start) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_recs.push_back(ProfRec{kernel, e.start, e.stop});
}

void prof_record(const char* kernel, hipStream_t s) {
  if (!g_prof_pending) return;
  hipEvent_t e;
  if (hipEventCreate(&e) == hipSuccess && hipEventRecord(e, s) == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_recs.push_back(ProfRec{kernel, g_prof_pending, e});
  } else {
    (void)hipEventDestroy(g_prof_pending);
  }
  g_prof_pending = nullptr;
}

namespace {

constexpr int kMaxLevels = 6;

int64_t pow7(int j) {
  int64_t r = 1;
  while (j-- > 0) r *= 7;
  return r;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
  int P = 2, L = 0;
  // the recursion's square-split core: each dimension rounded to a multiple
  // of 2^L, down (the few leftover rows, columns or k peeled off as Block
  // products) or up (padded with zeros), whichever is nearer
  int64_t mc = 0, nc = 0, lc = 0;
  int64_t m[kMaxLevels + 1], n[kMaxLevels + 1], l[kMaxLevels + 1];
  size_t offA[kMaxLevels + 1], offB[kMaxLevels + 1], offM[kMaxLevels + 1];
  size_t off_exp = 0;  // int32 equilibration exponents: m for A's rows, n for B's columns
  size_t off_leaf = 0, leaf_bytes = 0, total = 0;
};

// Depth actually used: stop before any dimension of a level's parents drops
// below 2 (such a parent is a Block product in the paper's scheme too).
// Orders that 2^L does not divide (Sec. 3 uses n = 1023 and 1025) get a core
// that it does: a remainder r of at most 2^(L-1) is peeled (the last r rows,
// columns or k by Block products at the top level only), a larger one is
// padded with zeros up to the next multiple (the top level's pre-adds read
// the padding as zeros, its post-adds write only the caller's entries).
// Either way every level halves exactly and the leaves keep their size.
int64_t core_dim(int64_t d, int L) {
  const int64_t q = (int64_t)1 << L, r = d % q;
  if (r == 0) return d;
  if (2 * r <= q && d - r >= q) return d - r;
  return d + (q - r);
}

Plan make_plan(int P, int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
               int slices) {
  Plan pl;
  pl.P = P;
  pl.m[0] = m;
  pl.n[0] = n;
  pl.l[0] = l;
  int L = 0;
  if (algo == DDQD_STRASSEN || algo == DDQD_WINOGRAD) {
    int64_t mm = m, nn = n, ll = l;
    while (L < levels && mm >= 2 && nn >= 2 && ll >= 2) {
      mm /= 2;
      nn /= 2;
      ll /= 2;
      L++;
    }
    pl.mc = core_dim(m, L);
    pl.nc = core_dim(n, L);
    pl.lc = core_dim(l, L);
    for (int j = 1; j <= L; j++) {
      pl.m[j] = pl.mc >> j;
      pl.n[j] = pl.nc >> j;
      pl.l[j] = pl.lc >> j;
    }
  }
  pl.L = L;
  size_t off = 0;
  for (int j = 1; j <= L; j++) {
    int64_t cnt = pow7(j);
    pl.offA[j] = off;
    off = align_up(off + sizeof(double) * (size_t)(cnt * P * pl.m[j] * pl.l[j]));
    pl.offB[j] = off;
    off = align_up(off + sizeof(double) * (size_t)(cnt * P * pl.l[j] * pl.n[j]));
    pl.offM[j] = off;
    off = align_up(off + sizeof(double) * (size_t)(cnt * P * pl.m[j] * pl.n[j]));
  }
  if (L > 0) {
    pl.off_exp = off;
    off = align_up(off + sizeof(int) * (size_t)(m + n));
  }
  pl.off_leaf = off;
  if (base == DDQD_BASE_OZAKI_I8 && algo != DDQD_SIMPLE)
    pl.leaf_bytes = ozaki_workspace(P, pl.m[L], pl.n[L], pl.l[L], pow7(L), slices);
  if (base == DDQD_BASE_CRT_I8 && algo != DDQD_SIMPLE)
    pl.leaf_bytes = crt_workspace(P, pl.m[L], pl.n[L], pl.l[L], pow7(L));
  pl.total = off + pl.leaf_bytes;
  return pl;
}

// view helpers for level-j batches (tight leading dimensions)
CMat opA(const Plan& pl, char* ws, int j) {
  int64_t r = pl.m[j], c = pl.l[j];
  return CMat{(const double*)(ws + pl.offA[j]), c, r * c, pl.P * r * c};
}
CMat opB(const Plan& pl, char* ws, int j) {
  int64_t r = pl.l[j], c = pl.n[j];
  return CMat{(const double*)(ws + pl.offB[j]), c, r * c, pl.P * r * c};
}
Mat prodM(const Plan& pl, char* ws, int j) {
  int64_t r = pl.m[j], c = pl.n[j];
  return Mat{(double*)(ws + pl.offM[j]), c, r * c, pl.P * r * c};
}

// tile: the FMA Block tile (DD 64 or 32, QD 32 or 16; 0 = the larger);
// band: the Ozaki tile order's band of tile rows (0 = 4)
int leaf(int P, const GemmBatch& g, int base, int slices, int tile, int band, void* ws,
         size_t ws_bytes, hipStream_t s) {
  if (base == DDQD_BASE_OZAKI_I8) return launch_ozaki(P, g, slices, ws, ws_bytes, s, band);
  if (base == DDQD_BASE_CRT_I8) return launch_crt(P, g, ws, ws_bytes, s, tile);
  return P == 2 ? launch_dd_block(g, tile ? tile : 64, s) : launch_qd_block(g, tile, s);
}

int block_fma(int P, const GemmBatch& g, hipStream_t s) {
  return P == 2 ? launch_dd_block(g, 64, s) : launch_qd_block(g, 32, s);
}

// A part peeled off the recursion's core: Simple when K is a few columns
// (a rank-r update of a large C, r multiply-adds per entry), the thin kernels
// for a few rows or columns over a long K, Block otherwise.
int peel_product(int P, const GemmBatch& g, hipStream_t s) {
  if (g.l <= 16 && (g.m + 15) / 16 <= 65535)
    return P == 2 ? launch_dd_simple(g, s) : launch_qd_simple(g, s);
  if (thin_shape(g)) return launch_thin(P, g, s);
  return block_fma(P, g, s);
}

int preadd(int P, CMat src, Mat dst, int64_t rows, int64_t cols, int64_t src_rows,
           int64_t src_cols, int64_t parents, int algo, int side, const int* expo,
           hipStream_t s) {
  return P == 2 ? launch_preadd<DDNum>(src, dst, rows, cols, src_rows, src_cols, parents, algo,
                                       side, expo, s)
                : launch_preadd<QDNum>(src, dst, rows, cols, src_rows, src_cols, parents, algo,
                                       side, expo, s);
}

int postadd(int P, CMat prod, Mat dst, int64_t rows, int64_t cols, int64_t dst_rows,
            int64_t dst_cols, int64_t parents, int algo, int alpha, int beta, const int* ea,
            const int* fb, hipStream_t s) {
  return P == 2 ? launch_postadd<DDNum>(prod, dst, rows, cols, dst_rows, dst_cols, parents,
                                        algo, alpha, beta, ea, fb, s)
                : launch_postadd<QDNum>(prod, dst, rows, cols, dst_rows, dst_cols, parents,
                                        algo, alpha, beta, ea, fb, s);
}


CMat shift(CMat X, int64_t i, int64_t j) {
  X.p += i * X.ld + j;
  return X;
}
Mat shift(Mat X, int64_t i, int64_t j) {
  X.p += i * X.ld + j;
  return X;
}

int run_gemm(int P, const GemmBatch& top, int algo, int levels, int base, int slices, void* ws,
             size_t ws_bytes, hipStream_t s, int tile = 0, int band = 0) {
  if (algo == DDQD_SIMPLE) return P == 2 ? launch_dd_simple(top, s) : launch_qd_simple(top, s);
  Plan pl = make_plan(P, top.m, top.n, top.l, algo, levels, base, slices);
  char* w = (char*)ws;
  const int L = pl.L;
  if (L == 0) return leaf(P, top, base, slices, tile, band, w, ws_bytes, s);
  int rc;
  // equilibration exponents of A's rows and B's columns (top level only)
  int* ea = (int*)(w + pl.off_exp);
  int* fb = ea + top.m;
  if ((rc = launch_exponents(top.A, top.B, top.m, top.n, top.l, ea, fb, s))) return rc;
  // pre-adds, level by level
  for (int j = 1; j <= L; j++) {
    CMat srcA = j == 1 ? top.A : opA(pl, w, j - 1);
    CMat srcB = j == 1 ? top.B : opB(pl, w, j - 1);
    CMat dA = opA(pl, w, j), dB = opB(pl, w, j);
    Mat dstA{(double*)dA.p, dA.ld, dA.ps, dA.bstride};
    Mat dstB{(double*)dB.p, dB.ld, dB.ps, dB.bstride};
    const int* xa = j == 1 ? ea : nullptr;
    const int* xb = j == 1 ? fb : nullptr;
    // the top level reads the caller's matrices (padding reads as zeros,
    // peeled rows / columns / k are not read)
    const int64_t am = j == 1 ? std::min(top.m, pl.mc) : 2 * pl.m[j];
    const int64_t al = j == 1 ? std::min(top.l, pl.lc) : 2 * pl.l[j];
    const int64_t bl = al, bn = j == 1 ? std::min(top.n, pl.nc) : 2 * pl.n[j];
    if ((rc = preadd(P, srcA, dstA, pl.m[j], pl.l[j], am, al, pow7(j - 1), algo, 0, xa, s)))
      return rc;
    if ((rc = preadd(P, srcB, dstB, pl.l[j], pl.n[j], bl, bn, pow7(j - 1), algo, 1, xb, s)))
      return rc;
  }
  // all leaf products in one batched launch
  GemmBatch lf{pl.m[L], pl.n[L], pl.l[L], 1, 0, opA(pl, w, L), opB(pl, w, L), prodM(pl, w, L),
               pow7(L)};
  if ((rc = leaf(P, lf, base, slices, tile, band, w + pl.off_leaf, pl.leaf_bytes, s)))
    return rc;
  // post-adds, level by level back up (the root writes only the caller's C)
  const int64_t mr = std::min(top.m, pl.mc), nr = std::min(top.n, pl.nc);
  for (int j = L; j >= 1; j--) {
    const bool root = j == 1;
    Mat dst = root ? top.C : prodM(pl, w, j - 1);
    const int alpha = root ? top.alpha : 1, beta = root ? top.beta : 0;
    const int64_t dm = root ? mr : 2 * pl.m[j], dn = root ? nr : 2 * pl.n[j];
    if ((rc = postadd(P, cview(prodM(pl, w, j)), dst, pl.m[j], pl.n[j], dm, dn, pow7(j - 1),
                      algo, alpha, beta, root ? ea : nullptr, root ? fb : nullptr, s)))
      return rc;
  }
  // peeled parts: the core's missing k, then the last rows (all columns) and
  // the last columns (the core's rows)
  if (pl.lc < top.l) {
    GemmBatch g{mr, nr, top.l - pl.lc, top.alpha, 1, shift(top.A, 0, pl.lc),
                shift(top.B, pl.lc, 0), top.C, 1};
    if ((rc = peel_product(P, g, s))) return rc;
  }
  if (pl.mc < top.m) {
    GemmBatch g{top.m - pl.mc, top.n, top.l, top.alpha, top.beta, shift(top.A, pl.mc, 0),
                top.B, shift(top.C, pl.mc, 0), 1};
    if ((rc = peel_product(P, g, s))) return rc;
  }
  if (pl.nc < top.n) {
    GemmBatch g{mr, top.n - pl.nc, top.l, top.alpha, top.beta, top.A, shift(top.B, 0, pl.nc),
                shift(top.C, 0, pl.nc), 1};
    if ((rc = peel_product(P, g, s))) return rc;
  }
  return DDQD_OK;
}

bool overlaps(const double* a, int64_t a_len, const double* b, int64_t b_len) {
  if (!a || !b || a_len <= 0 || b_len <= 0) return false;
  return a < b + b_len && b < a + a_len;
}

int64_t extent(int P, int64_t rows, int64_t cols, int64_t ld, int64_t ps) {
  if (rows <= 0 || cols <= 0) return 0;
  return (P - 1) * ps + (rows - 1) * ld + cols;
}

int check_mat(const char* name, int P, const void* p, int64_t rows, int64_t cols, int64_t ld,
              int64_t ps) {
  if (rows <= 0 || cols <= 0) return DDQD_OK;
  if (!p) return set_error(DDQD_E_ARG, "%s is NULL", name);
  if ((uintptr_t)p % 8) return set_error(DDQD_E_ARG, "%s is not 8-byte aligned", name);
  if (ld < cols) return set_error(DDQD_E_ARG, "ld of %s (%lld) < columns (%lld)", name,
                                  (long long)ld, (long long)cols);
  if (P > 1 && ps < (rows - 1) * ld + cols)
    return set_error(DDQD_E_ARG, "plane stride of %s (%lld) lets planes overlap", name,
                     (long long)ps);
  return DDQD_OK;
}

int device_ok() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return set_error(DDQD_E_NODEVICE, "no HIP device available");
  }
  return DDQD_OK;
}

size_t gemm_ws(int P, int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
               int slices) {
  if (m < 0 || n < 0 || l < 0 || algo < 0 || algo > DDQD_AUTO || levels < 0 ||
      levels > kMaxLevels || base < 0 || base > 2 || slices < 0 || slices > 40 ||
      (base == DDQD_BASE_CRT_I8 && slices != 0))
    return SIZE_MAX;
  if (m == 0 || n == 0 || l == 0) return 0;
  if (algo == DDQD_AUTO) return auto_workspace(P, m, n, l, base, slices);
  return make_plan(P, m, n, l, algo, levels, base, slices).total;
}

}  // namespace

size_t plan_workspace(int P, int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
                      int slices) {
  return gemm_ws(P, m, n, l, algo, levels, base, slices);
}

// tile: Block FMA leaf tile (DD 64 or 32, QD 32 or 16; 0 = the larger);
// band: Ozaki tile order band (0 = 4); algo DDQD_AUTO takes the tuned or
// default configuration of this shape.
int gemm_entry(int P, int64_t m, int64_t n, int64_t l, int alpha, const double* A, int64_t lda,
               int64_t psa, const double* B, int64_t ldb, int64_t psb, int beta, double* C,
               int64_t ldc, int64_t psc, int algo, int levels, int base, int slices, void* ws,
               size_t ws_bytes, void* stream, int tile, int band) {
  g_msg[0] = 0;
  if (m < 0 || n < 0 || l < 0) return set_error(DDQD_E_ARG, "negative dimension");
  if (alpha != 1 && alpha != -1) return set_error(DDQD_E_ARG, "alpha must be +1 or -1");
  if (beta != 0 && beta != 1) return set_error(DDQD_E_ARG, "beta must be 0 or 1");
  if (algo < 0 || algo > DDQD_AUTO) return set_error(DDQD_E_ARG, "unknown algo %d", algo);
  if (base == DDQD_BASE_CRT_I8 ? (tile != 0 && tile != 128 && tile != 256)
                               : (tile != 0 && tile != 32 && tile != (P == 2 ? 64 : 16)))
    return set_error(DDQD_E_ARG, base == DDQD_BASE_CRT_I8 ? "CRT tile must be 128 or 256"
                                 : P == 2 ? "tile must be 32 or 64" : "tile must be 16 or 32");
  if (band < 0 || band > 64) return set_error(DDQD_E_ARG, "band must be in 0..64");
  if (levels < 0 || levels > kMaxLevels)
    return set_error(DDQD_E_ARG, "levels must be in 0..%d", kMaxLevels);
  if (base != DDQD_BASE_FMA && base != DDQD_BASE_OZAKI_I8 && base != DDQD_BASE_CRT_I8)
    return set_error(DDQD_E_ARG, "unknown base %d", base);
  if (slices < 0 || slices > 40) return set_error(DDQD_E_ARG, "slices must be in 0..40");
  if (base == DDQD_BASE_CRT_I8 && slices != 0)
    return set_error(DDQD_E_ARG, "the CRT base takes no slice count (0)");
  if (base == DDQD_BASE_OZAKI_I8 && !ozaki_slices_ok(P, slices))
    return set_error(DDQD_E_UNSUPPORTED, "%d slices not supported (DD 8..20, QD 28..31)",
                     slices);
  int rc;
  if ((rc = check_mat("C", P, C, m, n, ldc, psc))) return rc;
  if (l > 0) {
    if ((rc = check_mat("A", P, A, m, l, lda, psa))) return rc;
    if ((rc = check_mat("B", P, B, l, n, ldb, psb))) return rc;
  }
  if (m == 0 || n == 0) return DDQD_OK;
  const int64_t ec = extent(P, m, n, ldc, psc);
  if (l > 0 && (overlaps(C, ec, A, extent(P, m, l, lda, psa)) ||
                overlaps(C, ec, B, extent(P, l, n, ldb, psb))))
    return set_error(DDQD_E_ALIAS, "C overlaps A or B");
  size_t need = gemm_ws(P, m, n, l, algo, levels, base, slices);
  if (need > ws_bytes || (need > 0 && !ws))
    return set_error(DDQD_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                     ws_bytes);
  if (need > 0 && (uintptr_t)ws % 8) return set_error(DDQD_E_WORKSPACE, "workspace misaligned");
  if ((rc = device_ok())) return rc;
  if (algo == DDQD_AUTO) auto_choice(P, m, n, l, base, slices, &algo, &levels, &tile, &band);
  hipStream_t s = (hipStream_t)stream;
  GemmBatch top{m, n, l, alpha, beta, CMat{A, lda, psa, 0}, CMat{B, ldb, psb, 0},
                Mat{C, ldc, psc, 0}, 1};
  if (l == 0) {  // C := beta*C: the Block kernel with an empty K loop does exactly this
    top.A = CMat{C, ldc, psc, 0};
    top.B = CMat{C, ldc, psc, 0};
    return block_fma(P, top, s);
  }
  return run_gemm(P, top, algo, levels, base, slices, ws, ws_bytes, s, tile, band);
}

// Internal entry points for other drivers (LU): no validation, no alias checks.
int gemm_internal(int P, const GemmBatch& g, int algo, int levels, int base, int slices,
                  void* ws, size_t ws_bytes, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0) return DDQD_OK;
  if (g.l <= 0) {
    GemmBatch t = g;
    t.A = cview(g.C);
    t.B = cview(g.C);
    return block_fma(P, t, s);
  }
  return run_gemm(P, g, algo, levels, base, slices, ws, ws_bytes, s);
}

size_t gemm_internal_ws(int P, int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
                        int slices) {
  return gemm_ws(P, m, n, l, algo, levels, base, slices);
}

int check_device() { return device_ok(); }

int check_matrix(const char* name, int P, const void* p, int64_t rows, int64_t cols, int64_t ld,
                 int64_t ps) {
  return check_mat(name, P, p, rows, cols, ld, ps);
}

int64_t matrix_extent(int P, int64_t rows, int64_t cols, int64_t ld, int64_t ps) {
  return extent(P, rows, cols, ld, ps);
}

bool ranges_overlap(const void* a, int64_t a_len, const void* b, int64_t b_len) {
  return overlaps((const double*)a, a_len, (const double*)b, b_len);
}

void clear_error() { g_msg[0] = 0; }

}  // namespace ddqd

using namespace ddqd;

extern "C" {

const char* ddqd_status_string(int status) {
  switch (status) {
    case DDQD_OK: return "DDQD_OK";
    case DDQD_E_ARG: return "DDQD_E_ARG: invalid argument";
    case DDQD_E_ALIAS: return "DDQD_E_ALIAS: output overlaps an input";
    case DDQD_E_WORKSPACE: return "DDQD_E_WORKSPACE: workspace missing or too small";
    case DDQD_E_UNSUPPORTED: return "DDQD_E_UNSUPPORTED: combination not supported";
    case DDQD_E_NODEVICE: return "DDQD_E_NODEVICE: no usable GPU";
    case DDQD_E_HIP: return "DDQD_E_HIP: HIP call or launch failed";
    default: return "unknown status";
  }
}

const char* ddqd_last_error(void) { return g_msg; }

void ddqd_profile_enable(int on) { g_prof.store(on ? 1 : 0); }

void ddqd_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof_recs.clear();
}

int ddqd_profile_query(const char* substr, double* ms, int64_t* count) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : g_prof_recs) {
    if (substr && r.name.find(substr) == std::string::npos) continue;
    float t = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      return set_error(DDQD_E_HIP, "profile event query failed");
    tot += t;
    cnt++;
  }
  if (ms) *ms = tot;
  if (count) *count = cnt;
  return DDQD_OK;
}

}  // extern "C"

namespace ddqd {
namespace {

// Problems of a grouped call that run on Ozaki leaves (m, n, l > 0), and the
// workspace each needs: the grouped launches take l <= 16384 (one exact INT32
// accumulation), longer K runs as a product of its own.
constexpr int64_t kGroupedOzakiMaxL = 16384;

GemmBatch desc_batch(const ddqd_gemm_desc& x) {
  GemmBatch g{x.m, x.n, x.l, x.alpha, x.beta, CMat{x.A, x.lda, x.psa, 0},
              CMat{x.B, x.ldb, x.psb, 0}, Mat{x.C, x.ldc, x.psc, 0}, 1};
  if (x.l == 0) {  // C := beta C: the empty K loop reads nothing from A or B
    g.A = CMat{x.C, x.ldc, x.psc, 0};
    g.B = g.A;
  }
  return g;
}

bool desc_ozaki(const ddqd_gemm_desc& x) {
  return x.base == DDQD_BASE_OZAKI_I8 && x.m > 0 && x.n > 0 && x.l > 0;
}

int desc_slices(const ddqd_gemm_desc& x) {
  return x.slices == 0 ? ozaki_default_slices(2) : x.slices;
}

size_t desc_ozaki_bytes(const ddqd_gemm_desc& x) {
  const GemmBatch g = desc_batch(x);
  if (x.l <= kGroupedOzakiMaxL) return ozaki_grouped_bytes(g, desc_slices(x));
  return align_up(ozaki_workspace(2, x.m, x.n, x.l, 1, desc_slices(x)));
}

int check_descs(int count, const ddqd_gemm_desc* d) {
  if (count < 0) return set_error(DDQD_E_ARG, "negative count");
  if (count > 0 && !d) return set_error(DDQD_E_ARG, "descriptor array is NULL");
  int rc;
  for (int i = 0; i < count; i++) {
    const ddqd_gemm_desc& x = d[i];
    if (x.m < 0 || x.n < 0 || x.l < 0)
      return set_error(DDQD_E_ARG, "problem %d: negative dimension", i);
    if ((x.alpha != 1 && x.alpha != -1) || (x.beta != 0 && x.beta != 1))
      return set_error(DDQD_E_ARG, "problem %d: alpha must be +-1 and beta 0 or 1", i);
    if (x.base == DDQD_BASE_CRT_I8)
      return set_error(DDQD_E_UNSUPPORTED, "problem %d: grouped launches take the FMA or Ozaki base",
                       i);
    if (x.base != DDQD_BASE_FMA && x.base != DDQD_BASE_OZAKI_I8)
      return set_error(DDQD_E_ARG, "problem %d: unknown base %d", i, x.base);
    if (x.slices < 0 || x.slices > 40)
      return set_error(DDQD_E_ARG, "problem %d: slices must be in 0..40", i);
    if (x.base == DDQD_BASE_OZAKI_I8 && !ozaki_slices_ok(2, x.slices))
      return set_error(DDQD_E_UNSUPPORTED, "problem %d: %d slices not supported (DD 8..20)", i,
                       x.slices);
    if ((rc = check_mat("C", 2, x.C, x.m, x.n, x.ldc, x.psc))) return rc;
    if (x.l > 0 && x.m > 0 && x.n > 0) {
      if ((rc = check_mat("A", 2, x.A, x.m, x.l, x.lda, x.psa))) return rc;
      if ((rc = check_mat("B", 2, x.B, x.l, x.n, x.ldb, x.psb))) return rc;
    }
  }
  return DDQD_OK;
}

size_t grouped_ws(int count, const ddqd_gemm_desc* d) {
  size_t need = 0;
  for (int i = 0; i < count; i++)
    if (desc_ozaki(d[i])) need += desc_ozaki_bytes(d[i]);
  return need;
}

}  // namespace
}  // namespace ddqd

extern "C" {

size_t dd_gemm_grouped_workspace(int count, const ddqd_gemm_desc* d) {
  if (check_descs(count, d)) return SIZE_MAX;
  return grouped_ws(count, d);
}

int dd_gemm_grouped(int count, const ddqd_gemm_desc* d, void* ws, size_t ws_bytes,
                    void* stream) {
  g_msg[0] = 0;
  int rc;
  if ((rc = check_descs(count, d))) return rc;
  if (count == 0) return DDQD_OK;
  // no output may overlap any input or any other output of the group
  for (int i = 0; i < count; i++) {
    const ddqd_gemm_desc& x = d[i];
    const int64_t ec = extent(2, x.m, x.n, x.ldc, x.psc);
    for (int j = 0; j < count; j++) {
      const ddqd_gemm_desc& y = d[j];
      if (y.l > 0 && (overlaps(x.C, ec, y.A, extent(2, y.m, y.l, y.lda, y.psa)) ||
                      overlaps(x.C, ec, y.B, extent(2, y.l, y.n, y.ldb, y.psb))))
        return set_error(DDQD_E_ALIAS, "output of problem %d overlaps an input of problem %d", i,
                         j);
      if (j != i && overlaps(x.C, ec, y.C, extent(2, y.m, y.n, y.ldc, y.psc)))
        return set_error(DDQD_E_ALIAS, "outputs of problems %d and %d overlap", i, j);
    }
  }
  const size_t need = grouped_ws(count, d);
  if (need > ws_bytes || (need > 0 && !ws))
    return set_error(DDQD_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                     ws_bytes);
  if (need > 0 && (uintptr_t)ws % 8) return set_error(DDQD_E_WORKSPACE, "workspace misaligned");
  if ((rc = device_ok())) return rc;
  hipStream_t s = (hipStream_t)stream;
  // FMA problems (and every C := beta C): persistent Block launches of up to
  // kMaxGroup problems
  std::vector<GemmBatch> fma;
  for (int i = 0; i < count; i++)
    if (d[i].m > 0 && d[i].n > 0 && !desc_ozaki(d[i])) fma.push_back(desc_batch(d[i]));
  for (size_t c0 = 0; c0 < fma.size(); c0 += kMaxGroup) {
    GroupArgs ga;
    ga.count = 0;
    ga.start[0] = 0;
    for (size_t i = c0; i < fma.size() && i < c0 + kMaxGroup; i++) {
      ga.g[ga.count] = fma[i];
      ga.start[ga.count + 1] = ga.start[ga.count] + dd_block_tiles(fma[i].m, fma[i].n);
      ga.count++;
    }
    const int64_t tiles = ga.start[ga.count];
    const int grid = (int)(tiles < 512 ? tiles : 512);
    if ((rc = launch_dd_grouped(ga, grid, s))) return rc;
  }
  // Ozaki problems: grouped launches per slice count, each problem with its
  // own part of the workspace (laid out slice count by slice count, in the
  // order of the descriptors); longer K as products of their own
  char* w = (char*)ws;
  size_t off = 0;
  std::vector<int> done(count, 0);
  for (int i = 0; i < count; i++) {
    if (!desc_ozaki(d[i]) || done[i]) continue;
    const int S = desc_slices(d[i]);
    std::vector<GemmBatch> grp;
    const size_t off0 = off;
    for (int j = i; j < count; j++) {
      if (!desc_ozaki(d[j]) || done[j] || desc_slices(d[j]) != S ||
          d[j].l > kGroupedOzakiMaxL)
        continue;
      grp.push_back(desc_batch(d[j]));
      off += desc_ozaki_bytes(d[j]);
      done[j] = 1;
    }
    if (!grp.empty() &&
        (rc = launch_ozaki_grouped(grp.data(), (int)grp.size(), S, w + off0, off - off0, s)))
      return rc;
  }
  for (int i = 0; i < count; i++) {
    if (!desc_ozaki(d[i]) || done[i]) continue;
    const size_t b = desc_ozaki_bytes(d[i]);
    GemmBatch g = desc_batch(d[i]);
    if ((rc = launch_ozaki(2, g, d[i].slices, w + off, b, s))) return rc;
    off += b;
  }
  return DDQD_OK;
}

size_t dd_gemm_workspace(int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
                         int slices) {
  return gemm_ws(2, m, n, l, algo, levels, base, slices);
}

size_t qd_gemm_workspace(int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
                         int slices) {
  return gemm_ws(4, m, n, l, algo, levels, base, slices);
}

int dd_gemm(int64_t m, int64_t n, int64_t l, int alpha, const double* A, int64_t lda,
            int64_t psa, const double* B, int64_t ldb, int64_t psb, int beta, double* C,
            int64_t ldc, int64_t psc, int algo, int levels, int base, int slices, void* ws,
            size_t ws_bytes, void* stream) {
  return gemm_entry(2, m, n, l, alpha, A, lda, psa, B, ldb, psb, beta, C, ldc, psc, algo,
                    levels, base, slices, ws, ws_bytes, stream, 0, 0);
}

int qd_gemm(int64_t m, int64_t n, int64_t l, int alpha, const double* A, int64_t lda,
            int64_t psa, const double* B, int64_t ldb, int64_t psb, int beta, double* C,
            int64_t ldc, int64_t psc, int algo, int levels, int base, int slices, void* ws,
            size_t ws_bytes, void* stream) {
  return gemm_entry(4, m, n, l, alpha, A, lda, psa, B, ldb, psb, beta, C, ldc, psc, algo,
                    levels, base, slices, ws, ws_bytes, stream, 0, 0);
}

}  // extern "C"
