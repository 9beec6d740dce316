// Blocked right-looking LU (dd_getrf / qd_getrf) and the solve (dd_getrs /
// qd_getrs): host-side drivers over the kernels of lu.hip and the matrix
// product, the same for DD (P = 2 planes) and QD (P = 4).
//
// getrf follows the paper's Sec. 4: for each block column of width K,
//   step 2  factor the (n - j) x K panel, form U12 = L11^-1 A12 (and L21),
//   step 3  A22 := A22 - L21 U12 through the chosen product algorithm
//           (Simple / Block / Strassen / Winograd, FMA or Ozaki leaves),
// then continue on A22; the last block may be narrower than K.  With partial
// pivoting each panel column's interchange is applied to whole rows.
//
// The panel itself is factored recursively: halves of the panel are
// factored in turn, the right half updated with a triangular solve and a
// thin product in between; strips of at most 8 columns (fewer for tall or QD
// panels) are factored by one workgroup holding the strip in registers
// (getf2), and every strip's
// interchanges are applied to all other columns by laswp, which also keeps
// the row permutation in `perm`.  U12 = L11^-1 A12 is a recursive triangular
// solve (diagonal solves of up to 64 rows in DD, 32 in QD, one wave per
// column; products for the off-diagonal parts).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "ddqd.h"

namespace ddqd {

int gemm_internal(int P, const GemmBatch& g, int algo, int levels, int base, int slices,
                  void* ws, size_t ws_bytes, hipStream_t s);
size_t gemm_internal_ws(int P, int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
                        int slices);
int check_device();
int check_matrix(const char* name, int P, const void* p, int64_t rows, int64_t cols, int64_t ld,
                 int64_t ps);
int64_t matrix_extent(int P, int64_t rows, int64_t cols, int64_t ld, int64_t ps);
bool ranges_overlap(const void* a, int64_t a_len, const void* b, int64_t b_len);
void clear_error();

int launch_lu_init(int32_t* info, int32_t* perm, int64_t n, hipStream_t s);
int launch_rowwise_lu(int P, double* A, int64_t lda, int64_t ps, int64_t n, int32_t* ipiv,
                      int32_t* info, hipStream_t s);
int getf2_width(int P, int64_t m);
int trsm_max_rows(int P);
int launch_getf2(int P, double* A, int64_t lda, int64_t ps, int64_t r0, int64_t m, int64_t c0,
                 int w, int32_t* ipiv, int32_t* info, int pivot, hipStream_t s);
int launch_laswp(int P, double* A, int64_t lda, int64_t ps, int64_t n_cols, int64_t skip0,
                 int64_t skip1, int64_t k0, int64_t k1, const int32_t* ipiv, int32_t* perm,
                 hipStream_t s);
int launch_trsm_wave(int P, double* A, int64_t lda, int64_t ps, int64_t r0, int64_t c0, int nb,
                     int64_t x0, int64_t ncols, hipStream_t s);
int launch_lu_update(int P, const double* A, const double* B, double* C, int64_t ld, int64_t ps,
                     int64_t m, int64_t n, int64_t l, hipStream_t s);
int launch_trsm_update(int P, double* A, int64_t lda, int64_t ps, int64_t r0, int nb,
                       int64_t x0, int64_t ncols, int64_t mb, hipStream_t s);
int launch_trsm_nodes(int P, double* A, int64_t lda, int64_t ps, const TrsmNodes& nodes,
                      hipStream_t s);
int launch_perm_from_ipiv(const int32_t* ipiv, int64_t n, int32_t* perm, hipStream_t s);
int launch_gather_rows(int P, const double* B, int64_t ldb, int64_t psb, const int32_t* perm,
                       int64_t n, int64_t nrhs, double* X, int* flags, int nflags,
                       hipStream_t s);
int launch_scatter_rows(int P, const double* X, int64_t n, int64_t nrhs, double* B, int64_t ldb,
                        int64_t psb, hipStream_t s);
int launch_trsv_chain(int P, const double* T, int64_t ldt, int64_t pst, double* X, int64_t n,
                      int64_t nrhs, int upper, int* flags, hipStream_t s);

namespace {

constexpr int64_t kMaxLuRows = 8192;

// trailing-update bases: FMA, Ozaki and CRT, in DD and QD
bool lu_base_ok(int P, int base) {
  return (P == 2 || P == 4) &&
         (base == DDQD_BASE_FMA || base == DDQD_BASE_OZAKI_I8 || base == DDQD_BASE_CRT_I8);
}

struct Lu {
  int P;  // 2 = DD, 4 = QD
  double* A;
  int64_t lda, ps, n;
  int32_t* ipiv;
  int32_t* perm;
  int32_t* info;
  int pivot, algo, levels, base;
  void* ws;
  size_t ws_bytes;
  hipStream_t s;
};

Mat sub(const Lu& c, int64_t i, int64_t j) { return Mat{c.A + i * c.lda + j, c.lda, c.ps, 0}; }

// C -= A B inside the panel and the triangular solves (no workspace).  These
// products are thin (one side <= the panel width), so they rarely give the
// Block kernel one 64 x 64 tile per compute unit; below that a kernel with
// one thread per entry and no tile staging finishes sooner.
int block_update(const Lu& c, int64_t m, int64_t n, int64_t l, Mat Am, Mat Bm, Mat Cm) {
  const int64_t tiles = ((m + 63) / 64) * ((n + 63) / 64);
  if (tiles < 256) return launch_lu_update(c.P, Am.p, Bm.p, Cm.p, c.lda, c.ps, m, n, l, c.s);
  GemmBatch g{m, n, l, -1, 1, cview(Am), cview(Bm), Cm, 1};
  return gemm_internal(c.P, g, DDQD_BLOCK, 0, DDQD_BASE_FMA, 0, nullptr, 0, c.s);
}

// X := L^-1 X, L unit lower nb x nb at (r0, r0), X = rows [r0, r0+nb) of
// columns [x0, x0 + nc)
int trsm(const Lu& c, int64_t r0, int64_t nb, int64_t x0, int64_t nc) {
  if (nb <= 0 || nc <= 0) return 0;
  const int64_t R = trsm_max_rows(c.P);
  if (nb <= R) return launch_trsm_wave(c.P, c.A, c.lda, c.ps, r0, r0, (int)nb, x0, nc, c.s);
  const int64_t n1 = (nb / 2 + R - 1) / R * R;
  int rc;
  if ((rc = trsm(c, r0, n1, x0, nc))) return rc;
  if ((rc = block_update(c, nb - n1, nc, n1, sub(c, r0 + n1, r0), sub(c, r0, x0),
                         sub(c, r0 + n1, x0))))
    return rc;
  return trsm(c, r0 + n1, nb - n1, x0, nc);
}

// Stores the solves the fused steps of a panel left pending, and empties the list.
int flush_nodes(const Lu& c, TrsmNodes& nodes) {
  const int rc = launch_trsm_nodes(c.P, c.A, c.lda, c.ps, nodes, c.s);
  nodes.count = 0;
  return rc;
}

// factor columns [c0, c0 + w) of rows [c0, n).  A step whose solve is small
// and whose update is thin runs both in one launch (trsm_update_kernel) and
// leaves X to be stored from `nodes` when the whole panel is factored (DD
// only).  Every row block of that launch repeats the solve: for DD solves of
// up to one triangular block (64 rows) that costs less than the launch it
// saves (getrf n = 2048: 14.1 -> 13.4 ms, n = 4096: 45.5 -> 42.8 ms), for QD,
// whose multiply-add costs about ten DD ones, more, even at 8 rows (QD getrf
// n = 1024: 14.0 -> 14.8 ms).
int panel(const Lu& c, int64_t c0, int64_t w, TrsmNodes& nodes) {
  const int64_t m = c.n - c0;
  const int wb = getf2_width(c.P, m);
  int rc;
  if (w <= wb) {
    if ((rc = launch_getf2(c.P, c.A, c.lda, c.ps, c0, m, c0, (int)w, c.ipiv, c.info, c.pivot,
                           c.s)))
      return rc;
    return launch_laswp(c.P, c.A, c.lda, c.ps, c.n, c0, c0 + w, c0, c0 + w, c.ipiv, c.perm, c.s);
  }
  int64_t w1 = (w / 2) / wb * wb;
  if (w1 < wb) w1 = wb;
  if ((rc = panel(c, c0, w1, nodes))) return rc;
  const int64_t tiles = ((m - w1 + 63) / 64) * ((w - w1 + 63) / 64);
  if (c.P == 2 && w1 <= trsm_max_rows(c.P) && tiles < 256) {
    if (nodes.count == kTrsmNodesMax && (rc = flush_nodes(c, nodes))) return rc;
    if ((rc = launch_trsm_update(c.P, c.A, c.lda, c.ps, c0, (int)w1, c0 + w1, w - w1, m - w1,
                                 c.s)))
      return rc;
    const int q = nodes.count++;
    nodes.r0[q] = (int)c0;
    nodes.nb[q] = (int)w1;
    nodes.x0[q] = (int)(c0 + w1);
    nodes.nc[q] = (int)(w - w1);
  } else {
    if ((rc = trsm(c, c0, w1, c0 + w1, w - w1))) return rc;
    if ((rc = block_update(c, m - w1, w - w1, w1, sub(c, c0 + w1, c0), sub(c, c0, c0 + w1),
                           sub(c, c0 + w1, c0 + w1))))
      return rc;
  }
  return panel(c, c0 + w1, w - w1, nodes);
}

int getrf(const Lu& c, int64_t K) {
  int rc;
  if ((rc = launch_lu_init(c.info, c.perm, c.n, c.s))) return rc;
  for (int64_t j0 = 0; j0 < c.n; j0 += K) {
    const int64_t kb = c.n - j0 < K ? c.n - j0 : K;
    TrsmNodes nodes;
    nodes.count = 0;
    if ((rc = panel(c, j0, kb, nodes))) return rc;
    if ((rc = flush_nodes(c, nodes))) return rc;
    const int64_t r = c.n - j0 - kb;
    if (r <= 0) break;
    // step 2: U12 = L11^-1 A12
    if ((rc = trsm(c, j0, kb, j0 + kb, r))) return rc;
    // step 3: A22 := A22 - L21 U12
    GemmBatch g{r, r, kb, -1, 1, cview(sub(c, j0 + kb, j0)), cview(sub(c, j0, j0 + kb)),
                sub(c, j0 + kb, j0 + kb), 1};
    if ((rc = gemm_internal(c.P, g, c.algo, c.levels, c.base, 0, c.ws, c.ws_bytes, c.s)))
      return rc;
  }
  return 0;
}

size_t getrf_ws(int P, int64_t n, int64_t K, int algo, int levels, int base) {
  size_t mx = 0;
  for (int64_t j0 = 0; j0 < n; j0 += K) {
    const int64_t kb = n - j0 < K ? n - j0 : K, r = n - j0 - kb;
    if (r <= 0) break;
    size_t w = gemm_internal_ws(P, r, r, kb, algo, levels, base, 0);
    if (w == SIZE_MAX) return SIZE_MAX;
    if (w > mx) mx = w;
  }
  return mx;
}

// getrs workspace: the gathered right-hand sides (P x n x min(nrhs, 16)
// doubles), the triangular solves' block flags, the permutation (n int32) if
// only ipiv is given.
constexpr size_t getrs_x_bytes(int P, int64_t n, int64_t nrhs) {
  return (sizeof(double) * P * (size_t)(n * (nrhs < 16 ? nrhs : 16)) + 255) & ~(size_t)255;
}

constexpr size_t getrs_flag_bytes(int64_t n) {
  return (sizeof(int) * (size_t)trsv_flag_words(n) + 255) & ~(size_t)255;
}

constexpr size_t getrs_ws(int P, int64_t n, int64_t nrhs) {
  return getrs_x_bytes(P, n, nrhs) + getrs_flag_bytes(n) + sizeof(int32_t) * (size_t)n;
}

// ---- panel width per order (DDQD_PANEL_AUTO, ddqd_getrf_tune) -----------
// Sec. 4 factors with panel widths K = 32 alpha, alpha = 1..10, and Sec. 5
// leaves the block size open; the tuner times those widths (the ones not
// above n; n itself for orders below 32) and keeps the fastest per order,
// pivoting and trailing-update product.  Untuned orders use 128.
constexpr int kDefaultPanel = 128;

std::vector<int> panel_candidates(int64_t n) {
  std::vector<int> c;
  for (int a = 1; a <= 10; a++)
    if (32 * a <= n) c.push_back(32 * a);
  if (c.empty()) c.push_back((int)std::max<int64_t>(n, 1));
  return c;
}

struct PanelKey {
  int P;
  int64_t n;
  int pivot, algo, levels, base;
  bool operator<(const PanelKey& o) const {
    return std::tie(P, n, pivot, algo, levels, base) <
           std::tie(o.P, o.n, o.pivot, o.algo, o.levels, o.base);
  }
};
struct PanelChoice {
  int panel, candidates;
  double ms;
};
std::mutex g_panel_mu;
std::map<PanelKey, PanelChoice> g_panel_cache;

PanelChoice panel_choice(int P, int64_t n, int pivot, int algo, int levels, int base) {
  std::lock_guard<std::mutex> lk(g_panel_mu);
  auto it = g_panel_cache.find(PanelKey{P, n, pivot, algo, levels, base});
  if (it != g_panel_cache.end()) return it->second;
  return PanelChoice{kDefaultPanel, 0, 0.0};
}

// the product workspace of every width DDQD_PANEL_AUTO may resolve to
size_t auto_panel_ws(int P, int64_t n, int algo, int levels, int base) {
  size_t w = getrf_ws(P, n, kDefaultPanel, algo, levels, base);
  for (int K : panel_candidates(n)) {
    const size_t k = getrf_ws(P, n, K, algo, levels, base);
    if (k == SIZE_MAX || w == SIZE_MAX) return SIZE_MAX;
    w = std::max(w, k);
  }
  return w;
}

size_t getrf_workspace_entry(int P, int64_t n, int panel_width, int algo, int levels, int base) {
  if (n < 0 || panel_width < DDQD_PANEL_AUTO || algo < 0 || algo > 3 || levels < 0 ||
      levels > 6 || !lu_base_ok(P, base))
    return SIZE_MAX;
  if (panel_width == 0) return 0;  // the row-wise comparator needs none
  if (panel_width == DDQD_PANEL_AUTO) return auto_panel_ws(P, n, algo, levels, base);
  return getrf_ws(P, n, panel_width, algo, levels, base);
}

int getrf_entry(int P, int64_t n, double* A, int64_t lda, int64_t psa, int32_t* ipiv,
                int32_t* perm, int32_t* info, int panel_width, int pivot, int algo, int levels,
                int base, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (n < 0) return set_error(DDQD_E_ARG, "negative order");
  if (panel_width < DDQD_PANEL_AUTO)
    return set_error(DDQD_E_ARG, "panel width must be >= 0 or DDQD_PANEL_AUTO");
  if (pivot != DDQD_PIVOT_NONE && pivot != DDQD_PIVOT_PARTIAL)
    return set_error(DDQD_E_ARG, "pivot must be DDQD_PIVOT_NONE or DDQD_PIVOT_PARTIAL");
  if (panel_width == DDQD_PANEL_AUTO && algo >= 0 && algo <= 3 && levels >= 0 && levels <= 6 &&
      lu_base_ok(P, base))
    panel_width = panel_choice(P, n, pivot, algo, levels, base).panel;
  if (panel_width == 0 && pivot != DDQD_PIVOT_NONE)
    return set_error(DDQD_E_UNSUPPORTED, "the row-wise form (panel width 0) does not pivot");
  if (algo < 0 || algo > 3 || levels < 0 || levels > 6 || !lu_base_ok(P, base))
    return set_error(DDQD_E_ARG, "bad product algorithm / levels / base");
  if (!info) return set_error(DDQD_E_ARG, "info is NULL");
  if (n > 0 && !ipiv) return set_error(DDQD_E_ARG, "ipiv is NULL");
  if (n > kMaxLuRows)
    return set_error(DDQD_E_UNSUPPORTED, "LU of order above %lld", (long long)kMaxLuRows);
  int rc;
  if ((rc = check_matrix("A", P, A, n, n, lda, psa))) return rc;
  const size_t need = panel_width == 0 ? 0 : getrf_ws(P, n, panel_width, algo, levels, base);
  if (need == SIZE_MAX) return set_error(DDQD_E_ARG, "bad product arguments");
  if (need > ws_bytes || (need > 0 && !ws))
    return set_error(DDQD_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                     ws_bytes);
  if ((rc = check_device())) return rc;
  Lu c{P, A, lda, psa, n, ipiv, perm, info, pivot, algo, levels, base, ws, ws_bytes,
       (hipStream_t)stream};
  if (n == 0) return launch_lu_init(info, nullptr, 0, c.s);
  if (panel_width == 0) {
    if ((rc = launch_lu_init(info, perm, n, c.s))) return rc;
    return launch_rowwise_lu(P, A, lda, psa, n, ipiv, info, c.s);
  }
  return getrf(c, panel_width);
}

size_t getrs_workspace_entry(int P, int64_t n, int64_t nrhs) {
  if (n < 0 || nrhs < 0) return SIZE_MAX;
  if (n == 0 || nrhs == 0) return 0;
  return getrs_ws(P, n, nrhs);
}

int getrs_entry(int P, int64_t n, int64_t nrhs, const double* LU, int64_t ldlu, int64_t pslu,
                const int32_t* ipiv, const int32_t* perm, double* B, int64_t ldb, int64_t psb,
                void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (n < 0 || nrhs < 0) return set_error(DDQD_E_ARG, "negative dimension");
  if (n == 0 || nrhs == 0) return DDQD_OK;
  if (!ipiv && !perm) return set_error(DDQD_E_ARG, "ipiv and perm are both NULL");
  int rc;
  if ((rc = check_matrix("LU", P, LU, n, n, ldlu, pslu))) return rc;
  if ((rc = check_matrix("B", P, B, n, nrhs, ldb, psb))) return rc;
  if (ranges_overlap(LU, matrix_extent(P, n, n, ldlu, pslu), B,
                     matrix_extent(P, n, nrhs, ldb, psb)))
    return set_error(DDQD_E_ALIAS, "B overlaps LU");
  const size_t need = getrs_ws(P, n, nrhs);
  if (need > ws_bytes || !ws)
    return set_error(DDQD_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                     ws_bytes);
  if ((rc = check_device())) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t chunk = nrhs < 16 ? nrhs : 16;
  double* X = (double*)ws;
  int* flags = (int*)((char*)ws + getrs_x_bytes(P, n, nrhs));
  int32_t* pm = (int32_t*)((char*)flags + getrs_flag_bytes(n));
  if (!perm) {
    if ((rc = launch_perm_from_ipiv(ipiv, n, pm, s))) return rc;
    perm = pm;
  }
  for (int64_t c0 = 0; c0 < nrhs; c0 += chunk) {
    const int64_t nc = nrhs - c0 < chunk ? nrhs - c0 : chunk;
    if ((rc = launch_gather_rows(P, B + c0, ldb, psb, perm, n, nc, X, flags,
                                 (int)trsv_flag_words(n), s)))
      return rc;
    if ((rc = launch_trsv_chain(P, LU, ldlu, pslu, X, n, nc, 0, flags, s))) return rc;
    if ((rc = launch_trsv_chain(P, LU, ldlu, pslu, X, n, nc, 1, flags, s))) return rc;
    if ((rc = launch_scatter_rows(P, X, n, nc, B + c0, ldb, psb, s))) return rc;
  }
  return DDQD_OK;
}

// Tuning workspace: a copy of A, the pivots (ipiv, perm, info) and the
// factorization's workspace for every candidate width.
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t getrf_tune_ws(int P, int64_t n, int algo, int levels, int base) {
  if (n < 0 || n > kMaxLuRows || algo < 0 || algo > 3 || levels < 0 || levels > 6 ||
      !lu_base_ok(P, base))
    return SIZE_MAX;
  const size_t prod = auto_panel_ws(P, n, algo, levels, base);
  if (prod == SIZE_MAX) return SIZE_MAX;
  return align256(sizeof(double) * P * (size_t)(n * n)) +
         align256(sizeof(int32_t) * (size_t)(2 * n + 1)) + prod;
}

int getrf_tune(int P, int64_t n, const double* A, int64_t lda, int64_t psa, int pivot, int algo,
               int levels, int base, int reps, void* ws, size_t ws_bytes, void* stream,
               int* panel_out, double* ms_out) {
  clear_error();
  if (reps < 1 || reps > 100) return set_error(DDQD_E_ARG, "reps must be in 1..100");
  if (n < 0) return set_error(DDQD_E_ARG, "negative order");
  if (n > kMaxLuRows)
    return set_error(DDQD_E_UNSUPPORTED, "LU of order above %lld", (long long)kMaxLuRows);
  if (pivot != DDQD_PIVOT_NONE && pivot != DDQD_PIVOT_PARTIAL)
    return set_error(DDQD_E_ARG, "pivot must be DDQD_PIVOT_NONE or DDQD_PIVOT_PARTIAL");
  if (algo < 0 || algo > 3 || levels < 0 || levels > 6 || !lu_base_ok(P, base))
    return set_error(DDQD_E_ARG, "bad product algorithm / levels / base");
  int rc;
  if ((rc = check_matrix("A", P, A, n, n, lda, psa))) return rc;
  const size_t need = getrf_tune_ws(P, n, algo, levels, base);
  if (need == SIZE_MAX) return set_error(DDQD_E_ARG, "bad product arguments");
  if (need > ws_bytes || (need > 0 && !ws))
    return set_error(DDQD_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                     ws_bytes);
  if ((rc = check_device())) return rc;
  if (n == 0) {
    if (panel_out) *panel_out = kDefaultPanel;
    if (ms_out) *ms_out = 0.0;
    return DDQD_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  double* Ac = (double*)ws;
  int32_t* ipiv = (int32_t*)((char*)ws + align256(sizeof(double) * P * (size_t)(n * n)));
  int32_t* perm = ipiv + n;
  int32_t* info = perm + n;
  char* pw = (char*)ipiv + align256(sizeof(int32_t) * (size_t)(2 * n + 1));
  const size_t pw_bytes = need - (size_t)(pw - (char*)ws);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return set_error(DDQD_E_HIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(DDQD_E_HIP, "hipEventCreate failed");
  }
  const std::vector<int> cs = panel_candidates(n);
  PanelChoice best{kDefaultPanel, (int)cs.size(), 0.0};
  bool have = false;
  for (int K : cs) {
    double total = 0.0;
    for (int r = 0; r <= reps && !rc; r++) {  // the first factorization is not timed
      for (int c = 0; c < P && !rc; c++)
        if (hipMemcpy2DAsync(Ac + c * n * n, sizeof(double) * n, A + c * psa, sizeof(double) * lda,
                             sizeof(double) * n, n, hipMemcpyDeviceToDevice, s) != hipSuccess)
          rc = set_error(DDQD_E_HIP, "copy of A failed");
      if (rc) break;
      float ms = 0.0f;
      if (hipEventRecord(e0, s) != hipSuccess) {
        rc = set_error(DDQD_E_HIP, "hipEventRecord failed");
        break;
      }
      if ((rc = getrf_entry(P, n, Ac, n, n * n, ipiv, perm, info, K, pivot, algo, levels, base, pw,
                            pw_bytes, stream)))
        break;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = set_error(DDQD_E_HIP, "timing events failed");
        break;
      }
      if (r > 0) total += ms;
    }
    if (rc) break;
    const double per = total / reps;
    if (!have || per < best.ms) {
      best.panel = K;
      best.ms = per;
      have = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_panel_mu);
    g_panel_cache[PanelKey{P, n, pivot, algo, levels, base}] = best;
  }
  if (panel_out) *panel_out = best.panel;
  if (ms_out) *ms_out = best.ms;
  return DDQD_OK;
}

// ---- allocation-free solve (dd_getrs_noalloc) --------------------------
//
// The workspace of a DD solve of order up to kMaxLuRows (any number of
// right-hand sides: they are solved 16 at a time in the same buffer) lives in
// a file-scope device array.  In host code `scratch` names a host-side stand-in;
// the device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and only that address is passed to kernels.
constexpr size_t kNoAllocBytes = getrs_ws(2, kMaxLuRows, 16);

}  // namespace
}  // namespace ddqd

static __device__ __align__(256) unsigned char scratch[ddqd::kNoAllocBytes];

namespace ddqd {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, once known

// The device address of this device's `scratch`, looked up on first use with
// the device current.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(DDQD_E_UNSUPPORTED, "device %d above the %d the library tracks", dev,
                     kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
      return set_error(DDQD_E_HIP, "hipGetDevice failed");
    if (cur != dev && hipSetDevice(dev) != hipSuccess)
      return set_error(DDQD_E_HIP, "hipSetDevice(%d) failed", dev);
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return set_error(DDQD_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DDQD_OK;
}

int getrs_noalloc_entry(int64_t n, int64_t nrhs, const double* LU, int64_t ldlu, int64_t pslu,
                        const int32_t* ipiv, const int32_t* perm, double* B, int64_t ldb,
                        int64_t psb, void* stream) {
  clear_error();
  if (n < 0 || nrhs < 0) return set_error(DDQD_E_ARG, "negative dimension");
  if (n == 0 || nrhs == 0) return DDQD_OK;
  if (n > kMaxLuRows)
    return set_error(DDQD_E_UNSUPPORTED,
                     "dd_getrs_noalloc: order %lld above its scratch limit of %lld",
                     (long long)n, (long long)kMaxLuRows);
  static_assert(getrs_ws(2, kMaxLuRows, 16) <= kNoAllocBytes, "scratch too small");
  int rc;
  if ((rc = check_device())) return rc;
  int dev = -1;
  hipStream_t s = (hipStream_t)stream;
  if (s) {
    if (hipStreamGetDevice(s, &dev) != hipSuccess)
      return set_error(DDQD_E_ARG, "stream has no device");
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return set_error(DDQD_E_HIP, "hipGetDevice failed");
  }
  void* ws = nullptr;
  if ((rc = scratch_address(dev, &ws))) return rc;
  return getrs_entry(2, n, nrhs, LU, ldlu, pslu, ipiv, perm, B, ldb, psb, ws, kNoAllocBytes,
                     stream);
}

}  // namespace
}  // namespace ddqd

namespace ddqd {
void lu_tune_clear() {
  std::lock_guard<std::mutex> lk(g_panel_mu);
  g_panel_cache.clear();
}
}  // namespace ddqd

using namespace ddqd;

extern "C" {

int ddqd_getrf_tune(int precision, int64_t n, const double* A, int64_t lda, int64_t psa,
                    int pivot, int algo, int levels, int base, int reps, void* ws,
                    size_t ws_bytes, void* stream, int* panel, double* ms) {
  if (precision != 2 && precision != 4) {
    clear_error();
    return set_error(DDQD_E_ARG, "precision must be 2 (DD) or 4 (QD)");
  }
  return getrf_tune(precision, n, A, lda, psa, pivot, algo, levels, base, reps, ws, ws_bytes,
                    stream, panel, ms);
}

size_t ddqd_getrf_tune_workspace(int precision, int64_t n, int algo, int levels, int base) {
  if (precision != 2 && precision != 4) return SIZE_MAX;
  return getrf_tune_ws(precision, n, algo, levels, base);
}

int ddqd_getrf_panel_lookup(int precision, int64_t n, int pivot, int algo, int levels, int base,
                            int* panel, int* candidates, double* ms) {
  clear_error();
  if (!panel) return set_error(DDQD_E_ARG, "panel is NULL");
  if ((precision != 2 && precision != 4) || n < 0 ||
      (pivot != DDQD_PIVOT_NONE && pivot != DDQD_PIVOT_PARTIAL) || algo < 0 || algo > 3 ||
      levels < 0 || levels > 6 || !lu_base_ok(precision, base))
    return set_error(DDQD_E_ARG, "invalid panel lookup arguments");
  const PanelChoice c = panel_choice(precision, n, pivot, algo, levels, base);
  *panel = c.panel;
  if (candidates) *candidates = c.candidates;
  if (ms) *ms = c.ms;
  return DDQD_OK;
}

size_t dd_getrf_workspace(int64_t n, int panel_width, int algo, int levels, int base) {
  return getrf_workspace_entry(2, n, panel_width, algo, levels, base);
}

int dd_getrf(int64_t n, double* A, int64_t lda, int64_t psa, int32_t* ipiv, int32_t* perm,
             int32_t* info, int panel_width, int pivot, int algo, int levels, int base, void* ws,
             size_t ws_bytes, void* stream) {
  return getrf_entry(2, n, A, lda, psa, ipiv, perm, info, panel_width, pivot, algo, levels, base,
                     ws, ws_bytes, stream);
}

size_t dd_getrs_workspace(int64_t n, int64_t nrhs) { return getrs_workspace_entry(2, n, nrhs); }

int dd_getrs(int64_t n, int64_t nrhs, const double* LU, int64_t ldlu, int64_t pslu,
             const int32_t* ipiv, const int32_t* perm, double* B, int64_t ldb, int64_t psb,
             void* ws, size_t ws_bytes, void* stream) {
  return getrs_entry(2, n, nrhs, LU, ldlu, pslu, ipiv, perm, B, ldb, psb, ws, ws_bytes, stream);
}

size_t qd_getrf_workspace(int64_t n, int panel_width, int algo, int levels, int base) {
  return getrf_workspace_entry(4, n, panel_width, algo, levels, base);
}

int qd_getrf(int64_t n, double* A, int64_t lda, int64_t psa, int32_t* ipiv, int32_t* perm,
             int32_t* info, int panel_width, int pivot, int algo, int levels, int base, void* ws,
             size_t ws_bytes, void* stream) {
  return getrf_entry(4, n, A, lda, psa, ipiv, perm, info, panel_width, pivot, algo, levels, base,
                     ws, ws_bytes, stream);
}

int dd_getrs_noalloc(int64_t n, int64_t nrhs, const double* LU, int64_t ldlu, int64_t pslu,
                     const int32_t* ipiv, const int32_t* perm, double* B, int64_t ldb,
                     int64_t psb, void* stream) {
  return getrs_noalloc_entry(n, nrhs, LU, ldlu, pslu, ipiv, perm, B, ldb, psb, stream);
}

size_t qd_getrs_workspace(int64_t n, int64_t nrhs) { return getrs_workspace_entry(4, n, nrhs); }

int qd_getrs(int64_t n, int64_t nrhs, const double* LU, int64_t ldlu, int64_t pslu,
             const int32_t* ipiv, const int32_t* perm, double* B, int64_t ldb, int64_t psb,
             void* ws, size_t ws_bytes, void* stream) {
  return getrs_entry(4, n, nrhs, LU, ldlu, pslu, ipiv, perm, B, ldb, psb, ws, ws_bytes, stream);
}

}  // extern "C"
