// Autotuner: per-shape choice of product algorithm, recursion depth, Block
// tile (FMA leaves) and tile-order band (Ozaki leaves), timed on the device
// and cached process-wide (DDQD_AUTO).
//
// The paper names the block size and the recursion depth as the tuning
// parameters left open (Sec. 5).  The candidates of one shape all compute a
// correct product with the caller's base and slice count; only their speed
// is compared, so the cache never trades accuracy.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "ddqd.h"

namespace ddqd {

int gemm_entry(int P, int64_t m, int64_t n, int64_t l, int alpha, const double* A, int64_t lda,
               int64_t psa, const double* B, int64_t ldb, int64_t psb, int beta, double* C,
               int64_t ldc, int64_t psc, int algo, int levels, int base, int slices, void* ws,
               size_t ws_bytes, void* stream, int tile, int band);
size_t plan_workspace(int P, int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
                      int slices);
void clear_error();
void lu_tune_clear();

namespace {

struct Key {
  int P;
  int64_t m, n, l;
  int base, slices;
  bool operator<(const Key& o) const {
    return std::tie(P, m, n, l, base, slices) < std::tie(o.P, o.m, o.n, o.l, o.base, o.slices);
  }
};

struct Choice {
  int algo, levels, tile, band, candidates;
  double ms;
};

std::mutex g_mu;
std::map<Key, Choice> g_cache;

constexpr int kMaxTuneLevels = 3, kMinLeaf = 16;

int64_t min3(int64_t a, int64_t b, int64_t c) { return std::min(a, std::min(b, c)); }

// Block FMA leaves: the smaller tile (DD 32x32, QD 16x16) when the larger
// one would not give every compute unit one workgroup; 0 for Ozaki leaves.
int leaf_tile(int P, int base, int64_t m, int64_t n, int64_t batch) {
  if (base != DDQD_BASE_FMA) return 0;
  const int big = P == 2 ? 64 : 32;
  const int64_t tiles = ((m + big - 1) / big) * ((n + big - 1) / big) * batch;
  return tiles < 256 ? big / 2 : big;
}

std::vector<Choice> candidates(int P, int64_t m, int64_t n, int64_t l, int base) {
  std::vector<Choice> c;
  if (base == DDQD_BASE_FMA) {
    const int big = P == 2 ? 64 : 32;
    c.push_back(Choice{DDQD_BLOCK, 0, big, 0, 0, 0.0});
    c.push_back(Choice{DDQD_BLOCK, 0, big / 2, 0, 0, 0.0});
  } else if (base == DDQD_BASE_OZAKI_I8) {
    // Ozaki leaves: the band of tile rows an XCD's consecutive tiles span
    for (int band : {2, 4, 8, 16}) c.push_back(Choice{DDQD_BLOCK, 0, 0, band, 0, 0.0});
  } else {
    // CRT leaves: 128 x 128 or 256 x 256 product tiles
    for (int t : {128, 256}) c.push_back(Choice{DDQD_BLOCK, 0, t, 0, 0, 0.0});
  }
  int64_t batch = 1;
  for (int L = 1; L <= kMaxTuneLevels; L++) {
    batch *= 7;
    const int64_t d = min3(m, n, l) >> L;
    if (d < kMinLeaf) break;
    const int t = leaf_tile(P, base, m >> L, n >> L, batch);
    c.push_back(Choice{DDQD_STRASSEN, L, t, 0, 0, 0.0});
    c.push_back(Choice{DDQD_WINOGRAD, L, t, 0, 0, 0.0});
  }
  return c;
}

Choice default_choice(int P, int64_t m, int64_t n, int64_t l, int base) {
  if (P == 4 && base == DDQD_BASE_FMA) {
    int L = 0;
    while (L < kMaxTuneLevels && (min3(m, n, l) >> (L + 1)) >= 128) L++;
    int64_t batch = 1;
    for (int j = 0; j < L; j++) batch *= 7;
    return Choice{L ? DDQD_WINOGRAD : DDQD_BLOCK, L, leaf_tile(P, base, m >> L, n >> L, batch),
                  0, 0, 0.0};
  }
  return Choice{DDQD_BLOCK, 0, leaf_tile(P, base, m, n, 1), 0, 0, 0.0};
}

int tune(int P, int64_t m, int64_t n, int64_t l, const double* A, int64_t lda, int64_t psa,
         const double* B, int64_t ldb, int64_t psb, double* C, int64_t ldc, int64_t psc, int base,
         int slices, int reps, void* ws, size_t ws_bytes, void* stream, ddqd_tune_result* out) {
  clear_error();
  if (reps < 1 || reps > 1000) return set_error(DDQD_E_ARG, "reps must be in 1..1000");
  // validation (and the no-op cases) exactly as the product itself
  int rc = gemm_entry(P, m, n, l, 1, A, lda, psa, B, ldb, psb, 0, C, ldc, psc, DDQD_AUTO, 0, base,
                      slices, ws, ws_bytes, stream, 0, 0);
  if (rc) return rc;
  if (m == 0 || n == 0 || l == 0) {
    if (out) *out = ddqd_tune_result{DDQD_BLOCK, 0, 0, 0, 0, 0.0};
    return DDQD_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return set_error(DDQD_E_HIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(DDQD_E_HIP, "hipEventCreate failed");
  }
  std::vector<Choice> cs = candidates(P, m, n, l, base);
  Choice best{0, 0, 0, 0, 0, 0.0};
  bool have = false;
  for (const Choice& c : cs) {
    auto run = [&]() {
      return gemm_entry(P, m, n, l, 1, A, lda, psa, B, ldb, psb, 0, C, ldc, psc, c.algo, c.levels,
                        base, slices, ws, ws_bytes, stream, c.tile, c.band);
    };
    if ((rc = run())) break;
    if (hipEventRecord(e0, s) != hipSuccess) {
      rc = set_error(DDQD_E_HIP, "hipEventRecord failed");
      break;
    }
    for (int r = 0; r < reps && !rc; r++) rc = run();
    if (rc) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = set_error(DDQD_E_HIP, "timing events failed");
      break;
    }
    const double per = (double)ms / reps;
    if (!have || per < best.ms) {
      best = c;
      best.ms = per;
      have = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  best.candidates = (int)cs.size();
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[Key{P, m, n, l, base, slices}] = best;
  }
  if (out)
    *out = ddqd_tune_result{best.algo, best.levels, best.tile, best.band, best.candidates,
                            best.ms};
  return DDQD_OK;
}

}  // namespace

void auto_choice(int P, int64_t m, int64_t n, int64_t l, int base, int slices, int* algo,
                 int* levels, int* tile, int* band) {
  Choice c = default_choice(P, m, n, l, base);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(Key{P, m, n, l, base, slices});
    if (it != g_cache.end()) c = it->second;
  }
  *algo = c.algo;
  *levels = c.levels;
  *tile = c.tile;
  *band = c.band;
}

size_t auto_workspace(int P, int64_t m, int64_t n, int64_t l, int base, int slices) {
  size_t w = 0;
  for (const Choice& c : candidates(P, m, n, l, base))
    w = std::max(w, plan_workspace(P, m, n, l, c.algo, c.levels, base, slices));
  const Choice d = default_choice(P, m, n, l, base);
  return std::max(w, plan_workspace(P, m, n, l, d.algo, d.levels, base, slices));
}

}  // namespace ddqd

using namespace ddqd;

extern "C" {

int dd_gemm_tune(int64_t m, int64_t n, int64_t l, const double* A, int64_t lda, int64_t psa,
                 const double* B, int64_t ldb, int64_t psb, double* C, int64_t ldc, int64_t psc,
                 int base, int slices, int reps, void* ws, size_t ws_bytes, void* stream,
                 ddqd_tune_result* out) {
  return tune(2, m, n, l, A, lda, psa, B, ldb, psb, C, ldc, psc, base, slices, reps, ws, ws_bytes,
              stream, out);
}

int qd_gemm_tune(int64_t m, int64_t n, int64_t l, const double* A, int64_t lda, int64_t psa,
                 const double* B, int64_t ldb, int64_t psb, double* C, int64_t ldc, int64_t psc,
                 int base, int slices, int reps, void* ws, size_t ws_bytes, void* stream,
                 ddqd_tune_result* out) {
  return tune(4, m, n, l, A, lda, psa, B, ldb, psb, C, ldc, psc, base, slices, reps, ws, ws_bytes,
              stream, out);
}

int ddqd_tune_lookup(int precision, int64_t m, int64_t n, int64_t l, int base, int slices,
                     ddqd_tune_result* out) {
  clear_error();
  if (!out) return set_error(DDQD_E_ARG, "out is NULL");
  if ((precision != 2 && precision != 4) || m < 0 || n < 0 || l < 0 ||
      (base != DDQD_BASE_FMA && base != DDQD_BASE_OZAKI_I8 && base != DDQD_BASE_CRT_I8) ||
      slices < 0 || slices > 40)
    return set_error(DDQD_E_ARG, "invalid tune lookup arguments");
  Choice c = default_choice(precision, m, n, l, base);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(Key{precision, m, n, l, base, slices});
    if (it != g_cache.end()) c = it->second;
  }
  *out = ddqd_tune_result{c.algo, c.levels, c.tile, c.band, c.candidates, c.ms};
  return DDQD_OK;
}

void ddqd_tune_clear(void) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
  }
  lu_tune_clear();
}

}  // extern "C"
