/*
 * ddqd — double-double (DD) and quad-double (QD) matrix products and DD LU
 * on AMD Instinct MI355X (gfx950).  C ABI of libddqd.so.
 *
 * The operations follow Kouya, "Performance evaluation of multiple precision
 * matrix multiplications using parallelized Strassen and Winograd
 * algorithms" (arXiv 1510.08642):
 *   - the product C := AB of an m x l matrix A and an l x n matrix B, any
 *     sizes, with c_ij = sum_k a_ik b_kj (Sec. 2, Eq. 1), computed by the
 *     Simple, Block, Strassen or Winograd algorithm (Sec. 2, Sec. 3);
 *   - LU decomposition by blocks whose trailing update A22 := A22 - L21 U12
 *     is such a product (Sec. 4, steps 1-3), and the solve of A x = b with
 *     the factors (Sec. 4, Eq. 2).
 *
 * Numbers.  A DD number is an unevaluated sum hi + lo of two doubles (about
 * 106 bits); a QD number is c0 + c1 + c2 + c3 (about 212 bits).  Inputs are
 * expected non-overlapping (|lo| <= ulp(hi)/2); outputs are written that way.
 *
 * Matrices.  Every matrix argument is a device pointer p to P row-major
 * float64 planes (P = 2 for DD, 4 for QD): component c of element (i, j) is
 * p[c*ps + i*ld + j].  ld >= number of columns; ps (plane stride, in
 * elements) must keep the planes from overlapping.  Only 8-byte alignment is
 * required.
 *
 * Ownership and ordering.  The caller owns every buffer, including the
 * workspace, whose size it obtains from the matching *_workspace query.  The
 * library never allocates or frees device memory on these calls.  All work is
 * enqueued on `stream` (a hipStream_t; NULL = the default stream) and the
 * calls return without waiting for it.
 *
 * Errors.  The return value is decided before anything is enqueued (except
 * DDQD_E_HIP, a failed launch).  ddqd_last_error() gives a message for the
 * last failure on the calling thread.  Non-finite inputs give unspecified
 * results.
 */
#ifndef DDQD_H
#define DDQD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DDQD_OK 0
#define DDQD_E_ARG 1         /* an argument is out of range */
#define DDQD_E_ALIAS 2       /* an output overlaps an input */
#define DDQD_E_WORKSPACE 3   /* workspace missing or too small */
#define DDQD_E_UNSUPPORTED 4 /* a valid combination the library does not implement */
#define DDQD_E_NODEVICE 5    /* no usable GPU */
#define DDQD_E_HIP 6         /* a HIP call or launch failed */

/* algorithms (Sec. 2 and Sec. 3 of the paper) */
#define DDQD_SIMPLE 0   /* one thread per c_ij, k ascending (Eq. 1)      */
#define DDQD_BLOCK 1    /* tiled product                                  */
#define DDQD_STRASSEN 2 /* Strassen's recursion, `levels` deep            */
#define DDQD_WINOGRAD 3 /* Strassen-Winograd recursion, `levels` deep     */
#define DDQD_AUTO 4     /* tuned (dd_gemm_tune) or default configuration  */

/* base (leaf) product kernels */
#define DDQD_BASE_FMA 0      /* FP64 FMA error-free products                 */
#define DDQD_BASE_OZAKI_I8 1 /* slices on INT8 matrix cores, FP64 recombine  */
/* (an Ozaki-style split, not in the paper: each operand is scaled by powers
 * of two per row of A / column of B and cut into `slices` signed 7-bit digits;
 * the digit products run exactly on v_mfma_i32_32x32x32_i8 and are recombined
 * in FP64.  Leaf error at most about l (S+3) 2^(-7S-2) max|a_i.| max|b_.j|
 * times 16, S the slice count.) */
#define DDQD_BASE_CRT_I8 2 /* residues on INT8 matrix cores, CRT rebuild      */
/* (the same scaling, each operand then rounded to integers of at most 107
 * bits and reduced modulo N pairwise coprime moduli <= 256, N = 29..31 by K;
 * one exact INT8 product per modulus, the integer product rebuilt by the
 * Chinese remainder theorem in 160-bit fixed point.  Leaf error at most about
 * 2^-103 l max|a_i.| max|b_.j| for normalised DD inputs (|lo| at most half an
 * ulp of hi).  QD: integers of 214 bits, each split into a high part H of
 * 107 bits and a low part L of 108; H_a H_b and H_a L_b + L_a H_b run as two
 * exact products per modulus (the second over 2 K), L_a L_b is dropped, and
 * the rebuild works in 270-bit fixed point; leaf error at most about
 * 2^-211 l max|a_i.| max|b_.j| for normalised QD inputs (each term at most
 * half an ulp of the one before).  `slices` must be 0.) */

/*
 * The moduli DDQD_BASE_CRT_I8 uses for a product with K = l in precision 2
 * (DD) or 4 (QD): writes the first min(N, cap) of them to out (host memory)
 * and returns N, the count (the product of the N moduli exceeds
 * 2 min(l, 65536) 2^214 in DD, min(l, 32768) 2^215 (1 + 2^-35) in QD); -1 for
 * another precision, l <= 0, a negative cap, or out NULL with cap > 0.  No
 * device work.
 */
int ddqd_crt_moduli(int precision, int64_t l, int* out, int cap);

/* pivoting for dd_getrf */
#define DDQD_PIVOT_NONE 0
#define DDQD_PIVOT_PARTIAL 1

/* panel width for dd_getrf / qd_getrf: the tuned width (ddqd_getrf_tune) */
#define DDQD_PANEL_AUTO (-1)

/* Human-readable name of a status code. */
const char* ddqd_status_string(int status);

/* Message describing the last failed call on this thread ("" if none). */
const char* ddqd_last_error(void);

/* Diagnostics: per-kernel timing.  While enabled (on != 0), every kernel the
 * library launches is bracketed by HIP events on its stream (creating two
 * events per launch).  ddqd_profile_query sums the elapsed milliseconds and
 * counts the launches whose kernel name contains `substr` (all if NULL),
 * waiting for the recorded events; ddqd_profile_reset forgets them. */
void ddqd_profile_enable(int on);
void ddqd_profile_reset(void);
int ddqd_profile_query(const char* substr, double* ms, int64_t* count);

/*
 * C := beta*C + alpha*(A B) in DD (Sec. 2, Eq. 1).
 *   m, n, l   A is m x l, B is l x n, C is m x n; each >= 0.  m == 0 or
 *             n == 0 is a no-op; l == 0 gives C := beta*C.
 *   alpha     +1 or -1.      beta  0 or 1 (0: C is not read).
 *   A, B, C   device plane-layout DD matrices (2 planes) with leading
 *             dimensions lda, ldb, ldc and plane strides psa, psb, psc.
 *             C must not overlap A or B (DDQD_E_ALIAS); A and B may overlap.
 *   algo      DDQD_SIMPLE, DDQD_BLOCK, DDQD_STRASSEN or DDQD_WINOGRAD, or
 *             DDQD_AUTO (see dd_gemm_tune; `levels` is then ignored).
 *   levels    recursion depth L for Strassen/Winograd (0..6); the depth
 *             actually used stops early once a dimension would drop below 2.
 *             Each level splits m, l and n in half: a dimension that 2^L
 *             does not divide is cut down to a multiple (remainder <=
 *             2^(L-1): the last rows / columns / k become Block products at
 *             the top level) or padded with zeros up to one inside the
 *             workspace (the padding is never read from A, B or C, nor
 *             written to C).
 *   base      DDQD_BASE_FMA, DDQD_BASE_OZAKI_I8 or DDQD_BASE_CRT_I8 for the
 *             leaf products (ignored by DDQD_SIMPLE).
 *   slices    Ozaki slice count (0 = automatic); ignored for FMA; 0 for CRT.
 *   ws        device workspace of ws_bytes >= dd_gemm_workspace(...) bytes,
 *             8-byte aligned (may be NULL when that size is 0).
 *   stream    hipStream_t to enqueue on.
 */
int dd_gemm(int64_t m, int64_t n, int64_t l, int alpha, const double* A, int64_t lda,
            int64_t psa, const double* B, int64_t ldb, int64_t psb, int beta, double* C,
            int64_t ldc, int64_t psc, int algo, int levels, int base, int slices, void* ws,
            size_t ws_bytes, void* stream);

/* Workspace bytes dd_gemm needs for these arguments (0 if none; SIZE_MAX if
 * the arguments are invalid). */
size_t dd_gemm_workspace(int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
                         int slices);

/* One problem of a grouped launch: C := beta*C + alpha*(A B), as in dd_gemm
 * with DDQD_BLOCK and the given base (DDQD_BASE_FMA or DDQD_BASE_OZAKI_I8)
 * and Ozaki slice count (0 = 16, else 8..20; ignored for FMA). */
typedef struct {
  int64_t m, n, l;
  int alpha, beta;
  int base, slices;
  const double* A;
  int64_t lda, psa;
  const double* B;
  int64_t ldb, psb;
  double* C;
  int64_t ldc, psc;
} ddqd_gemm_desc;

/*
 * `count` unrelated DD products of any shapes and bases (host array of
 * descriptors, read before the call returns) in grouped launches instead of
 * one per problem, for the uneven small products of a serving batch or of
 * an LU step (the paper runs independent products as parallel sections,
 * Sec. 2): FMA problems in persistent Block launches of up to 24 problems
 * each; Ozaki problems, per slice count, in launches of up to 12 problems
 * (one exponent, one slicing and one product launch per group; a problem
 * with l > 16384 runs as a product of its own).  Each problem's result is
 * bit-identical to the same dd_gemm call with DDQD_BLOCK and its base and
 * slices.  No output may overlap any input or another output of the group
 * (DDQD_E_ALIAS).
 *   ws     device workspace of ws_bytes >= dd_gemm_grouped_workspace(count,
 *          descs) bytes, 8-byte aligned (may be NULL when that size is 0:
 *          a group of FMA problems needs none).
 */
int dd_gemm_grouped(int count, const ddqd_gemm_desc* descs, void* ws, size_t ws_bytes,
                    void* stream);

/* Workspace bytes dd_gemm_grouped needs for these descriptors (SIZE_MAX if
 * one of them is invalid). */
size_t dd_gemm_grouped_workspace(int count, const ddqd_gemm_desc* descs);

/* As dd_gemm, in QD (4 planes per matrix; Sec. 3, Table 2's precision).
 * With DDQD_BASE_OZAKI_I8 the slice count is 0 = 31 or 28..31 (else
 * DDQD_E_UNSUPPORTED); 31 slices keep the leaf error below about
 * 2^-209 l max|a_i.| max|b_.j|, QD's accuracy class.  DDQD_BASE_CRT_I8
 * (slices 0) keeps it below about 2^-211 l max|a_i.| max|b_.j| plus the
 * rebuild's QD rounding. */
int qd_gemm(int64_t m, int64_t n, int64_t l, int alpha, const double* A, int64_t lda,
            int64_t psa, const double* B, int64_t ldb, int64_t psb, int beta, double* C,
            int64_t ldc, int64_t psc, int algo, int levels, int base, int slices, void* ws,
            size_t ws_bytes, void* stream);

size_t qd_gemm_workspace(int64_t m, int64_t n, int64_t l, int algo, int levels, int base,
                         int slices);

/*
 * In-place LU factorisation P A = L U of the n x n DD matrix A by the blocked
 * right-looking method of the paper (Sec. 4, steps 1-3): panels of width
 * `panel` (the last may be narrower); after each panel, U12 := L11^-1 A12 and
 * the trailing update A22 := A22 - L21 U12 is a product computed with
 * `algo`, `levels` and `base` as in dd_gemm.
 *   A        device plane-layout DD matrix (lda >= n, psa), overwritten by L
 *            (unit lower, below the diagonal) and U (upper, with diagonal).
 *   ipiv     device int32[n]: row i was interchanged with row ipiv[i]
 *            (0-based, LAPACK order).
 *   perm     device int32[n] or NULL: the resulting permutation, row i of
 *            P A is row perm[i] of A (lets dd_getrs gather in parallel).
 *   info     device int32[1]: 0, or 1 + the first column whose pivot is
 *            exactly zero (the factorisation still completes).
 *   pivot    DDQD_PIVOT_PARTIAL (largest |a_ic| below the diagonal, first row
 *            on ties, compared in DD) or DDQD_PIVOT_NONE (the paper's choice).
 *   panel    >= 1: the blocked method above.  0: the paper's comparator,
 *            row-wise parallel elimination without blocking (one launch per
 *            elimination step, every trailing row updated in parallel; Sec. 4
 *            compares the blocked LU against it); requires DDQD_PIVOT_NONE
 *            (else DDQD_E_UNSUPPORTED), ignores algo / levels / base and needs
 *            no workspace.  DDQD_PANEL_AUTO: the width ddqd_getrf_tune chose
 *            for this order, pivoting and product, else 128.
 *   ws       workspace of dd_getrf_workspace(...) bytes (the product's; with
 *            DDQD_PANEL_AUTO, enough for every width the tuner may choose).
 * Orders above 8192 return DDQD_E_UNSUPPORTED.
 */
int dd_getrf(int64_t n, double* A, int64_t lda, int64_t psa, int32_t* ipiv, int32_t* perm,
             int32_t* info, int panel, int pivot, int algo, int levels, int base, void* ws,
             size_t ws_bytes, void* stream);

size_t dd_getrf_workspace(int64_t n, int panel, int algo, int levels, int base);

/*
 * Solves A X = B (Sec. 4, Eq. 2) with dd_getrf's factors: X = U^-1 L^-1 P B.
 *   LU       the factored matrix (ldlu, pslu); ipiv its interchanges; perm
 *            its permutation or NULL (then it is rebuilt from ipiv, serially).
 *   B        device DD n x nrhs (ldb >= nrhs), overwritten by X; must not
 *            overlap LU.
 *   ws       workspace of dd_getrs_workspace(n, nrhs) bytes (the gathered
 *            right-hand sides and a counter of the block solves); calls
 *            that share one workspace must not run at the same time.
 */
int dd_getrs(int64_t n, int64_t nrhs, const double* LU, int64_t ldlu, int64_t pslu,
             const int32_t* ipiv, const int32_t* perm, double* B, int64_t ldb, int64_t psb,
             void* ws, size_t ws_bytes, void* stream);

size_t dd_getrs_workspace(int64_t n, int64_t nrhs);

/*
 * dd_getrs without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): the same kernels and the same result, bit for bit,
 * as dd_getrs, with the workspace taken from a fixed buffer that the library
 * holds on each GPU until the process ends (about 2 MiB: the gathered
 * right-hand sides, 16 at a time, the block solves' counter and the
 * permutation for orders up to 8192).  The call allocates and frees nothing.
 *   n        order, at most 8192 (else DDQD_E_UNSUPPORTED, nothing enqueued);
 *            nrhs any (solved 16 at a time).
 *   other arguments and errors as dd_getrs.
 * The buffer's device address is looked up once per device (on that device's
 * first call; DDQD_E_HIP if the lookup fails).  Every call on one GPU uses
 * the same buffer, which keeps the last call's contents (the counter is
 * reset by the call's own kernels): calls that overlap on one GPU (on
 * different streams, or from several threads, with no ordering between them)
 * race and give wrong results; calls ordered on one stream are safe.
 */
int dd_getrs_noalloc(int64_t n, int64_t nrhs, const double* LU, int64_t ldlu, int64_t pslu,
                     const int32_t* ipiv, const int32_t* perm, double* B, int64_t ldb,
                     int64_t psb, void* stream);

/*
 * The same factorisation and solve in QD (4 planes per matrix; the paper's
 * second LU workload, Sec. 4): arguments, layouts, ipiv / perm / info and
 * errors as dd_getrf / dd_getrs.  Pivots are compared, and the panel is
 * factored, in QD; the trailing update is qd_gemm's product (any base;
 * Ozaki leaves with 31 slices).  Orders up to 8192.
 */
int qd_getrf(int64_t n, double* A, int64_t lda, int64_t psa, int32_t* ipiv, int32_t* perm,
             int32_t* info, int panel, int pivot, int algo, int levels, int base, void* ws,
             size_t ws_bytes, void* stream);
size_t qd_getrf_workspace(int64_t n, int panel, int algo, int levels, int base);
int qd_getrs(int64_t n, int64_t nrhs, const double* LU, int64_t ldlu, int64_t pslu,
             const int32_t* ipiv, const int32_t* perm, double* B, int64_t ldb, int64_t psb,
             void* ws, size_t ws_bytes, void* stream);
size_t qd_getrs_workspace(int64_t n, int64_t nrhs);

/*
 * Autotuning.  The paper leaves the choice of block size and recursion depth
 * per shape as future work (Sec. 5); here the library times the candidate
 * configurations of one shape on the device and keeps the fastest in a
 * process-wide, thread-safe cache that algo = DDQD_AUTO then uses.
 * Candidates: Block (FMA leaves: two tiles, DD 64x64 and 32x32, QD 32x32
 * and 16x16, which give bit-identical results; Ozaki leaves: tile orders in
 * bands of 2, 4, 8 or 16 tile rows, bit-identical too; CRT leaves: 128x128
 * or 256x256 product tiles, bit-identical), and Strassen and
 * Winograd with 1..3 levels while the leaves keep at least 16 rows and
 * columns.  The base and the slice count are the caller's: they set the
 * accuracy, the tuner only the speed.  Without a cache entry DDQD_AUTO takes
 * a default: Block for DD (the smaller tile when the larger would leave
 * compute units idle), Winograd for QD with levels while the leaves stay
 * >= 128.
 *   A, B, C  as dd_gemm with alpha = 1, beta = 0; C receives A B (computed
 *            by every candidate in turn).
 *   reps     timed calls per candidate (>= 1; one untimed call precedes).
 *   ws       dd_gemm_workspace(m, n, l, DDQD_AUTO, 0, base, slices) bytes,
 *            which also covers every later DDQD_AUTO call of this shape.
 *   out      the chosen configuration (may be NULL).
 * Blocks the calling thread until the timing on `stream` is done; cannot be
 * recorded in a graph.  Argument errors as dd_gemm.
 */
typedef struct {
  int algo;       /* DDQD_BLOCK, DDQD_STRASSEN or DDQD_WINOGRAD */
  int levels;     /* recursion depth */
  int tile;       /* Block leaf tile edge (FMA: DD 64 or 32, QD 32 or 16; CRT: 128 or
                     256), 0 for Ozaki */
  int band;       /* Ozaki leaves: tile rows per band of the tile order, 0 = default */
  int candidates; /* configurations timed; 0 = not tuned, default shown */
  double ms;      /* time per call of the chosen configuration (0 if not tuned) */
} ddqd_tune_result;

int dd_gemm_tune(int64_t m, int64_t n, int64_t l, const double* A, int64_t lda, int64_t psa,
                 const double* B, int64_t ldb, int64_t psb, double* C, int64_t ldc, int64_t psc,
                 int base, int slices, int reps, void* ws, size_t ws_bytes, void* stream,
                 ddqd_tune_result* out);
int qd_gemm_tune(int64_t m, int64_t n, int64_t l, const double* A, int64_t lda, int64_t psa,
                 const double* B, int64_t ldb, int64_t psb, double* C, int64_t ldc, int64_t psc,
                 int base, int slices, int reps, void* ws, size_t ws_bytes, void* stream,
                 ddqd_tune_result* out);
/* The configuration DDQD_AUTO uses for this shape (precision 2 = DD, 4 = QD);
 * DDQD_E_ARG for bad arguments. */
int ddqd_tune_lookup(int precision, int64_t m, int64_t n, int64_t l, int base, int slices,
                     ddqd_tune_result* out);
/*
 * Diagnostic: dependent-chain latencies, in s_memtime ticks per step, of the
 * operations the LU column step is made of, timed inside one workgroup of
 * `threads` (64, 256 or 1024) threads over `steps` steps (1..2^20): out[0] a
 * dependent FP64 FMA, out[1] a dependent FP64 add, out[2] a TwoSum, out[3] a
 * lane shuffle with a max, out[4] two readlanes and an add, out[5] an LDS
 * write and read, out[6] two barriers around an LDS exchange, out[7] one step
 * of four independent FMA chains.  out: device double[9] (out[8] is
 * scratch).  Computes nothing the library uses.  DDQD_E_ARG for bad
 * arguments.
 */
int ddqd_latency_probe(double* out, int threads, int steps, void* stream);

/* Empties the caches (products and LU panel widths). */
void ddqd_tune_clear(void);

/*
 * LU panel width per order.  Sec. 4 runs the blocked LU with panel widths
 * K = 32 alpha, alpha = 1..10; the fastest K depends on the order and on the
 * product that updates the trailing matrix (Sec. 5 leaves the block size
 * open).  ddqd_getrf_tune factors a copy of A with every such K <= n (K = n
 * for n < 32), each `reps` times after one untimed run, and keeps the fastest
 * in a process-wide, thread-safe cache keyed by (precision, n, pivot, algo,
 * levels, base) that DDQD_PANEL_AUTO then uses.  Every width gives a correct
 * factorization; only the speed is compared.
 *   precision  2 (DD, dd_getrf) or 4 (QD, qd_getrf).
 *   A          device plane-layout n x n matrix (lda, psa); not modified.
 *   pivot, algo, levels, base  as dd_getrf.
 *   reps       timed factorizations per width (1..100).
 *   ws         ddqd_getrf_tune_workspace(precision, n, algo, levels, base)
 *              bytes: the copy of A, its pivots and the factorization's
 *              workspace for every width.
 *   panel, ms  the chosen width and its time per factorization (either may
 *              be NULL).
 * Blocks the calling thread until the timing on `stream` is done; cannot be
 * recorded in a graph.  Errors as dd_getrf (DDQD_E_ARG for a bad precision or
 * reps; SIZE_MAX from the workspace query for bad arguments).
 */
int ddqd_getrf_tune(int precision, int64_t n, const double* A, int64_t lda, int64_t psa,
                    int pivot, int algo, int levels, int base, int reps, void* ws,
                    size_t ws_bytes, void* stream, int* panel, double* ms);
size_t ddqd_getrf_tune_workspace(int precision, int64_t n, int algo, int levels, int base);
/* The width DDQD_PANEL_AUTO uses (tuned, else 128); candidates = widths
 * timed (0 if not tuned), ms = the chosen width's time (0 if not tuned); the
 * last two may be NULL.  DDQD_E_ARG for bad arguments. */
int ddqd_getrf_panel_lookup(int precision, int64_t n, int pivot, int algo, int levels, int base,
                            int* panel, int* candidates, double* ms);

/*
 * Captured launch sequences.  The calls above, issued on one non-null stream
 * between ddqd_graph_begin and ddqd_graph_end, are recorded into a HIP graph
 * instead of being executed; ddqd_graph_launch replays them on any stream:
 * the same kernels with the same arguments, so every buffer (operands,
 * outputs, workspaces, ipiv/perm/info) must stay allocated and in place, and
 * each replay rewrites the outputs and workspaces exactly as the recorded
 * calls would.  No library call allocates, frees, synchronises or clears
 * memory with a memset node, so all of them can be recorded (this is how
 * the LU's fixed chain of small launches, or a repeated small product, is
 * replayed without the host cost of each launch).  Per-kernel profiling
 * records nothing while capturing.
 *   begin    DDQD_E_ARG for a null stream, DDQD_E_HIP if capture fails to start.
 *   end      returns the graph in *graph (owned by the caller, released by
 *            ddqd_graph_destroy); DDQD_E_HIP (and *graph = NULL) if the
 *            capture was invalidated, e.g. by a foreign call on the stream.
 *   launch   DDQD_E_ARG for a null graph; asynchronous on `stream`.
 *   destroy  accepts NULL.
 */
typedef struct ddqd_graph* ddqd_graph_t;
int ddqd_graph_begin(void* stream);
int ddqd_graph_end(void* stream, ddqd_graph_t* graph);
int ddqd_graph_launch(ddqd_graph_t graph, void* stream);
int ddqd_graph_destroy(ddqd_graph_t graph);

#ifdef __cplusplus
}
#endif

#endif /* DDQD_H */
