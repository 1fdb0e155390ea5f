/* svdu.h -- rank-1 SVD update on one AMD MI355X (gfx950), C ABI.
 *
 * Method: Gandhi & Rajgor, "Updating Singular Value Decomposition for Rank
 * One Matrix Perturbation". Given A = U diag(sigma) V^T (U m x m, V n x n,
 * m <= n) and vectors a (m), b (n), return the SVD of A^ = A + a b^T
 * (Section 3, equation APurturbation1; Section 6.1, the algorithm "Update SVD
 * of rank-1 modified matrix"). The update runs the four symmetric rank-one
 * eigen-updates of A^ A^T and A^T A^ (equations U+D+U+T and V+D+V+T, Section
 * 6.2 RankOneUpdate): a secular-equation solve (equation
 * GolubEigenvalUpdate), the Cauchy eigenvector matrix C~ (equation
 * CTildeFinalForm1) and the product X C~ (equation UCTildeProduct).
 *
 * Conventions for every entry point:
 *  - Calls that enqueue work take a context (svdu_ctx, from svdu_create): it
 *    holds the options, the tile-shape tables and the phase-timing record of
 *    the calls made with it, and is bound to one device, which must be the
 *    current HIP device when such a call is made (SVDU_EINVAL otherwise).
 *    Contexts share no state: two threads may each use their own context at
 *    the same time; one context is used by one thread at a time.
 *  - Matrices are row-major float64 with an explicit leading dimension
 *    (element (r, c) of X is X[r * ldx + c]).
 *  - Every pointer argument is a DEVICE pointer owned by the caller, unless
 *    the comment says "host". The library never allocates device memory in
 *    these calls; scratch space comes from the caller's workspace.
 *  - `stream` is a hipStream_t (NULL: the default stream). Calls only enqueue
 *    work and return; results are valid once the stream has reached them.
 *  - Return value: 0 on success; a negative SVDU_E* code for an argument
 *    error found on the host (nothing is enqueued then). Errors found on the
 *    device (non-finite input, unsorted sigma, secular iteration cap) are
 *    recorded in the workspace and reported by svdu_get_status().
 */
#ifndef SVDU_H
#define SVDU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SVDU_OK 0
#define SVDU_EINVAL (-1)        /* an argument is out of range, NULL or aliased */
#define SVDU_ENOMEM (-2)        /* workspace smaller than svdu_*_workspace_bytes() */
#define SVDU_EHIP (-3)          /* a HIP runtime call failed */
#define SVDU_ENONFINITE (-4)    /* NaN or Inf in U, sigma, V, a or b (device check) */
#define SVDU_EBADSIGMA (-5)     /* sigma not descending or negative (device check) */
#define SVDU_ENOCONV (-6)       /* a secular root reached the iteration cap */
#define SVDU_ENOTSUP (-7)       /* path / precision combination not available */

/* product path for X C~ */
#define SVDU_PATH_DIRECT 0      /* dense FP64 MFMA GEMM, C~ generated in LDS */
#define SVDU_PATH_FMM 1         /* row-batched 1-D fast multipole (Section 5, Appendix D) */

/* arithmetic of the product X C~ (roots, deflation and norms are always FP64) */
#define SVDU_PREC_FP64 0
#define SVDU_PREC_SPLIT32 1     /* split FP32 hi/lo, three FP32 MFMA passes, FP32 accumulation drained to
                                   FP64 every 16 k; then every column of U^ and V^ rescaled to unit FP64 norm
                                   (kept as a measured negative result: about 1e-7 error, slower than FP64) */
#define SVDU_PREC_SLICED_INT8 2 /* exact slices on the INT8 matrix cores: every row of X and column of C~ is
                                   scaled by a power of two and cut into S signed 7-bit slices
                                   (SVDU_OPT_SLICES, default 7); the S (S + 1) / 2 slice products with
                                   s + t <= S + 1 are exact in INT32 and combined in FP64. Error about
                                   2^(1 - 7 S) relative to the largest entry (S = 7: about 1e-14) */

/* options of a context (svdu_set_option) */
#define SVDU_OPT_SECULAR_MAXIT 1 /* iteration cap of the secular solver (default 200) */
#define SVDU_OPT_TIMING 2        /* 1: record phase timings of svdu_rank1_update (resets the record) */
#define SVDU_OPT_TILE_SHAPE 3    /* -1 (default): tile shape of the products from the tuning table;
                                    0..5 force SVDU_TILE_* (results are bitwise the same for every shape;
                                    the split-FP32 precision form runs SVDU_TILE_128x128_K32 and
                                    SVDU_TILE_256x128_K64 as 128 x 128) */
#define SVDU_OPT_PERSISTENT 4    /* 1: products of svdu_rank1_update and svdu_rank1_update_batched use the
                                    persistent schedule (see SVDU_BATCH_PERSISTENT); default 0 */
#define SVDU_OPT_SLICES 6        /* slices S of SVDU_PREC_SLICED_INT8: 6, 7 (default) or 8 */
#define SVDU_OPT_SECULAR_FMM 7   /* 1 (default): for eigenproblems of order above 2048 the secular sums
                                    (Section 3.1) take their far field from Chebyshev interpolants sampled
                                    once per eigen-update, for each leaf of 64 consecutive poles (32
                                    points; a pole is far from a leaf when its distance is at least the
                                    leaf's width); near poles and the extreme root beyond the last pole
                                    take the direct sums. Every iterate then costs O(leaf + p) instead of
                                    O(K). Roots agree with the direct sums to rounding. Orders up to 2048
                                    take the direct sums. 0: direct sums for every order. 2: the far field
                                    at every order (for tests; slower below 2048). Other values:
                                    SVDU_EINVAL. */
#define SVDU_OPT_REFINE 5        /* 1 (default): FP64 results get the close-cluster refinement (not in the
                                    paper): for consecutive sigma^ with relative gaps <= 1e-6, in clusters
                                    of up to 8 and up to min(m, 128) columns in all, the block
                                    U^_c^T A^ V^_c is formed from the inputs and its SVD rotates U^_c and
                                    V^_c (sigma^ is kept); also for SVDU_PREC_SLICED_INT8. 0: off. Read when
                                    a call is enqueued (a batch graph keeps the value it was captured with). */

/* tile shapes of the product kernels (rows x columns of one block tile) */
#define SVDU_TILE_128x128 0
#define SVDU_TILE_64x128 1
#define SVDU_TILE_128x64 2
#define SVDU_TILE_64x64 3
#define SVDU_TILE_128x128_K32 4  /* 128 x 128, C~ staged 32 k rows at a time (one barrier per 32 k) */
#define SVDU_TILE_256x128_K64 5  /* 256 x 128 on 8 waves, 64-k stages: each generated C~ entry serves 256 rows */
#define SVDU_TILE_SHAPES 6
#define SVDU_TILE_BUCKETS 8      /* tuning-table buckets by order N: (0,64], (64,128], ..., (4096, inf) */

/* ---- contexts ---------------------------------------------------------------
 * The interface of Section 6.1 (input A = U Sigma V^T, a, b; output U^,
 * Sigma^, V^) is svdu_rank1_update below; the context carries what stays the
 * same between such calls. */
typedef struct svdu_ctx svdu_ctx;

/* Creates a context for HIP device `device` (>= 0) with the default options
 * (secular cap 200, refinement on, grid schedule, tile shapes from the
 * built-in tables, timing off). It allocates host memory only. Returns
 * SVDU_OK (*ctx set), SVDU_EINVAL or SVDU_ENOMEM (*ctx = NULL). */
int svdu_create(svdu_ctx** ctx, int device);

/* Frees a context (NULL: nothing). Work already enqueued with it is not
 * affected; batches created with it must be destroyed first (they record
 * their eager launches in its timing ring). */
void svdu_destroy(svdu_ctx* ctx);

/* Sets option `option` (SVDU_OPT_*) of `ctx`; returns the previous value, or
 * SVDU_EINVAL. A change applies to the calls enqueued after it; a batch or
 * server keeps the options its context had when it was created. */
int svdu_set_option(svdu_ctx* ctx, int option, int value);

/* Bytes of device workspace svdu_rank1_update needs for (m, n, path, precision). */
size_t svdu_workspace_bytes(int m, int n, int path, int precision);

/* Rank-1 SVD update (Section 6.1, Steps 1-8).
 *  m, n        1 <= m <= n.
 *  U, ldu      m x m orthogonal, ldu >= m.            (input, not modified)
 *  sigma       m singular values, descending, >= 0.    (input)
 *  V, ldv      n x n orthogonal, ldv >= n.             (input, not modified)
 *  a, b        update vectors of length m and n.       (input)
 *  eps         FMM tolerance (ignored by SVDU_PATH_DIRECT), 0 < eps < 1; the
 *              expansion order is p = ceil(log_5(1/eps)) (Appendix D Step 1),
 *              at least 8. An eps that needs p > 16 (eps < 5^-16, about
 *              6.6e-12) is rejected with SVDU_ENOTSUP.
 *  path        SVDU_PATH_DIRECT or SVDU_PATH_FMM. The FMM path copies the
 *              roots of each level of eigen-updates to the host to build its
 *              trees (the call waits for them, and returns once the second
 *              level's products are enqueued); it runs part of its products
 *              on two more streams of the context, forked from and joined to
 *              `stream` with events. It works with SVDU_PREC_FP64 only.
 *  precision   SVDU_PREC_FP64, SVDU_PREC_SPLIT32 or SVDU_PREC_SLICED_INT8 (the
 *              last two on SVDU_PATH_DIRECT only; SVDU_PREC_SLICED_INT8 for
 *              n <= 32768, above which its INT32 sums could overflow:
 *              SVDU_ENOTSUP).
 *  U_out       m x m, ldu_out >= m: left singular vectors of A^, columns by
 *              descending singular value. Must not overlap U.
 *  sigma_out   m singular values of A^, descending.
 *  V_out       n x n, ldv_out >= n: right singular vectors; column i pairs with
 *              column i of U_out (signs chosen so that U^ S^ V^^T = A^), and
 *              columns m..n-1 span the null space of A^. Must not overlap V.
 *  defl        NULL, or 4*n int8 deflation flags, one row of n per eigen-update
 *              in the order (left, rho+), (left, rho-), (right, rho+),
 *              (right, rho-); entry j of a row describes input column j of that
 *              update (left side: entries m..n-1 are 0): 0 kept, 1 zero
 *              component dropped, 2 merged into an exactly repeated pole.
 *              (Section 3.1 names the deflation cases; code 1 is the case of a
 *              zero component. Poles that are close but distinct are never
 *              merged -- pole-relative roots resolve them -- so no rotation of
 *              a near-equal pair exists; exact repeats, including the n - m
 *              zero poles of the right-hand updates when n > m, all get code 2,
 *              one reflection per repeated group.)
 *  workspace   device buffer of workspace_bytes >= svdu_workspace_bytes(...),
 *              256-byte aligned; it also holds the device status word, so one
 *              workspace serves one call in flight at a time.
 * Returns 0 or a negative SVDU_E* code (see the conventions above). */
int svdu_rank1_update(svdu_ctx* ctx, int m, int n, const double* U, int ldu, const double* sigma, const double* V,
                      int ldv, const double* a, const double* b, double eps, int path, int precision, double* U_out,
                      int ldu_out, double* sigma_out, double* V_out, int ldv_out, int8_t* defl,
                      void* workspace, size_t workspace_bytes, void* stream);

/* ---- rank-k update ---------------------------------------------------------
 * The SVD of A + sum_j a_j b_j^T (j = 0..k-1), the extension the paper's
 * conclusion names, as k rank-1 updates (Section 6.1) applied in order, all
 * enqueued by this one call: update j works on the factors update j - 1
 * produced (each pairs its own signs). No host synchronisation on
 * SVDU_PATH_DIRECT.
 *  A, lda      k x m, row-major: row j is a_j (lda >= m).
 *  B, ldb      k x n, row-major: row j is b_j (ldb >= n).
 *  workspace   >= svdu_rankk_workspace_bytes(m, n, k, path, precision): one
 *              update's workspace plus one intermediate factor set (k > 1).
 *              svdu_get_status(workspace, ...) reports the first device error
 *              of any of the k updates (their status bits combined).
 * Other arguments as for svdu_rank1_update (no deflation flags). Returns 0 or
 * a negative SVDU_E* code; on an argument error found on the host for some
 * update j, updates before j have been enqueued. */
size_t svdu_rankk_workspace_bytes(int m, int n, int k, int path, int precision);
int svdu_rankk_update(svdu_ctx* ctx, int m, int n, int k, const double* U, int ldu, const double* sigma,
                      const double* V, int ldv, const double* A, int lda, const double* B, int ldb, double eps,
                      int path, int precision, double* U_out, int ldu_out, double* sigma_out, double* V_out,
                      int ldv_out, void* workspace, size_t workspace_bytes, void* stream);

/* ---- the update without a caller workspace --------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The same
 * update as svdu_rank1_update on SVDU_PATH_DIRECT (bitwise the same results),
 * with its workspace in a device array of SVDU_NOALLOC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends; the call
 * allocates no device memory. An update whose workspace
 * (svdu_workspace_bytes(m, n, SVDU_PATH_DIRECT, precision)) exceeds the array
 * is refused with SVDU_ENOMEM: the array holds one update up to m = n = 1024
 * in either precision. All calls on one device share that device's array, so
 * calls that overlap on a device (other streams, other threads, other
 * contexts) race; a caller serialises them, e.g. on one stream.
 *  status   NULL, or a device int that receives the call's device status
 *           (SVDU_OK, SVDU_ENONFINITE, SVDU_EBADSIGMA or SVDU_ENOCONV) once
 *           the stream has reached the end of the update.
 * Other arguments as for svdu_rank1_update. Returns 0 or a negative SVDU_E*
 * code found on the host (nothing is enqueued then). */
#define SVDU_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int svdu_rank1_update_noalloc(svdu_ctx* ctx, int m, int n, const double* U, int ldu, const double* sigma,
                              const double* V, int ldv, const double* a, const double* b, int precision,
                              double* U_out, int ldu_out, double* sigma_out, double* V_out, int ldv_out,
                              int8_t* defl, int* status, void* stream);

/* Waits for `stream` and returns the device-side status of the last call that
 * used `workspace`: SVDU_OK, SVDU_ENONFINITE, SVDU_EBADSIGMA or SVDU_ENOCONV
 * (the first that applies, in that order), or SVDU_EHIP. */
int svdu_get_status(const void* workspace, void* stream);

/* Bytes of workspace svdu_eig_update needs for an R x N basis and `path`. */
size_t svdu_eig_update_workspace_bytes(int R, int N, int path);

/* One symmetric rank-one eigen-update (Section 6.2, RankOneUpdate Steps 2-7)
 * of X diag(lam) X^T + rho X z z^T X^T, with the projection z = X^T v already
 * formed (Step 1):
 *  R, N        X is R x N (R >= 0, N >= 1), ldx >= N.
 *  lam         N eigenvalues of the columns of X, ascending.
 *  z           N projected components.
 *  rho         host scalar, nonzero.
 *  path, eps   SVDU_PATH_DIRECT, or SVDU_PATH_FMM with tolerance 0 < eps < 1
 *              (the FMM path synchronises `stream` once to build its tree).
 *  X_out, ldo  R x N, ldo >= N: X C~, columns by ascending new eigenvalue.
 *  lam_out     N new eigenvalues, ascending.
 *  defl        NULL or N int8 flags (as for svdu_rank1_update).
 *  workspace   >= svdu_eig_update_workspace_bytes(R, N, path) bytes. */
int svdu_eig_update(svdu_ctx* ctx, int R, int N, const double* X, int ldx, const double* lam, const double* z,
                    double rho, int path, double eps, double* X_out, int ldo, double* lam_out, int8_t* defl,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Roots of the secular equation w(mu) = 1 + rho sum_k z_k^2 / (d_k - mu)
 * (equation GolubEigenvalUpdate) for K distinct poles d (ascending) and
 * nonzero z, rho nonzero (host scalar). Root i is returned pole-relative:
 * mu_i = d[org[i]] + tau[i], with org[i] the nearer end of its interval.
 * iters (may be NULL) receives the iteration count per root.
 * workspace >= svdu_secular_workspace_bytes(K). */
size_t svdu_secular_workspace_bytes(int K);
int svdu_secular(svdu_ctx* ctx, int K, const double* d, const double* z, double rho, int* org, double* tau,
                 int* iters, void* workspace, size_t workspace_bytes, void* stream);

/* Phase timings recorded in `ctx` while its SVDU_OPT_TIMING is on (at most
 * 256 calls since it was switched on; svdu_rank1_update and eager
 * svdu_batch_launch calls made with the context are recorded). For call c, ms[5 c + k] (host array of 5 max_calls doubles)
 * receives the milliseconds of phase k, measured with HIP events on the
 * call's stream: 0 projections, 1 the O(n^2) eigen-update work of all four
 * updates (deflation, secular roots, weights, signs, singular values), 2 and
 * 3 the products X C~ (direct path: first level U C~_L+ and V C~_R+, then
 * second level U~ C~_L- and V~ C~_R-, with the column rescaling of the
 * precision form; on the FMM path the first level's products partly run
 * beside phase 1, so phase 2 holds what remains of them), 4 the flag copies.
 * Waits for those events. Returns the number of calls filled, or SVDU_EHIP. */
int svdu_timing_read(svdu_ctx* ctx, double* ms, int max_calls);

/* ---- batched updates (many independent problems of uneven sizes) ----------
 * Every step of the update is one launch over all problems of the batch (a
 * product launch per tile shape in use); a problem's results are bitwise the
 * same as from svdu_rank1_update with the same inputs, whatever else is in
 * the batch. Direct path only (any SVDU_PREC_*). */
typedef struct {
  int m, n;                       /* 1 <= m <= n */
  const double* U; int ldu;       /* as for svdu_rank1_update (device pointers) */
  const double* sigma;
  const double* V; int ldv;
  const double* a;
  const double* b;
  double* U_out; int ldu_out;
  double* sigma_out;
  double* V_out; int ldv_out;
  int8_t* defl;                   /* NULL or 4 x n flags */
} svdu_problem;

typedef struct svdu_batch svdu_batch;   /* opaque; owns host-side tables, a graph, an event */

#define SVDU_BATCH_PERSISTENT 1  /* product kernels run as many blocks as fit on the device at once, each
                                    taking tiles (largest problems first) from a counter */

/* Workspace bytes for the batch `probs` (host array of `count`). */
size_t svdu_batch_workspace_bytes(int count, const svdu_problem* probs, int precision);

/* Validates every problem (as svdu_rank1_update does) and that no output
 * overlaps another output, an input or the workspace; carves the workspace;
 * builds the job tables (ordered largest first), and enqueues their upload on
 * `stream`. The problem array may be freed on return; the buffers it names
 * and the workspace must stay valid until svdu_batch_destroy. flags: 0 or
 * SVDU_BATCH_PERSISTENT. The batch keeps a copy of the options of `ctx`
 * (tile shapes, secular cap, refinement) and records its eager launches in
 * the context's timing ring, so `ctx` must outlive it. Returns 0 or a
 * negative SVDU_E* code (*out = NULL). */
int svdu_batch_create(svdu_ctx* ctx, svdu_batch** out, int count, const svdu_problem* probs, int precision,
                      int flags, void* workspace, size_t workspace_bytes, void* stream);

/* Enqueues one update of every problem on `stream` (it may differ from the
 * creation stream; the table upload is waited for). use_graph = 0: the
 * launches are enqueued one by one. use_graph = 1: the first call captures
 * the whole sequence into a HIP graph (on a stream the batch owns) and every
 * call launches that graph once. Inputs may change between launches; sizes,
 * pointers and the workspace may not. One launch in flight per batch. */
int svdu_batch_launch(svdu_batch* b, int use_graph, void* stream);

/* Waits for `stream` and writes each problem's device status (SVDU_OK,
 * SVDU_ENONFINITE, SVDU_EBADSIGMA or SVDU_ENOCONV) to status[0..count-1]
 * (host). Returns the first nonzero one, SVDU_OK, or SVDU_EHIP. */
int svdu_batch_status(svdu_batch* b, int* status, void* stream);

/* Waits for the table upload and frees the batch (not the workspace). */
void svdu_batch_destroy(svdu_batch* b);

/* create + eager launch + wait for `stream` + destroy (persistent schedule
 * when the context's SVDU_OPT_PERSISTENT is set). */
int svdu_rank1_update_batched(svdu_ctx* ctx, int count, const svdu_problem* probs, int precision, void* workspace,
                              size_t workspace_bytes, void* stream);

/* ---- tile-shape autotuner --------------------------------------------------
 * For each size bucket up to max_n (<= 8192 recommended), times the product
 * kernel of every tile shape on the same set of synthetic products of four
 * orders spread over the bucket (up to its upper end, or max_n), each as many
 * times as make 1024 tiles of 128 x 128 (4096 in all, 16 per compute unit, so
 * every shape runs on a full device), and stores the
 * fastest shape in the table of `ctx` used by every later call of that
 * precision made with it. times_ms (host, SVDU_TILE_BUCKETS x SVDU_TILE_SHAPES, may be NULL) receives the
 * best of three timed launches per shape (-1 for buckets above max_n), table
 * (host, SVDU_TILE_BUCKETS, may be NULL) the chosen shapes. Synchronises
 * `stream`. */
size_t svdu_autotune_workspace_bytes(int max_n);
int svdu_autotune(svdu_ctx* ctx, int precision, int max_n, double* times_ms, int* table, void* workspace,
                  size_t workspace_bytes, void* stream);
/* Reads (set = 0) or writes (set = 1) the tuning table of a precision in
 * `ctx` (host array of SVDU_TILE_BUCKETS shapes). */
int svdu_tile_table(svdu_ctx* ctx, int precision, int* table, int set);

/* ---- serving runtime (resident matrices, memory admission, continuous batching)
 * The server holds matrices registered with two buffer sets each (U m x m,
 * sigma m, V n x n, row-major with ld = m and n; device memory owned by the
 * caller): an update reads the current set and writes the other, which then
 * becomes current. Requests name a matrix, device vectors a (m) and b (n),
 * which must stay valid until the request completes, and a release time on
 * the server clock (svdu_server_now; a request is not started before it).
 * `workers` threads, each with its own stream, form batches continuously:
 * the oldest released request whose matrix is idle, plus further released
 * requests, oldest first, at most one per matrix, each costing between
 * min_cost_ratio times the first's and the first's, while the batch's
 * product flops stay within
 * max(batch_cost_factor x the first's, min_batch_cost) and its workspace fits
 * in the largest free block of the caller's arena (memory admission; a
 * request that cannot fit even in an empty arena completes with
 * SVDU_ENOMEM). Updates of one matrix run in release order; each result
 * is bitwise the one svdu_rank1_update gives for the same inputs on the same
 * path. Requests for matrices of order >= fmm_min_n (if > 0, FP64 only) run
 * alone through the FMM path with tolerance fmm_eps. */
typedef struct {
  int workers;                 /* 1..8 batches in flight */
  int max_batch;               /* updates per batch at most */
  int precision;               /* SVDU_PREC_FP64, SVDU_PREC_SPLIT32 or SVDU_PREC_SLICED_INT8 */
  int fmm_min_n;
  double fmm_eps;
  double batch_cost_factor;    /* >= 1 */
  double min_batch_cost;       /* flops, >= 0 */
  double min_cost_ratio;       /* 0..1: smaller requests do not join a batch (they go to another worker) */
} svdu_server_config;

typedef struct {
  long long id;                /* as returned by svdu_server_submit */
  int matrix;
  int status;                  /* SVDU_OK or an SVDU_E* code of the update */
  int batch;                   /* updates in the batch it ran in */
  double t_release, t_start, t_done;   /* server clock, seconds */
} svdu_completion;

typedef struct svdu_server svdu_server;

/* arena: device memory of arena_bytes (>= 1 MiB, 256-byte aligned) that the
 * server carves its workspaces from; it allocates no device memory itself.
 * The server runs on the device of `ctx` with a copy of its options taken
 * here: later changes to `ctx` do not reach the server, and `ctx` may be
 * destroyed while the server runs. */
int svdu_server_create(svdu_ctx* ctx, svdu_server** out, const svdu_server_config* cfg, void* arena,
                       size_t arena_bytes);
/* Registers a matrix (before svdu_server_start); *id receives its index. */
int svdu_server_add_matrix(svdu_server* s, int m, int n, double* U0, double* sigma0, double* V0, double* U1,
                           double* sigma1, double* V1, int* id);
/* Starts the worker threads and resets the server clock to 0. */
int svdu_server_start(svdu_server* s);
/* Seconds since svdu_server_start (or create). */
double svdu_server_now(svdu_server* s);
/* Queues an update of `matrix` released at t_release; *req_id (may be NULL)
 * receives its id. */
int svdu_server_submit(svdu_server* s, int matrix, const double* a, const double* b, double t_release,
                       long long* req_id);
/* Moves up to max_out completions (host array) out of the server; returns
 * their number. */
int svdu_server_poll(svdu_server* s, svdu_completion* out, int max_out);
/* stats (host, 6): queued requests, batches running, batches run, updates
 * run, largest free arena block (bytes), first runtime error (0 if none). */
int svdu_server_stats(svdu_server* s, long long* stats);
/* Waits until nothing is queued or running, or timeout_s passes
 * (SVDU_ENOCONV); returns the first runtime error or SVDU_OK. */
int svdu_server_drain(svdu_server* s, double timeout_s);
/* Current factors of an idle matrix (SVDU_EINVAL while it is being updated). */
int svdu_server_current(svdu_server* s, int matrix, double** U, double** sigma, double** V);
/* Stops the workers after the batches they are running (queued requests are
 * dropped) and frees the server (not the arena or the matrices). */
void svdu_server_destroy(svdu_server* s);

/* Static description of a status code (host). */
const char* svdu_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* SVDU_H */
