/*
 * libspca -- alternating maximization (AM) for single-loading-vector sparse
 * PCA on AMD Instinct MI355X (gfx950).
 *
 * The method is Algorithm 2 of Richtarik, Jahani, Ahipasaoglu and Takac,
 * "Alternating maximization: unifying framework for 8 sparse PCA
 * formulations and efficient parallel codes" (arXiv:1212.4137), run from r
 * starting points at once (the batched scheme of Section 4, where the r
 * matrix-vector products of an iteration form one matrix product).
 *
 * Conventions shared by every entry point
 *   - A is n x p, column-major with leading dimension lda >= n (column a_i
 *     contiguous, Section 1: n samples of p variables), FP32, in device
 *     memory.  The library never writes to it.
 *   - Starting points X0 are r x p, start-major: row j (p contiguous floats)
 *     is x^(0) of start j, in device memory.
 *   - Every buffer passed in is owned by the caller and must stay valid until
 *     the call returns.  The library owns its workspace (inside spca_ctx).
 *   - Return value: SPCA_OK (0) or a negative SPCA_E* code; the message of
 *     the last failure on the calling thread is spca_last_error().  No C++
 *     exception crosses this boundary.  Argument checks happen before any
 *     device work.
 *   - Calls are synchronous with respect to the stream they are given.
 */
#ifndef SPCA_H
#define SPCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Formulations, numbered as in Table 1 (variance norm x sparsity norm x
 * constraint or penalty).  The parameter s_or_gamma is the sparsity level s
 * for 1-4 (L0: ||x||_0 <= s, s integral in [1, p]; L1: ||x||_1 <= sqrt(s),
 * real s >= 1) and the penalty weight gamma >= 0 for 5-8.                  */
enum {
  SPCA_L2_L0_CON = 1, /* max ||Ax||_2   s.t. ||x||_2 <= 1, ||x||_0 <= s    */
  SPCA_L1_L0_CON = 2, /* max ||Ax||_1   s.t. ||x||_2 <= 1, ||x||_0 <= s    */
  SPCA_L2_L1_CON = 3, /* max ||Ax||_2   s.t. ||x||_2 <= 1, ||x||_1 <= vs   */
  SPCA_L1_L1_CON = 4, /* max ||Ax||_1   s.t. ||x||_2 <= 1, ||x||_1 <= vs   */
  SPCA_L2_L0_PEN = 5, /* max ||Ax||_2^2 - gamma ||x||_0, ||x||_2 <= 1     */
  SPCA_L1_L0_PEN = 6, /* max ||Ax||_1^2 - gamma ||x||_0, ||x||_2 <= 1     */
  SPCA_L2_L1_PEN = 7, /* max ||Ax||_2   - gamma ||x||_1, ||x||_2 <= 1     */
  SPCA_L1_L1_PEN = 8  /* max ||Ax||_1   - gamma ||x||_1, ||x||_2 <= 1     */
};

/* Return codes */
#define SPCA_OK 0
#define SPCA_EINVAL (-1) /* bad argument (nothing was launched)            */
#define SPCA_ENOMEM (-2) /* workspace would exceed the context's budget    */
#define SPCA_EHIP (-3)   /* a HIP runtime call failed                      */

/* Per-start status (and spca_result.status of the best start) */
#define SPCA_CONVERGED 0  /* phi_k <= (1 + tol) phi_{k-1} (Section 2.2)     */
#define SPCA_MAXIT 1      /* maxit x-updates without meeting the stop test  */
#define SPCA_DEGENERATE 2 /* A x = 0 (excluded by Theorem 1): x = 0, f = 0  */
#define SPCA_ZERO 3       /* the x-operator returned 0: x = 0, f = 0         */

/* spca_result.warning: a property of the whole solve (all its starts), 0 or
 * positive; the solve itself succeeded (return code SPCA_OK) */
#define SPCA_WARN_NONE 0
#define SPCA_WARN_ALL_DEGENERATE 1 /* every start ended DEGENERATE (A x = 0) */
#define SPCA_WARN_ALL_ZERO 2       /* every start ended DEGENERATE or ZERO,
                                      at least one ZERO: x_out is 0, f = 0   */
#define SPCA_WARN_NO_CONVERGED 3   /* tol >= 0 and no start met the stop test
                                      within maxit (some ended MAXIT)        */

/* Arithmetic of the iterations */
#define SPCA_PREC_FP32 0        /* A, X, Y in FP32, FP32 MFMA accumulation   */
#define SPCA_PREC_BF16_POLISH 1 /* A, X, Y operands in BF16, FP32 accumulation,
                                   then up to polish_maxit FP32 AM iterations
                                   on the caller's FP32 A ("polish"): every
                                   start continues from its BF16-phase
                                   iterate for up to 4 iterations, then the
                                   16 best still-running ones to the end;
                                   the per-start results and the best start
                                   are those after the polish; objective and
                                   explained variance in FP64 on the FP32 A */

typedef struct {
  double objective;      /* f(x) of Table 1 at the returned x, FP64         */
  double explained_var;  /* ||Ax||_2^2 (L2 variance) or ||Ax||_1 (L1), FP64 */
  double phi;            /* last in-loop phi of the best start (Table 3)    */
  double iters_x_starts; /* AM iterations summed over all starts            */
  int32_t best_start;    /* index of the start with the largest objective   */
  int32_t nnz;           /* |support|                                       */
  int32_t iters;         /* x-updates done by the best start                */
  int32_t status;        /* SPCA_CONVERGED .. SPCA_ZERO of the best start   */
  double objective_pre_polish; /* BF16 mode: f before the FP32 polish
                                  (FP64, on the FP32 A) of the start whose
                                  BF16-phase in-loop objective phi is the
                                  largest; equal to objective otherwise     */
  int32_t polish_iters;  /* FP32 polish iterations of the best start (BF16) */
  int32_t warning;       /* SPCA_WARN_* over all starts of the solve        */
} spca_result;

/* ---------------------------------------------------------------------- */
/* One-call solve (Algorithm 2 from r starts, Section 4; best start kept).
 *
 * A        device, FP32, n x p column-major, lda >= n.
 * formulation 1..8 (Table 1); s_or_gamma as described above.
 * X0       device, FP32, r x p start-major; or NULL with r == 1, which starts
 *          from x0 = e_i for the column i of A with the largest 2-norm (ties
 *          to the lowest i), so that y0 is that column normalised.
 * tol      stop test phi_k <= (1 + tol) phi_{k-1}; tol < 0 disables it.
 * maxit    >= 1, maximum number of x-updates per start.
 * x_out    host, p doubles: the loading vector of the best start, normalised
 *          in FP64 (or all zero if every start ended DEGENERATE or ZERO).
 * support_out host, capacity p int32: the sorted indices of the nonzeros of
 *          x_out; res->nnz of them are written.
 * res      host.
 * Uses a per-device default context and the null stream.
 * Errors: SPCA_EINVAL if n, p or r < 1, lda < n, formulation outside 1..8,
 * s outside [1, p] (L0 constraint) or < 1 (L1 constraint), gamma < 0 or not
 * finite, maxit < 1, a NULL pointer, X0 NULL with r != 1.                  */
int spca_am_solve(const float* A, int64_t n, int64_t p, int64_t lda,
                  int formulation, double s_or_gamma, const float* X0,
                  int32_t r, double tol, int32_t maxit, double* x_out,
                  int32_t* support_out, spca_result* res);

/* ---------------------------------------------------------------------- */
/* Context: device binding, workspace and HBM budget.                      */
typedef struct spca_ctx spca_ctx;

/* device: HIP device ordinal.  hbm_budget_bytes: upper bound on the
 * workspace the context may hold (0 = no limit beyond the device).       */
int spca_ctx_create(spca_ctx** ctx, int device, size_t hbm_budget_bytes);
int spca_ctx_destroy(spca_ctx* ctx);
/* Bytes of workspace a solve of this shape needs (for admission control);
 * with SPCA_PREC_BF16_POLISH it includes the FP32 polish sub-solve.       */
size_t spca_workspace_bytes(int64_t n, int64_t p, int32_t r, int precision);
/* Makes the context use caller-owned device memory (256-byte aligned) as its
 * workspace instead of allocating its own; a solve that needs more than
 * `bytes` then fails with SPCA_ENOMEM.  NULL / 0 returns the context to
 * allocating.  The memory must stay valid while solves run on the context;
 * the context never frees it.                                              */
int spca_ctx_set_workspace(spca_ctx* ctx, void* dev_ptr, size_t bytes);

typedef struct {
  const float* A; /* device, FP32, n x p column-major                        */
  int64_t n, p, lda;
  int32_t formulation;
  double s_or_gamma;
} spca_problem;

typedef struct {
  const float* X0;      /* device r x p start-major, or NULL (needs r == 1) */
  int32_t r;
  double tol;
  int32_t maxit;
  int32_t precision;    /* SPCA_PREC_FP32 or SPCA_PREC_BF16_POLISH          */
  int32_t polish_maxit; /* FP32 iterations on the final support (BF16 mode) */
  int32_t check_every;  /* iterations between polls of the active count     */
  int32_t flags;        /* SPCA_FLAG_* below                                */
  /* On-the-fly replacement (Section 4.3): 0 or r runs the r starts of X0
   * together.  A value l > r makes X0 hold l starts that flow through r
   * slots: whenever a start stops, it is evaluated and the next start takes
   * its slot, until all l have run (each for at most maxit iterations).
   * Per-start outputs then have l entries, and X_final (when set) holds l
   * rows: the final iterate of each start, filed as it finishes; FP32 only.
   * The workspace grows by about 40 bytes per start beyond
   * spca_workspace_bytes(n, p, r, ...) plus 4p bytes.                    */
  int32_t total_starts;
  /* Sparsity-targeted warm-up (the experiments of Section 4.1): during the
   * first warmup_iters x-updates the parameter follows v and is then frozen
   * per start.  L1 constraint (formulations 3, 4): lambda = lambda_s(v),
   * then fixed.  Penalties (5..8): gamma = the (target_nnz + 1)-th largest
   * v_i^2 (L0 penalty) or |v_i| (L1 penalty), so that target_nnz entries
   * pass the strict threshold (ties aside), then fixed; s_or_gamma is
   * unused.  The stop test applies once the parameter is frozen; with
   * per-start gamma the best start is the one with the largest explained
   * variance.  0 disables it.  FP32 only, not with total_starts > r.      */
  int32_t warmup_iters;
  int32_t target_nnz;   /* penalties under warm-up: 1..p                    */
  /* Deflation for a further component: the solve works on
   * A (I - x_1 x_1^T) ... (I - x_k x_k^T) for the deflate_k loadings in
   * deflate_X (device, deflate_k x p, FP64, unit norm, in the order they
   * were found), applied implicitly.  0..16 loadings; FP32 only, not with
   * total_starts > r.  f and the explained variance are those of the
   * deflated matrix.                                                       */
  const double* deflate_X;
  int32_t deflate_k;
} spca_solve_opts;

/* SPCA_FLAG_GRAPH: capture check_every iterations once per solve into a HIP
 * graph (on a stream of the context) and replay it on the caller's stream
 * between stop-test polls; the leftover maxit % check_every iterations run
 * eagerly.  Results are identical to the eager path.  Ignored when
 * kernel_times is requested.                                               */
#define SPCA_FLAG_GRAPH 1
#define SPCA_FLAG_CHECK_FINITE 2 /* reject A holding NaN or Inf (EINVAL)     */
#define SPCA_FLAG_DENSE_ONLY 4   /* never use the sparse A x product         */
/* SPCA_FLAG_AUTOTUNE: before iterating, time every compiled tile shape and
 * K split of the two products on this solve's own operands (products whose
 * size bucket already has a tuning-table entry are skipped) and record the
 * fastest in the process-wide tuning table, which later plans use.  A
 * product's result depends on its K split, so tuned solves are
 * reproducible given the table (see spca_tune_table_export).              */
#define SPCA_FLAG_AUTOTUNE 8
/* SPCA_FLAG_NO_UNION: never use the union-of-supports product; its gather
 * and product kernels are then not launched at all (each launch that a
 * solve's planner gates off still costs a few microseconds).  Without it a
 * solve launches them while its planner picks the union product or finds it
 * within 1.25x of the best product at its latest probe, checked at each
 * poll.                                                                    */
#define SPCA_FLAG_NO_UNION 16
/* Sparse solve only: A^T Y reads a copy of the columns split into row
 * panels (one panel's rows per XCD at a time, so that the gathered rows of
 * Y stay in that XCD's L2), built at the start of each solve.  By default
 * the solve uses panels when Y is larger than one L2 and A has at least
 * 2^20 nonzeros; these flags force them on or off.  Results differ from
 * the unpanelled product only in the order of the sums.                   */
#define SPCA_FLAG_SPARSE_PANELS 32
#define SPCA_FLAG_SPARSE_NO_PANELS 64
/* SPCA_FLAG_TIME_SAMPLED: with kernel_times, record the HIP events only
 * around the launches of every 8th iteration (iterations 0, 8, 16, ...);
 * each event pair costs the stream a few microseconds, so timing every
 * launch slows a long solve measurably.  The times and launch counts in
 * kernel_times are then those of the sampled launches.                    */
#define SPCA_FLAG_TIME_SAMPLED 128

typedef struct {
  double* x;           /* host, p doubles (see spca_am_solve), or NULL      */
  int32_t* support;    /* host, capacity p, or NULL                         */
  spca_result* res;    /* host, required                                    */
  /* optional host arrays of length r (NULL to skip)                        */
  double* f_per_start;     /* f(x_j) of Table 1, FP64                       */
  double* ev_per_start;    /* explained variance of x_j, FP64               */
  double* phi_per_start;   /* last in-loop phi                              */
  int32_t* iters_per_start;
  int32_t* status_per_start;
  int32_t* nnz_per_start;
  float* X_final;      /* optional device r x p (l x p with total_starts > r):
                          final iterates (FP32; with SPCA_PREC_BF16_POLISH
                          those of the BF16 phase, before the polish)      */
  /* optional host array of 12 doubles: HIP-event times of the launches of
   * this solve, [0] total ms and [1] count of the V = A^T Y products,
   * [2] ms and [3] count of the x-updates, [4] ms and [5] count of the
   * dense U = A X products (including launches that found another product
   * selected and returned at once); [6], [7], [8] the iterations whose A x
   * used the dense product, the per-start lists (both list kernels), and
   * the product over the union of the supports; [9] of the list
   * iterations, those that used the row-block list kernel; [10] the
   * running starts summed over iterations (the A^T Y work is 2 n p per
   * unit) and [11] the nonzeros of the iterates that entered A x, summed
   * over iterations and starts (the algorithmic A x work is 2 n per unit).
   * NULL disables the events.                                              */
  double* kernel_times;
  /* optional host array (per start): the final lambda (formulations 3, 4)
   * or gamma (5..8) of each start under the warm-up; untouched otherwise */
  double* param_per_start;
} spca_outputs;

/* Several components, one after another: component c is the solve of
 * (prob, opts) on A deflated by the loadings of components 0..c-1 (the
 * paper's deflation, read as projection deflation of the data matrix), from
 * the same starts.  X_out: host ncomp x p FP64 (the loadings); res: host
 * ncomp results.  opts->deflate_X / deflate_k must be unset (NULL / 0);
 * 1 <= ncomp <= 16.  Allocates and frees a small device buffer for the
 * loadings and synchronizes the stream.                                   */
int spca_am_components(spca_ctx* ctx, void* stream, const spca_problem* prob,
                       const spca_solve_opts* opts, int32_t ncomp, double* X_out,
                       spca_result* res);

/* Sparse A (the paper's text corpora are word-count matrices): the same
 * batched solve with A held as compressed sparse columns and, for the
 * product with a dense iterate, compressed sparse rows of the same matrix.
 * All arrays are device memory owned by the caller, 16-byte aligned:
 * col_ptr (p + 1 int64), row_idx / col_val (nnz, rows strictly ascending
 * within a column), row_ptr (n + 1 int64), col_idx / row_val (nnz).  Both
 * pointer arrays start at 0 and end at the same nnz.  Options as
 * spca_am_solve_ex, with X0 required, FP32 only and no total_starts > r;
 * deflate_X / deflate_k as there (the scores A x_i are formed from the
 * columns in FP64).  The solve first checks the arrays on
 * the device (pointer arrays non-decreasing, every index in range, rows of
 * a column strictly ascending; SPCA_EINVAL otherwise, before any product
 * runs), synchronizing the stream; it synchronizes again when it builds row
 * panels (see SPCA_FLAG_SPARSE_PANELS).  The workspace holds, besides the
 * iterates, the transposed operands and, with panels, a copy of the
 * columns (8 bytes per nonzero).                                          */
typedef struct {
  int64_t n, p;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const float* col_val;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const float* row_val;
  int32_t formulation;
  double s_or_gamma;
} spca_sparse_problem;

int spca_am_solve_sparse(spca_ctx* ctx, void* stream, const spca_sparse_problem* prob,
                         const spca_solve_opts* opts, spca_outputs* out);

/* Further components on a sparse A: the component loop of
 * spca_am_components over spca_am_solve_sparse (deflate_X / deflate_k
 * unset in opts; 1 <= ncomp <= 16; same outputs and synchronization).     */
int spca_am_components_sparse(spca_ctx* ctx, void* stream, const spca_sparse_problem* prob,
                              const spca_solve_opts* opts, int32_t ncomp, double* X_out,
                              spca_result* res);

/* Full solve on a caller-chosen context and HIP stream (hipStream_t passed
 * as void*; NULL = null stream).  Same semantics as spca_am_solve.
 * Additional errors: SPCA_ENOMEM when the workspace exceeds the budget;
 * SPCA_EINVAL for precision outside {0, 1}, check_every < 1 and, with
 * SPCA_FLAG_CHECK_FINITE, a non-finite entry of A.                         */
int spca_am_solve_ex(spca_ctx* ctx, void* stream, const spca_problem* prob,
                     const spca_solve_opts* opts, spca_outputs* out);

/* Grouped solve: `count` independent requests (probs[q], opts[q],
 * outs[q]; each its own A, formulation, parameter, starts, tol and maxit)
 * iterated together, so that every kernel launch of an AM iteration
 * (Algorithm 2, from every start of every request, Section 4) covers the
 * starts of all of them.  Meant for requests too small to fill the GPU,
 * whose cost is the launch count: products are always dense, with a K split
 * that follows from each request's own n and p, and the iteration runs
 * until every start of every request has stopped.  A request's results are
 * bit-identical alone (count = 1) and in any group; they are those of
 * spca_am_solve up to the order of the sums in the products.
 * Restrictions (SPCA_EINVAL, the message names the request): FP32
 * precision, no total_starts > r, warm-up or deflation; p at most
 * SPCA_GROUP_MAX_P (the register-resident x-update); at most
 * SPCA_GROUP_MAX_REQUESTS requests and SPCA_GROUP_MAX_STARTS starts in all;
 * each request is checked as in spca_am_solve_ex.  Flags are ignored; the
 * host polls every min(check_every) iterations.  outs[q] as in
 * spca_am_solve_ex (kernel_times and param_per_start are not written).
 * Workspace: spca_group_workspace_bytes of the same arguments, taken from
 * ctx (SPCA_ENOMEM beyond its budget).  Synchronizes the stream.          */
#define SPCA_GROUP_MAX_REQUESTS 1024
#define SPCA_GROUP_MAX_P 12288
#define SPCA_GROUP_MAX_STARTS 65536
size_t spca_group_workspace_bytes(int32_t count, const spca_problem* probs,
                                  const spca_solve_opts* opts);
int spca_am_solve_group(spca_ctx* ctx, void* stream, int32_t count, const spca_problem* probs,
                        const spca_solve_opts* opts, spca_outputs* outs);

/* Thread-local message of the last failure ("" if none).                 */
const char* spca_last_error(void);

/* ---------------------------------------------------------------------- */
/* Building blocks of one AM iteration, exported for testing and tuning.   */

/* C = P * Q^T in FP32 with FP32 MFMA accumulation (the two products of an
 * AM iteration, Section 4: U^T = X^T A^T and V^T = Y^T A).  P is M x K,
 * Q is N x K, C is M x N, all row-major in device memory with leading
 * dimensions ldp, ldq >= K and ldc >= N.  ldp and ldq must be multiples of
 * 4 and P, Q 16-byte aligned (SPCA_EINVAL otherwise).                    */
int spca_gemm_nt_f32(void* stream, const float* P, int64_t ldp, const float* Q,
                     int64_t ldq, float* C, int64_t ldc, int64_t M, int64_t N,
                     int64_t K);

/* The same product with BF16 operands (raw bfloat16 bit patterns), FP32
 * accumulation and FP32 output (the products of the SPCA_PREC_BF16_POLISH
 * iterations).  ldp and ldq must be multiples of 8, P and Q 16-byte
 * aligned.                                                                */
int spca_gemm_nt_bf16(void* stream, const uint16_t* P, int64_t ldp,
                      const uint16_t* Q, int64_t ldq, float* C, int64_t ldc,
                      int64_t M, int64_t N, int64_t K);
/* The BF16 product with a given tile shape and K split, as
 * spca_gemm_nt_f32_shape (C holds `splits` partial products).             */
int spca_gemm_nt_bf16_shape(void* stream, const uint16_t* P, int64_t ldp,
                            const uint16_t* Q, int64_t ldq, float* C, int64_t ldc,
                            int64_t M, int64_t N, int64_t K, int shape, int splits);

/* Tuning and testing variant of spca_gemm_nt_f32 with a forced tile shape
 * (0 .. 8: BMxBN of 128x128, 128x160, 128x96, 128x64, 64x128, 32x128,
 * 64x256, 256x128, 256x256) and
 * K split count (1 .. 64).  With splits > 1, C must hold splits x M rows:
 * split s writes its partial product (K slabs s*ceil(K/32/splits) onward)
 * at C + s * M * ldc, and the product is the sum of the partials.       */
int spca_gemm_nt_f32_shape(void* stream, const float* P, int64_t ldp,
                           const float* Q, int64_t ldq, float* C, int64_t ldc,
                           int64_t M, int64_t N, int64_t K, int shape,
                           int splits);

/* The tile shape and K split the library picks for an M x N x K product
 * (deterministic, from a model of CU occupancy and tile efficiency).     */
/* Tuning table of the product tiles: one line per entry,
 *   "elem_bytes max_splits bucket(M) bucket(N) bucket(K) shape splits"
 * with bucket(x) = round(2 log2 x).  Export writes the table as text into
 * buf (cap bytes, NUL-terminated; *len = its length, also when buf is NULL
 * or too small, in which case EINVAL is returned for the too-small buffer);
 * import adds (or replaces) entries from such text (EINVAL on a malformed
 * line, and then nothing is imported); clear removes every entry.  Plans
 * (spca_gemm_nt_f32_plan and the solves) use an entry of their bucket
 * before the cost model.  Host-only: no device is touched.                */
int spca_tune_table_export(char* buf, size_t cap, size_t* len);
int spca_tune_table_import(const char* text);
int spca_tune_table_clear(void);

int spca_gemm_nt_f32_plan(int64_t M, int64_t N, int64_t K, int max_splits,
                          int* shape, int* splits);

/* The x-update of Algorithm 2 for formulation fid applied to each row of V
 * (r x p row-major, ldv >= p, device): X_j = op(V_j) / ||op(V_j)||_2 with op
 * T_s, V_{lambda_s}, U_gamma or V_gamma (Table 3, rows S3-S6).  Writes X
 * (r x p, ldx >= p, device), phi (r doubles, device: the subproblem optimum
 * of Table 3) and nnz (r int32, device).  A zero image gives X_j = 0.
 * Same parameter checks as spca_am_solve.  For p > 12288 (except the L1
 * constraint) the chunked kernels run on scratch that this call allocates
 * and frees, so the call then synchronizes the stream before returning.   */
int spca_x_update(void* stream, int formulation, const float* V, int64_t ldv,
                  int64_t r, int64_t p, double s_or_gamma, float* X,
                  int64_t ldx, double* phi, int32_t* nnz);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid allocation): spca_x_update with the
 * same arguments, checks and results, whose chunked kernels (rows longer
 * than 12288) take their scratch from a fixed array of
 * SPCA_X_UPDATE_NOALLOC_SCRATCH bytes that every device the library runs
 * on holds until the process ends, instead of allocating it.  The call
 * neither allocates, frees nor synchronizes: it enqueues kernels on the
 * stream and returns.  SPCA_EINVAL (nothing launched) when r rows of
 * length p need more scratch than that (about 19 KB per row at p = 200000;
 * split the rows into batches).  Every call on one device shares that
 * device's array: calls that overlap in time on one device (different
 * streams, or host threads) race and must be serialized by the caller.
 * The call clears what must start at zero itself.  The first call on a
 * device looks up the array's address there (a one-time set-up).        */
#define SPCA_X_UPDATE_NOALLOC_SCRATCH (64ull << 20)
int spca_x_update_noalloc(void* stream, int formulation, const float* V,
                          int64_t ldv, int64_t r, int64_t p, double s_or_gamma,
                          float* X, int64_t ldx, double* phi, int32_t* nnz);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of independent solves on one GPU.         */

/* One request.  A is either the caller's (device, column-major, lda >= n,
 * kept valid until the request completes) or, with A == NULL, generated in
 * the server's memory by spca_generate_spiked(seed, n, p, k, thetas, U, V).
 * The r starts are always generated: row j of X0 is column j of the
 * generator's p x r noise matrix for start_seed (the AM iteration does not
 * depend on the scale of a start).  For penalties, gamma_rel > 0 sets
 * gamma = gamma_rel * max_i ||a_i||_2 (computed on the device); otherwise
 * s_or_gamma is used as given.  Host arrays (thetas, U, V) are copied at
 * submission; x_out and support_out (host, p entries, or NULL) are written
 * before the completion is posted and must stay valid until then.         */
typedef struct {
  const float* A;
  int64_t n, p, lda;
  uint64_t seed;
  int32_t k;
  int32_t formulation;
  const double* thetas; /* k values */
  const double* U;      /* n x k, column-major */
  const double* V;      /* p x k, column-major */
  uint64_t start_seed;
  double s_or_gamma;
  double gamma_rel;
  int32_t r;
  int32_t maxit;
  double tol;
  int32_t precision;
  int32_t polish_maxit;
  int32_t check_every;  /* 0: 8 */
  int32_t flags;        /* SPCA_FLAG_* */
  double* x_out;
  int32_t* support_out;
} spca_request;

typedef struct {
  int64_t id;
  int32_t rc;           /* SPCA_OK or the solve's error code */
  int32_t reserved;
  spca_result res;
  double s_or_gamma;    /* the parameter the solve used */
  double t_submit;      /* seconds on the monotonic clock: submission,  */
  double t_admit;       /* admission (memory and worker granted),       */
  double t_solve;       /* inputs generated, solve starts,              */
  double t_done;        /* result written                               */
  size_t footprint;     /* bytes of the server arena the request held */
  char error[160];      /* message when rc != SPCA_OK */
} spca_completion;

typedef struct {
  size_t arena_bytes, in_use_bytes, peak_in_use_bytes;
  int64_t queued;
  int32_t running, peak_running;
  int64_t completed;
  double now;           /* monotonic clock, seconds */
} spca_server_stats_t;

typedef struct spca_server spca_server;

/* Bytes of server memory a request holds while it runs: its generated A,
 * spike factors, starts and spca_workspace_bytes of the solve (for a
 * request served in groups, see below, the grouped workspace of the request
 * alone; its group's workspace is shared).                                */
size_t spca_request_footprint(const spca_request* req);
/* Allocates an arena of hbm_bytes on the device and starts `workers` worker
 * threads, each with its own stream and context.  Requests are admitted in
 * arrival order when a worker is free and their footprint fits in the free
 * part of the arena (first fit); admitted requests run concurrently.
 * Small requests (FP32, p <= SPCA_GROUP_MAX_P, n p r <= 5.4e8, no flag but
 * SPCA_FLAG_GRAPH, valid arguments) are served in groups: the worker that
 * admits one also admits the small requests queued right behind it (up to
 * 32 requests and 4096 starts, as far as the arena allows) and solves them
 * with spca_am_solve_group; their completions are posted together.  A
 * request's result is the same alone and in any mix.                      */
int spca_server_create(spca_server** srv, int device, size_t hbm_bytes,
                       int32_t workers);
/* Largest number of requests served as one group (default 32); 0 serves
 * every request alone with spca_am_solve_ex, 1 serves small requests alone
 * with spca_am_solve_group.  Only while no request is queued or running
 * (EINVAL otherwise).                                                      */
int spca_server_set_group_limit(spca_server* srv, int32_t max_requests);
/* Queues a request; EINVAL when its footprint exceeds the whole arena. */
int spca_server_submit(spca_server* srv, const spca_request* req, int64_t* id);
/* Moves up to max completions (in completion order) to out; waits up to
 * wait_ms for the first one (0: no wait, < 0: until one arrives).          */
int spca_server_poll(spca_server* srv, spca_completion* out, int32_t max,
                     int32_t* count, int32_t wait_ms);
int spca_server_stats(spca_server* srv, spca_server_stats_t* stats);
/* Finishes every queued request, then stops the workers and frees the
 * arena (completions not yet polled are dropped).                         */
int spca_server_destroy(spca_server* srv);

/* ---------------------------------------------------------------------- */
/* Synthetic data (workload generation, not part of the method).           */

/* Writes the n x p spiked matrix A = G + sum_k theta_k u_k v_k^T into A
 * (device, FP32, column-major, lda >= n).  G[i, j] is a function of
 * (seed, i, j) only: one Philox4x32-10 block (Salmon et al., SC'11) with
 * counter (i, j, 0, 0) and key (seed & 0xffffffff, seed >> 32); with w_q the
 * top 24 bits of its four outputs, G = ((w_0+w_1+w_2+w_3) 2^-24 - 2) sqrt(3)
 * in FP64 (mean 0, variance 1).  The spikes are added in FP64 left to right
 * in k, each term (theta_k U[i,k]) V[j,k], then rounded once to FP32.
 * thetas: host, k values (0 <= k <= 16); U: device FP64 n x k column-major
 * (ldu >= n); V: device FP64 p x k column-major (ldv >= p).  Enqueues on
 * the stream and returns.                                                  */
int spca_generate_spiked(void* stream, uint64_t seed, int64_t n, int64_t p,
                         float* A, int64_t lda, int32_t k, const double* thetas,
                         const double* U, int64_t ldu, const double* V,
                         int64_t ldv);

#ifdef __cplusplus
}
#endif
#endif /* SPCA_H */
