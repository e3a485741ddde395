// Launchers of the HIP kernels that make up one AM iteration.  All take a
// stream and device pointers; none allocates or synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace spca {

// x-operator kinds (Table 3): constraint L0 -> T_s, constraint L1 ->
// V_{lambda_s}, penalty L0 -> U_gamma, penalty L1 -> V_gamma.
enum XKind { kTopS = 0, kLambdaS = 1, kHardGamma = 2, kSoftGamma = 3 };

inline XKind xkind_of(int fid) {
  return fid <= 2 ? kTopS : fid <= 4 ? kLambdaS : fid <= 6 ? kHardGamma : kSoftGamma;
}
inline bool l1_variance(int fid) { return fid % 2 == 0; }

// The most K-split partials of one product that its consumer (the y-update,
// the grouped partial sums) adds up.
constexpr int kSplitsMax = 16;

// Per-start settings of a grouped solve (starts of several requests in one
// set of launches): the request's operator, parameter and stop rule.
struct RowCfg {
  double param;    // s or gamma of the start's request
  double tol;      // its stop tolerance (< 0: off)
  int32_t maxit;   // its iteration limit
  int32_t kind;    // XKind of its formulation
  int32_t l1;      // 1: L1 variance (y = sgn u), 0: L2 (y = u / ||u||)
  int32_t splits;  // K partials of its A x product that the y-update sums
  int32_t aty_splits;  // K partials of its A^T y product
};

// Per-start iteration state, device arrays of length r.
struct StartState {
  double* phi;       // phi after the last x-update (Table 3 optimum)
  double* phi_prev;  // phi after the one before
  int32_t* nnz;      // nonzeros of the current x
  int32_t* iters;    // x-updates done
  int32_t* status;   // kRunning or a SPCA_* status
  // the last x-update's selection threshold (T_s: the s-th largest |v_i|;
  // lambda_s: lambda), 0 when unknown; a starting guess for the next
  // x-update's exact selection (it never changes the result).  May be null.
  float* thr = nullptr;
  // per start, set by the candidate x-update: 1 when the row still needs
  // the full selection kernel, 0 when it was settled.  Null: every row.
  int32_t* redo = nullptr;
  // grouped solves: per-start settings; the x-update kernels then take
  // param, tol and maxit from here and skip the starts of other operator
  // kinds.  Null: the launch arguments hold for every start.
  const RowCfg* cfg = nullptr;
};

// How the next product A x is formed (chosen on the device by the planner):
//   kAxDense  MFMA GEMM over all p columns (split-K partials),
//   kAxList   per-start sums over each start's (index, value) list,
//   kAxUnion  MFMA GEMM over the union of the running starts' supports,
//             with X and A gathered onto those columns.
// kAxList: one workgroup per start, y-update fused; kAxListRows: the same
// product cut into row blocks (many workgroups per start, for few starts),
// followed by the separate y-update
enum AxMode { kAxDense = 0, kAxList = 1, kAxUnion = 2, kAxListRows = 3 };

struct Plan {
  int32_t mode;         // AxMode of the next A x
  int32_t active;       // starts still running
  int32_t union_close;  // the union product was picked, or came within 1.25x of
                        // the best product at the latest probe
  int64_t total_nnz;    // sum of nnz over running starts
  int32_t max_nnz;      // largest nnz over running starts
  int32_t union_size;   // columns used by the running starts (kAxUnion's K)
  int32_t epoch;        // column marks of the current x-update carry this
  int32_t ax_splits;    // K partials the y-update sums (dense mode)
  int32_t mark;         // the next x-update marks its columns
  int32_t iter;         // planner calls so far
  int32_t mode_count[4];  // iterations run in each mode (statistics)
  int32_t last_union;   // most recent measured union size (0: none yet)
  // work counters: summed over planner calls, each of which precedes the
  // iteration it plans (a stopped start is not counted), so they are the
  // sums over iterations of the running starts and of the nonzeros of the
  // iterates that enter A x
  double active_sum;
  double nnz_sum;
};

// Sparsity-targeted warm-up (Section 4.1): during x-updates 1..K the
// parameter follows v (lambda_s(v) for the L1 constraint; for the
// penalties gamma = the (target+1)-th largest v_i^2 or |v_i|, so that target
// entries pass), afterwards it is frozen at gam[j].  K = 0: off.
struct Warm {
  int32_t K = 0;
  int32_t target = 0;
  double* gam = nullptr;  // r: the parameter of each start
};

// Deflation by k previously found loadings (projection deflation of the
// data matrix), applied implicitly: see deflate.hip.
constexpr int kMaxDefl = 16;
struct Defl {
  int k = 0;
  int32_t* idx = nullptr;   // k x p: support of each loading
  double* val = nullptr;    // k x p: its values
  int32_t* cnt = nullptr;   // k: support sizes
  double* gram = nullptr;   // kMaxDefl x kMaxDefl: x_i^T x_l
  double* scores = nullptr; // n x kMaxDefl: A x_i (FP64)
  double* alpha = nullptr;  // r x kMaxDefl: coefficients of the final evaluation
};
size_t deflate_bytes(int64_t n, int64_t p, int64_t r, int k);
Defl carve_deflate(void* base, int64_t n, int64_t p, int64_t r, int k);
// lists and Gram matrix of the loadings Xd (device k x p FP64)
void deflate_loadings(hipStream_t st, const double* Xd, int64_t p, Defl d);
// the same plus the FP64 scores A x_i of a dense column-major A
void deflate_setup(hipStream_t st, const double* Xd, const float* A, int64_t lda,
                   int64_t n, int64_t p, Defl d);
// u -= sum alpha_i A x_i (first partial of U; not in the fused list mode)
void deflate_u(hipStream_t st, const float* X, int64_t ldx, int64_t p, float* U,
               int64_t ldu, int64_t n, int64_t r, StartState s, const Plan* plan, Defl d);
// v -= sum beta_i x_i
void deflate_v(hipStream_t st, float* V, int64_t ldv, int64_t p, int64_t r, StartState s,
               Defl d);
// alpha of each start's unit iterate, for the final evaluation
void deflate_final_alpha(hipStream_t st, const float* X, int64_t ldx, int64_t p,
                         int64_t r, Defl d);

// Tile shape (index into the compiled shapes) and K split of one product.
struct GemmPlan {
  int shape;
  int splits;
};

// Deterministic shape / split choice for an M x N x K product with
// elem_bytes-byte operands (4: FP32, 2: BF16).
GemmPlan plan_gemm_nt(int64_t M, int64_t N, int64_t K, int max_splits,
                      int elem_bytes = 4);
// the cost model alone (no tuning table)
GemmPlan model_plan_gemm_nt(int64_t M, int64_t N, int64_t K, int max_splits,
                            int elem_bytes = 4);
int gemm_num_shapes();
// rows of the output tile of a shape (0 for an unknown shape)
int gemm_shape_bm(int shape);
// largest power-of-two split count (<= max_splits) that leaves every split
// at least 8 K slabs
int max_feasible_splits(int64_t K, int max_splits, int elem_bytes);
// tuning table (process-wide, thread-safe)
bool tuned_plan(int64_t M, int64_t N, int64_t K, int max_splits, int elem_bytes,
                GemmPlan* out);
void record_tuned_plan(int64_t M, int64_t N, int64_t K, int max_splits,
                       int elem_bytes, GemmPlan plan);
std::string tune_table_text();
bool tune_table_load(const char* text, std::string* err);
void tune_table_clear();

// C (M x N, ldc) = P (M x K, ldp) * Q (N x K, ldq)^T, FP32 MFMA.  With
// plan.splits > 1, K split s writes its partial product at
// C + s * split_stride.  When gate != nullptr the kernel runs only if
// *gate == gate_run.  When kdev != nullptr, K is read from *kdev on the
// device (plan.splits must then be 1).
void gemm_nt_f32(hipStream_t st, const float* P, int64_t ldp, const float* Q,
                 int64_t ldq, float* C, int64_t ldc, int64_t M, int64_t N,
                 int64_t K, const int32_t* gate, int32_t gate_run,
                 GemmPlan plan, int64_t split_stride,
                 const int32_t* kdev = nullptr);

// The same product with BF16 operands (bit patterns, ld multiple of 8 and
// 16-byte aligned rows), FP32 accumulation and output.
void gemm_nt_bf16(hipStream_t st, const uint16_t* P, int64_t ldp,
                  const uint16_t* Q, int64_t ldq, float* C, int64_t ldc,
                  int64_t M, int64_t N, int64_t K, const int32_t* gate,
                  int32_t gate_run, GemmPlan plan, int64_t split_stride);

// Grouped products (requests sharing one launch): product q computes
// C = P * Q^T (M x N x K, leading dimensions ldp, ldq, ldc) with its own K
// split, split partials split_stride floats apart; req is the request it
// belongs to.  tiles_m, kslabs_per_split and tile0 are filled in by
// gemm_group_tiles, which also returns the launch's tile count.
struct GemmGroupDesc {
  const float* P;
  const float* Q;
  float* C;
  int64_t ldp, ldq, ldc, split_stride;
  int32_t M, N, K, splits, req;
  int32_t tiles_m, kslabs_per_split, tile0;
};
constexpr int kGroupBM = 64;   // tile of the grouped products
constexpr int kGroupBN = 128;
void gemm_group_tiles(GemmGroupDesc* d, int count, int* total_tiles);
// the products of d_dev (device copy of gemm_group_tiles' output); products
// of requests with running[req] == 0 are skipped (running may be null)
void gemm_nt_f32_group(hipStream_t st, const GemmGroupDesc* d_dev, int count, int total_tiles,
                       const int32_t* running);

// Row-major copy: At[i * ldat + k] = A[i + k * lda] (i < n, k < p).
void transpose_f32(hipStream_t st, const float* A, int64_t lda, float* At,
                   int64_t ldat, int64_t n, int64_t p);

// BF16 copies of A: column-major Ab (ldab, rows n..ldab zero) and row-major
// Atb (ldatb, columns p..ldatb zero).
void to_bf16_colmajor(hipStream_t st, const float* A, int64_t lda, int64_t n,
                      int64_t p, uint16_t* Ab, int64_t ldab);
void to_bf16_rowmajor(hipStream_t st, const float* A, int64_t lda, int64_t n,
                      int64_t p, uint16_t* Atb, int64_t ldatb);
// BF16 copy of the rows of a row-major FP32 matrix.
// Runs only when plan is null or selects the dense product.
void rows_to_bf16(hipStream_t st, const float* X, int64_t ldx, int64_t r,
                  int64_t p, uint16_t* Xb, int64_t ldxb, const Plan* plan);

// As[:, t] = A[:, idx[t]] for t < m (FP32, column-major, ldas).
void gather_columns(hipStream_t st, const float* A, int64_t lda, int64_t n,
                    const int32_t* idx, int64_t m, float* As, int64_t ldas);

// Column-major copy with a new leading dimension.
void copy_columns_f32(hipStream_t st, const float* A, int64_t lda, float* B,
                      int64_t ldb, int64_t n, int64_t p);

// Counts non-finite entries of A into *count (device int32, zeroed first by
// the caller).
void count_nonfinite(hipStream_t st, const float* A, int64_t lda, int64_t n,
                     int64_t p, int32_t* count);

// x0 = e_{i*}, i* = argmax_i ||a_i||_2 (ties to the lowest i), written to
// row 0 of X (ldx); colsq is p doubles of scratch.
void max_norm_column_start(hipStream_t st, const float* A, int64_t lda,
                           int64_t n, int64_t p, double* colsq, float* X,
                           int64_t ldx);

// Builds the compacted (index, value) lists of the rows of X, nnz per row;
// with colmark != nullptr also marks every used column with plan->epoch.
// (only: when not null, rows j with only[j] == 0 are skipped)
void compact_rows(hipStream_t st, const float* X, int64_t ldx, int64_t r,
                  int64_t p, int32_t* list_idx, float* list_val, int64_t ldl,
                  int32_t* nnz, const int32_t* status, int32_t* colmark,
                  const Plan* plan, const int32_t* only = nullptr);

// Resets the per-start state for a new solve.
void init_state(hipStream_t st, StartState s, int64_t r);

// Counts the running starts, gathers the union of their supports (columns
// marked with the current epoch) into ulist, and chooses the product mode
// for the next A x from a cost model; the list mode needs every running
// start to have at most list_cap nonzeros (only those keep lists).
void plan_next(hipStream_t st, StartState s, int64_t r, int64_t n, int64_t p,
               int list_cap, int dense_only, int dense_splits, int64_t ucap,
               const int32_t* colmark, int32_t* ulist, Plan* plan, int no_fused = 0,
               int allow_union = 1);

// Resets the plan (epoch 1, dense mode, zero statistics).
void init_plan(hipStream_t st, Plan* plan, int dense_splits);

// Rows of A that one workgroup of the row-block list product covers.  With
// n at most this, that product has one workgroup per start, as the fused
// list product does, but costs more, so the planner only considers it when
// the fused product is not allowed; solves then leave its launch out.
constexpr int64_t kRowsBlockN = 1024;
__host__ __device__ inline bool rows_product_possible(int64_t n, int no_fused) {
  return no_fused != 0 || n > kRowsBlockN;
}

// For kAxUnion: Xc[j][c] = X[j][ulist[c]] (r x u) and Qc[i][c] =
// A[i, ulist[c]] (n x u, row-major), u = plan->union_size.
void union_gather(hipStream_t st, const float* X, int64_t ldx, int64_t r,
                  const float* A, int64_t lda, int64_t n,
                  const int32_t* ulist, const Plan* plan, float* Xc,
                  int64_t ldxc, float* Qc, int64_t ldqc);

// y-update of Algorithm 2 from a dense U (r x n), given as plan->ax_splits
// partial products split_stride floats apart that are summed in order:
// V[i] = V[i] + V[stride + i] + ... + V[(splits - 1) stride + i] for i < count
// (the K-split partials of a product, summed in split order, in place)
void sum_splits(hipStream_t st, float* V, int64_t stride, int splits, int64_t count);

// Y = sgn(U) (L1 variance) or U / ||U||_2 per row (L2 variance); a zero row
// ends its start as DEGENERATE.  Skipped in list mode.
// With Yb != nullptr the rows are also written as BF16 (ldyb).
void y_update(hipStream_t st, int fid, const float* U, int64_t split_stride,
              float* Y, int64_t ldu, int64_t r, int64_t n, StartState s,
              const Plan* plan, uint16_t* Yb = nullptr, int64_t ldyb = 0);

// Grouped solves (s.cfg set): the y-update of every running start, with the
// variance type and the A x partial count of its request; the A^T y
// partials of every running start summed in split order into the first
// (split_stride floats apart, cfg.aty_splits of them, rows of p entries);
// and the running starts of each request (rows first[q] .. first[q+1]) into
// running[q], their total into running[count].
void group_y_update(hipStream_t st, const float* U, int64_t split_stride, float* Y,
                    int64_t ldu, int64_t r, int64_t n, StartState s);
void group_sum_splits(hipStream_t st, float* V, int64_t split_stride, int64_t ldv,
                      int64_t r, int64_t p, StartState s);
void group_count(hipStream_t st, const int32_t* status, const int64_t* first, int count,
                 int32_t* running);

// Sparse A x from the lists followed by the y-update, one block per start.
// Runs only in list mode.
void sparse_ax_y_update(hipStream_t st, int fid, const float* A, int64_t lda,
                        int64_t n, const int32_t* list_idx,
                        const float* list_val, int64_t ldl, float* Y,
                        int64_t ldu, int64_t r, StartState s, const Plan* plan);
// U (slot 0) = A X from the support lists in row blocks of 1024, FP64
// accumulation; runs only in mode kAxListRows (the y-update follows).
// Needs lda % 4 == 0 and a 16-byte aligned A.
void sparse_ax_rows(hipStream_t st, const float* A, int64_t lda, int64_t n,
                    const int32_t* list_idx, const float* list_val, int64_t ldl,
                    float* U, int64_t ldu, int64_t r, StartState s, const Plan* plan);
void sparse_ax_rows_bf16(hipStream_t st, const uint16_t* Ab, int64_t ldab, int64_t n,
                         const int32_t* list_idx, const float* list_val, int64_t ldl,
                         float* U, int64_t ldu, int64_t r, StartState s,
                         const Plan* plan);

// The same with a BF16 column-major A (ldab % 4 == 0); Y also as BF16.
void sparse_ax_y_update_bf16(hipStream_t st, int fid, const uint16_t* Ab,
                             int64_t ldab, int64_t n, const int32_t* list_idx,
                             const float* list_val, int64_t ldl, float* Y,
                             int64_t ldu, uint16_t* Yb, int64_t ldyb, int64_t r,
                             StartState s, const Plan* plan);

// x-update of Algorithm 2 on the rows of V with the stop test of Section
// 2.2.  Rows with at most list_cap nonzeros also get their (index, value)
// list.  When s.status is null every row is processed and no stop test or
// counters are touched (operator-only mode used by spca_x_update).
// Every kept column of a processed row is marked colmark[i] = plan->epoch
// (colmark may be null).
// Rows longer than kWideMinP use the chunked kernels when `wide` points to
// x_update_wide_bytes(fid, r, p) bytes of scratch whose histogram part was
// cleared by x_update_wide_reset (the kernels leave it cleared again).
void x_update(hipStream_t st, int fid, double s_or_gamma, const float* V,
              int64_t ldv, int64_t r, int64_t p, float* X, int64_t ldx,
              int32_t* list_idx, float* list_val, int64_t ldl, int list_cap,
              StartState s, double tol, int32_t maxit, int32_t* colmark,
              const Plan* plan, void* wide = nullptr, Warm wm = Warm{});

constexpr int64_t kWideMinP = 12288;
// scratch of the chunked x-update (0 when it does not apply: lambda_s, or
// p <= kWideMinP); the size is the same for every other formulation
size_t x_update_wide_bytes(int fid, int64_t r, int64_t p);
hipError_t x_update_wide_reset(hipStream_t st, void* scratch, int64_t r);
// 32-bit words at the start of that scratch which x_update_wide_reset clears
int64_t x_update_wide_clear_words(int64_t r);

// Argument checks shared by the entry points (SPCA_EINVAL with a message).
int check_problem(int64_t n, int64_t p, int64_t lda, int fid, double sg,
                  int64_t r, double tol, int32_t maxit);
// launches the chunked x-update; false (nothing launched) when it does not
// apply
bool x_update_wide(hipStream_t st, int fid, double s_or_gamma, const float* V,
                   int64_t ldv, int64_t r, int64_t p, float* X, int64_t ldx,
                   int32_t* list_idx, float* list_val, int64_t ldl, int list_cap,
                   StartState s, double tol, int32_t maxit, int32_t* colmark,
                   const Plan* plan, void* scratch, Warm wm);

// FP64 finalisation: per start, x64 = x / ||x||_2 from the lists, f(x64)
// of Table 1 and the explained variance; then the best start.
// gam: per-start gamma of the penalties (warm-up), or null for s_or_gamma;
// by_ev: pick the best start by explained variance instead of f
// X_dense (r x ldx FP32 iterates, the lists' dense twin): for mostly dense
// iterates, U = A X^T in FP64 on the matrix cores (partial needs
// 2 r ceil(n / 64) doubles) instead of per-start sums over the lists; with
// upart (final_gemm64_splits(n, p, r) r n doubles, at most r p floats' worth)
// that product is split over the columns for more workgroups
void finalize(hipStream_t st, int fid, double s_or_gamma, const float* A,
              int64_t lda, int64_t n, int64_t p, const int32_t* list_idx,
              const float* list_val, int64_t ldl, StartState s, int64_t r,
              double* partial, double* f, double* ev, double* xnorm,
              int32_t* best, double* x_out, int32_t* support_out,
              const double* gam = nullptr, bool by_ev = false, Defl defl = Defl{},
              const float* X_dense = nullptr, int64_t ldx = 0, double* upart = nullptr);
// column splits of that product: a function of the shape only
int final_gemm64_splits(int64_t n, int64_t p, int64_t r);
// The FP64 objective and explained variance of the rows with only[j] != 0
// (the first three steps of finalize); other rows are left untouched.
void evaluate_rows(hipStream_t st, int fid, double s_or_gamma, const float* A,
                   int64_t lda, int64_t n, const int32_t* list_idx,
                   const float* list_val, int64_t ldl, StartState s, int64_t r,
                   double* partial, double* f, double* ev, double* xnorm,
                   const int32_t* only, const double* gam = nullptr,
                   Defl defl = Defl{});

// The two ends of finalize, for products formed elsewhere (sparse A):
// ||x||_2 of each start's list; then f, the explained variance and the best
// start from per-start partial sums (sum u_i^2, sum |u_i|) of u = A x64.
void x_norms(hipStream_t st, const float* list_val, int64_t ldl, StartState s, int64_t r,
             double* xnorm);
void objective_and_best(hipStream_t st, int fid, double s_or_gamma, StartState s,
                        int64_t r, int64_t p, const double* partial, int nchunks,
                        const int32_t* list_idx, const float* list_val, int64_t ldl,
                        const double* xnorm, double* f, double* ev, int32_t* best,
                        double* x_out, int32_t* support_out, const double* gam,
                        bool by_ev);

// Sparse A (compressed sparse columns, with its row-compressed twin), plus
// the chunk tables of the balanced products (first nonempty column / row of
// every chunk of consecutive nonzeros; sparse_chunks(nnz) entries each).
struct SparseA {
  int64_t n, p, nnz;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const float* col_val;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const float* row_val;
  int32_t* col_first;
  int32_t* row_first;
  // row panels of the columns for A^T Y (npan = 0: none): panel P holds rows
  // [P prow, (P + 1) prow); "major" P p + c is column c restricted to panel
  // P, stored at pptr[P p + c] .. pptr[P p + c + 1] of pidx / pval
  int32_t npan = 0;
  int64_t prow = 0;
  int64_t* pptr = nullptr;  // npan p + 1
  int32_t* pidx = nullptr;
  float* pval = nullptr;
  int32_t* pfirst = nullptr;  // chunk table of the panel layout
  int64_t* ptmp = nullptr;    // sparse_panel_tmp(npan, p) int64 of scratch
  // majors crossing a chunk boundary (sparse_chunks(nnz) entries each): rows
  // of the row layout, columns (or panel majors) of the column layout
  int32_t* row_split = nullptr;
  int32_t* col_split = nullptr;
  int64_t nrow_split = 0, ncol_split = 0;
};
int64_t sparse_chunks(int64_t nnz);
// panels for A^T Y: 0 (none) or the count that keeps each panel's slice of
// YT within the gather window; force: 1 on, -1 off, 0 by size
int32_t sparse_panels(int64_t n, int64_t p, int64_t nnz, int64_t ldt, int force);
int64_t sparse_panel_tmp(int32_t npan, int64_t p);
// builds the panel layout from the (validated) columns
void sparse_build_panels(hipStream_t st, SparseA& a);
// lists the majors crossing chunk boundaries of both layouts (after the
// panels, if any); counts[0] (rows) and counts[1] (columns) must be zero
void sparse_split_lists(hipStream_t st, const SparseA& a, int32_t* counts);
// leading dimension of the transposed operands and products for r starts
int64_t sparse_ld(int64_t r);
// partial pairs per start of sparse_final
int64_t sparse_final_parts(int64_t n);
// checks (bits or-ed into *bad: 1 a pointer array decreases, 2 an index out
// of range, 4 row indices of a column not strictly increasing) and builds
// the chunk tables; reads only inside the arrays as sized by nnz
void sparse_prepare(hipStream_t st, const SparseA& a, int32_t* bad);
// U (r x n) = A X for dense X from the rows (XT: X transposed, p x ldxt;
// UT: n x ldxt; carry: 2 * sparse_chunks(nnz) x ldxt); runs in mode
// kAxDense, for the running starts
void sparse_ax_dense(hipStream_t st, const SparseA& a, const float* XT, int64_t ldxt,
                     int64_t r, float* UT, float* carry, float* U, int64_t ldu,
                     StartState s, const Plan* plan);
// y-update of the running starts from start-major U straight into YT (n x
// ldt); partial: r * sparse_y_parts(n) doubles
int64_t sparse_y_parts(int64_t n);
void sparse_y_update(hipStream_t st, int fid, const float* U, int64_t ldu, int64_t n,
                     int64_t r, StartState s, double* partial, float* YT, int64_t ldt);
// U row j = sum over the start's support columns; runs in mode kAxListRows
void sparse_ax_list(hipStream_t st, const SparseA& a, const int32_t* list_idx,
                    const float* list_val, int64_t ldl, float* U, int64_t ldu, int64_t r,
                    StartState s, const Plan* plan);
// V (r x p) = A^T Y from the columns, or from their row panels when
// a.npan > 0 (YT: Y transposed, n x ldyt; VT: max(npan, 1) p x ldyt; carry
// as above), for the running starts
void sparse_aty(hipStream_t st, const SparseA& a, const float* YT, int64_t ldyt, int64_t r,
                float* VT, float* carry, float* V, int64_t ldv, StartState s,
                const Plan* plan);
// per-start partial pairs (sparse_final_parts(n) each) of the FP64
// u = A x / ||x|| (minus sum alpha_i A x_i under deflation) for
// objective_and_best
void sparse_final(hipStream_t st, const SparseA& a, const int32_t* list_idx,
                  const float* list_val, int64_t ldl, StartState s, int64_t r,
                  const double* xnorm, double* partial, Defl defl);
// FP64 scores A x_i of the deflation loadings (after deflate_loadings)
void sparse_deflate_scores(hipStream_t st, const SparseA& a, Defl d);

// On-the-fly replacement of finished starts (Section 4.3): state of the
// slots and of the total_starts starts that flow through them.
struct Otf {
  int32_t* slot_start;  // r: start held by the slot, -1 once empty
  int32_t* retiring;    // r: the slot's start finished in this x-update
  int32_t* refill;      // r: start loaded into the slot now, -1 none
  int32_t* ctl;         // [0] next start to issue, [1] best start, [2] slot
                        // holding the best start now (-1 none)
  double* best_f;       // 1
  float* best_x;        // p: the best start's final iterate
  double* f;            // total: per start f, explained variance, phi
  double* ev;
  double* phi;
  int32_t* iters;       // total: per start iterations, status, nnz
  int32_t* status;
  int32_t* nnz;
  float* x_all;         // total x p or null: each start's final iterate
  int64_t total;
};
// per iteration, after the x-update: mark finished slots, evaluate them,
// record their results and the best so far, load the next starts
// (X0 rows) into the freed slots and reset their state
void otf_step(hipStream_t st, int fid, double s_or_gamma, const float* A,
              int64_t lda, int64_t n, int64_t p, float* X, int64_t ldx,
              const float* X0, int32_t* list_idx, float* list_val, int64_t ldl,
              StartState s, int64_t r, double* partial, double* f, double* ev,
              double* xnorm, Otf o, int force);
void otf_init(hipStream_t st, Otf o, int64_t r);
// x_out (FP64, unit norm) and the sorted support of the best start; writes
// {best start, nnz} to best
void otf_output(hipStream_t st, Otf o, int64_t p, int32_t* best, double* x_out,
                int32_t* support_out);

}  // namespace spca
