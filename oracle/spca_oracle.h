/*
 * FP64 CPU oracle for the alternating-maximization (AM) sparse PCA method
 * of Richtarik, Jahani, Ahipasaoglu and Takac, "Alternating maximization:
 * unifying framework for 8 sparse PCA formulations and efficient parallel
 * codes" (arXiv:1212.4137).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the HIP
 * path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library; the GPU library never links it.
 *
 * Conventions (all arrays are host memory, caller-owned):
 *   A   : n x p, column-major, leading dimension lda >= n, FP64.
 *   x   : length p.   X0 : r x p, start-major (row j is start j).
 *   fid : formulation number 1..8, numbered as in Table 1 of the paper.
 */
#ifndef SPCA_ORACLE_H
#define SPCA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-start termination status */
enum {
  ORC_CONVERGED = 0,  /* ratio stop test met                           */
  ORC_MAXIT = 1,      /* maxit x-updates done without meeting the test */
  ORC_DEGENERATE = 2, /* A x = 0 for the current iterate               */
  ORC_ZERO = 3        /* the x-operator returned the zero vector       */
};

/* Operators of Section 2.1 (Table 3 and the definitions of T_s, U_gamma,
 * V_gamma and lambda_s).  Each writes the operator's image of a into out
 * (length m) and returns the optimal value phi(z*) of the subproblem it
 * solves (Table 3, last column).                                           */
double orc_T_s(const double* a, int64_t m, int64_t s, double* out);
double orc_U_gamma(const double* a, int64_t m, double gamma, double* out);
double orc_V_gamma(const double* a, int64_t m, double gamma, double* out);
double orc_lambda_s(const double* a, int64_t m, double s);
double orc_V_lambda_s(const double* a, int64_t m, double s, double* out);

/* x-operator of Algorithm 2 for formulation fid applied to v (length p);
 * w receives the unnormalised image, return value is phi (Table 3).       */
double orc_x_operator(int fid, const double* v, int64_t p, double s_or_gamma,
                      double* w);

/* f(x) of Table 1 for formulation fid, and the explained variance
 * (||Ax||_2^2 for L2 variance, ||Ax||_1 for L1 variance).                 */
double orc_objective(int fid, const double* A, int64_t n, int64_t p,
                     int64_t lda, const double* x, double s_or_gamma,
                     double* explained_variance);

/* Algorithm 2 from one starting point.  x_out (p) receives the final unit
 * (or zero) loading vector; phi_trace (maxit entries, may be NULL) receives
 * phi after every x-update.  Returns the status, *iters = x-updates done.  */
int orc_am_single(const double* A, int64_t n, int64_t p, int64_t lda, int fid,
                  double s_or_gamma, const double* x0, double tol,
                  int32_t maxit, double* x_out, double* phi_trace,
                  int32_t* iters, double* f, double* ev);

/* Multi-start driver (Section 4): runs every start of X0 (r x p) and picks
 * the largest objective, ties to the lowest start index.  Per-start arrays
 * (length r) and X_out (r x p) may be NULL.  nthreads >= 1 splits the
 * independent starts over POSIX threads; results do not depend on it.
 * Returns the index of the best start.                                     */
int32_t orc_am_multi(const double* A, int64_t n, int64_t p, int64_t lda,
                     int fid, double s_or_gamma, const double* X0, int32_t r,
                     double tol, int32_t maxit, int nthreads, double* X_out,
                     double* f_out, double* ev_out, double* phi_out,
                     int32_t* iters_out, int32_t* status_out);

/* Algorithm 2 with the sparsity-targeted warm-up used in the experiments of
 * Section 4.1 (explained-variance hunt): during the first warm_iters
 * x-updates the parameter follows the current v, afterwards it is frozen at
 * its last value.
 *   L1 constraint (fid 3, 4): lambda = lambda_s(v) while warming up, then
 *     x = V_lambda(v) / ||.|| with the frozen lambda; phi = lambda sqrt(s)
 *     + ||V_lambda(v)|| throughout.  s_or_gamma is s.
 *   Penalties (fid 5..8): gamma = the (target_s + 1)-th largest v_i^2 (L0
 *     penalty, U_gamma) or |v_i| (L1 penalty, V_gamma) while warming up
 *     (0 when target_s >= p), so that exactly target_s entries pass the
 *     strict threshold (ties aside); then frozen.  s_or_gamma is unused
 *     when warm_iters > 0.
 * The ratio stop test applies once the parameter is frozen (from x-update
 * warm_iters + 1 on, and never before the second).  warm_iters = 0 is the
 * plain algorithm.  *param_out receives the final lambda or gamma, which
 * also enters f(x) for the penalties.  Returns the status.                 */
int orc_am_single_warm(const double* A, int64_t n, int64_t p, int64_t lda,
                       int fid, double s_or_gamma, int64_t target_s,
                       int32_t warm_iters, const double* x0, double tol,
                       int32_t maxit, double* x_out, int32_t* iters, double* f,
                       double* ev, double* param_out);

/* Multi-start driver of orc_am_single_warm.  The best start is the one with
 * the largest explained variance (ties to the lowest index): with the
 * warm-up every start ends with its own gamma, so f is not comparable
 * across starts.  Returns the index of the best start.                    */
int32_t orc_am_multi_warm(const double* A, int64_t n, int64_t p, int64_t lda,
                          int fid, double s_or_gamma, int64_t target_s,
                          int32_t warm_iters, const double* X0, int32_t r,
                          double tol, int32_t maxit, int nthreads, double* X_out,
                          double* f_out, double* ev_out, double* param_out,
                          int32_t* iters_out, int32_t* status_out);

/* Deflation for further components (the paper obtains them by replacing A
 * with a deflated matrix; the scheme is the projection deflation of the
 * data matrix): out = A (I - x x^T) = A - (A x) x^T, FP64, out n x p with
 * leading dimension ldo >= n.  Applied once per found loading x (unit
 * norm), in the order the loadings were found.                            */
void orc_deflate(const double* A, int64_t n, int64_t p, int64_t lda,
                 const double* x, double* out, int64_t ldo);

/* The same multi-start AM on a sparse A held in compressed sparse columns
 * (col_ptr: p + 1 offsets, row_idx / val: the nonzeros of each column),
 * FP64 values.  The products touch only the stored entries; otherwise it is
 * orc_am_multi step for step.  Returns the best start.                    */
int32_t orc_am_multi_csc(const int64_t* col_ptr, const int32_t* row_idx,
                         const double* val, int64_t n, int64_t p, int fid,
                         double s_or_gamma, const double* X0, int32_t r, double tol,
                         int32_t maxit, int nthreads, double* X_out, double* f_out,
                         double* ev_out, int32_t* iters_out, int32_t* status_out);

/* argmax_i ||a_i||_2 over the columns of A, ties to the lowest index.     */
int64_t orc_max_norm_column(const double* A, int64_t n, int64_t p,
                            int64_t lda);

#ifdef __cplusplus
}
#endif
#endif
