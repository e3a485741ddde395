/*
 * FP64 CPU oracle for the AM sparse PCA method (arXiv:1212.4137).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow and written to be checked against
 * the paper by eye.  No BLAS, no blocking, no fusion.  It shares no code
 * with the GPU library.  See spca_oracle.h for the conventions.
 *
 * Readings of the paper that the code takes where the text is silent:
 *   - sgn(0) = 0 (the sign of t, Notation paragraph of Section 1), so
 *     U_gamma keeps a_i only when a_i^2 > gamma strictly.
 *   - T_s breaks ties in |a_i| towards the lower index.
 *   - lambda_s is found exactly: it is the root of the derivative of the
 *     convex one-dimensional dual, which is piecewise quadratic in lambda
 *     between consecutive sorted |a_i|.
 *   - The stop test of Section 2.2 compares phi after consecutive
 *     x-updates in multiplicative form, phi_k <= (1 + tol) phi_{k-1};
 *     tol < 0 disables it; maxit counts x-updates.
 *   - A x = 0 (theorem 1 excludes it) ends the start as DEGENERATE; an
 *     x-operator image equal to zero ends it as ZERO.  Both report x = 0
 *     and f = 0 (x = 0 is feasible for every formulation).
 */
#include "spca_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

static int is_l1_variance(int fid) { return (fid % 2) == 0; }

static double sgn(double t) { return (t > 0.0) - (t < 0.0); }

/* ---------------------------------------------------------------------- */
/* Operators (Section 2.1)                                                 */
/* ---------------------------------------------------------------------- */

typedef struct {
  double key; /* |a_i| */
  int64_t idx;
} keyed_t;

/* descending |a_i|, then ascending index */
static int cmp_desc_then_index(const void* pa, const void* pb) {
  const keyed_t* a = (const keyed_t*)pa;
  const keyed_t* b = (const keyed_t*)pb;
  if (a->key > b->key) return -1;
  if (a->key < b->key) return 1;
  return (a->idx > b->idx) - (a->idx < b->idx);
}

/* T_s(a): keep the s entries largest in absolute value, zero the rest.
 * Returns ||T_s(a)||_2, the optimal value of subproblem S3.               */
double orc_T_s(const double* a, int64_t m, int64_t s, double* out) {
  keyed_t* order = (keyed_t*)malloc(sizeof(keyed_t) * (size_t)(m > 0 ? m : 1));
  for (int64_t i = 0; i < m; ++i) {
    order[i].key = fabs(a[i]);
    order[i].idx = i;
  }
  qsort(order, (size_t)m, sizeof(keyed_t), cmp_desc_then_index);
  for (int64_t i = 0; i < m; ++i) out[i] = 0.0;
  double sq = 0.0;
  for (int64_t t = 0; t < s && t < m; ++t) {
    int64_t i = order[t].idx;
    out[i] = a[i];
    sq += a[i] * a[i];
  }
  free(order);
  return sqrt(sq);
}

/* (U_gamma(a))_i = a_i [sgn(a_i^2 - gamma)]_+ .  Returns the S5 optimum
 * ||U||_2^2 - gamma ||U||_0 = sum over kept i of (a_i^2 - gamma).          */
double orc_U_gamma(const double* a, int64_t m, double gamma, double* out) {
  double phi = 0.0;
  for (int64_t i = 0; i < m; ++i) {
    double keep = fmax(0.0, sgn(a[i] * a[i] - gamma));
    out[i] = a[i] * keep;
    if (keep > 0.0) phi += a[i] * a[i] - gamma;
  }
  return phi;
}

/* (V_gamma(a))_i = sgn(a_i) (|a_i| - gamma)_+ .  Returns the S6 optimum
 * ||V_gamma(a)||_2.                                                        */
double orc_V_gamma(const double* a, int64_t m, double gamma, double* out) {
  double sq = 0.0;
  for (int64_t i = 0; i < m; ++i) {
    out[i] = sgn(a[i]) * fmax(0.0, fabs(a[i]) - gamma);
    sq += out[i] * out[i];
  }
  return sqrt(sq);
}

/* lambda_s(a) = argmin_{lambda >= 0} lambda sqrt(s) + ||V_lambda(a)||_2.
 *
 * With c_1 >= c_2 >= ... >= c_m > 0 the nonzero |a_i| and c_{m+1} = 0, on
 * [c_{k+1}, c_k] exactly the k largest entries are active and
 * ||V_lambda||_2^2 = S2_k - 2 lambda S1_k + k lambda^2 (prefix sums of c
 * and c^2).  The derivative of the objective is sqrt(s) - rho(lambda) with
 * rho = ||V_lambda||_1 / ||V_lambda||_2, non-increasing in lambda.  So
 * lambda = 0 when rho(0) <= sqrt(s); otherwise lambda solves
 * rho(lambda) = sqrt(s) in the first segment (largest lambda first) whose
 * lower end already has rho >= sqrt(s), where squaring gives
 * lambda_k = (S1_k - sqrt(s (k S2_k - S1_k^2) / (k - s))) / k.            */
double orc_lambda_s(const double* a, int64_t m, double s) {
  keyed_t* c = (keyed_t*)malloc(sizeof(keyed_t) * (size_t)(m > 0 ? m : 1));
  int64_t nz = 0;
  for (int64_t i = 0; i < m; ++i) {
    if (a[i] != 0.0) {
      c[nz].key = fabs(a[i]);
      c[nz].idx = i;
      ++nz;
    }
  }
  qsort(c, (size_t)nz, sizeof(keyed_t), cmp_desc_then_index);
  double total1 = 0.0, total2 = 0.0;
  for (int64_t t = 0; t < nz; ++t) {
    total1 += c[t].key;
    total2 += c[t].key * c[t].key;
  }
  const double rs = sqrt(s);
  double lambda = 0.0;
  if (nz > 0 && total1 > rs * sqrt(total2)) {
    double S1 = 0.0, S2 = 0.0;
    for (int64_t k = 1; k <= nz; ++k) {
      S1 += c[k - 1].key;
      S2 += c[k - 1].key * c[k - 1].key;
      if ((double)k <= s) continue;
      double lo = (k < nz) ? c[k].key : 0.0; /* c_{k+1} */
      double hi = c[k - 1].key;              /* c_k     */
      /* rho at the lower end of the segment */
      double l1 = S1 - (double)k * lo;
      double l2 = S2 - 2.0 * lo * S1 + (double)k * lo * lo;
      if (l2 > 0.0 && l1 >= rs * sqrt(l2)) {
        double disc = (double)k * S2 - S1 * S1;
        if (disc < 0.0) disc = 0.0;
        double lam = (S1 - sqrt(s * disc / ((double)k - s))) / (double)k;
        if (lam < lo) lam = lo;
        if (lam > hi) lam = hi;
        lambda = lam;
        break;
      }
    }
  }
  free(c);
  return lambda;
}

/* V_{lambda_s(a)}(a); returns the S4 optimum lambda sqrt(s) + ||V||_2.     */
double orc_V_lambda_s(const double* a, int64_t m, double s, double* out) {
  double lambda = orc_lambda_s(a, m, s);
  double norm = orc_V_gamma(a, m, lambda, out);
  return lambda * sqrt(s) + norm;
}

/* x-update operator of Algorithm 2 (Table 3, rows S3-S6).               */
double orc_x_operator(int fid, const double* v, int64_t p, double s_or_gamma,
                      double* w) {
  switch (fid) {
    case 1:
    case 2: /* L0 constraint: T_s */
      return orc_T_s(v, p, (int64_t)s_or_gamma, w);
    case 3:
    case 4: /* L1 constraint: V_{lambda_s} */
      return orc_V_lambda_s(v, p, s_or_gamma, w);
    case 5:
    case 6: /* L0 penalty: U_gamma */
      return orc_U_gamma(v, p, s_or_gamma, w);
    case 7:
    case 8: /* L1 penalty: V_gamma */
      return orc_V_gamma(v, p, s_or_gamma, w);
    default:
      return NAN;
  }
}

/* ---------------------------------------------------------------------- */
/* Linear algebra (plain loops)                                            */
/* ---------------------------------------------------------------------- */

/* u = A x */
static void matvec(const double* A, int64_t n, int64_t p, int64_t lda,
                   const double* x, double* u) {
  for (int64_t i = 0; i < n; ++i) u[i] = 0.0;
  for (int64_t j = 0; j < p; ++j) {
    double xj = x[j];
    const double* col = A + j * lda;
    for (int64_t i = 0; i < n; ++i) u[i] += col[i] * xj;
  }
}

/* v = A^T y */
static void matvec_t(const double* A, int64_t n, int64_t p, int64_t lda,
                     const double* y, double* v) {
  for (int64_t j = 0; j < p; ++j) {
    const double* col = A + j * lda;
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += col[i] * y[i];
    v[j] = acc;
  }
}

static double norm2(const double* z, int64_t m) {
  double sq = 0.0;
  for (int64_t i = 0; i < m; ++i) sq += z[i] * z[i];
  return sqrt(sq);
}

static double norm1(const double* z, int64_t m) {
  double s = 0.0;
  for (int64_t i = 0; i < m; ++i) s += fabs(z[i]);
  return s;
}

static double norm0(const double* z, int64_t m) {
  double c = 0.0;
  for (int64_t i = 0; i < m; ++i) c += (z[i] != 0.0);
  return c;
}

/* f(x) of Table 1 */
double orc_objective(int fid, const double* A, int64_t n, int64_t p,
                     int64_t lda, const double* x, double s_or_gamma,
                     double* explained_variance) {
  double* u = (double*)malloc(sizeof(double) * (size_t)n);
  matvec(A, n, p, lda, x, u);
  double var = is_l1_variance(fid) ? norm1(u, n) : norm2(u, n);
  free(u);
  if (explained_variance)
    *explained_variance = is_l1_variance(fid) ? var : var * var;
  const double gamma = s_or_gamma;
  switch (fid) {
    case 1: case 2: case 3: case 4:
      return var;                                /* ||Ax||            */
    case 5: case 6:
      return var * var - gamma * norm0(x, p);    /* ||Ax||^2 - g||x||_0 */
    case 7: case 8:
      return var - gamma * norm1(x, p);          /* ||Ax|| - g||x||_1 */
    default:
      return NAN;
  }
}

/* ---------------------------------------------------------------------- */
/* Algorithm 2                                                             */
/* ---------------------------------------------------------------------- */

int orc_am_single(const double* A, int64_t n, int64_t p, int64_t lda, int fid,
                  double s_or_gamma, const double* x0, double tol,
                  int32_t maxit, double* x_out, double* phi_trace,
                  int32_t* iters, double* f, double* ev) {
  double* x = (double*)malloc(sizeof(double) * (size_t)p);
  double* w = (double*)malloc(sizeof(double) * (size_t)p);
  double* v = (double*)malloc(sizeof(double) * (size_t)p);
  double* u = (double*)malloc(sizeof(double) * (size_t)n);
  memcpy(x, x0, sizeof(double) * (size_t)p);

  int status = ORC_MAXIT;
  double phi_prev = 0.0;
  int32_t k = 0;
  while (k < maxit) {
    /* y-update: u = A x, y = sgn(u) (L1 variance) or u / ||u||_2 (L2) */
    matvec(A, n, p, lda, x, u);
    double unorm = norm2(u, n);
    if (unorm == 0.0) {
      status = ORC_DEGENERATE;
      break;
    }
    for (int64_t i = 0; i < n; ++i)
      u[i] = is_l1_variance(fid) ? sgn(u[i]) : u[i] / unorm;
    /* x-update: v = A^T y, x = op(v) / ||op(v)||_2 */
    matvec_t(A, n, p, lda, u, v);
    double phi = orc_x_operator(fid, v, p, s_or_gamma, w);
    ++k;
    if (phi_trace) phi_trace[k - 1] = phi;
    double wnorm = norm2(w, p);
    if (wnorm == 0.0) {
      status = ORC_ZERO;
      break;
    }
    for (int64_t j = 0; j < p; ++j) x[j] = w[j] / wnorm;
    /* stop test: phi_k / phi_{k-1} <= 1 + tol */
    if (k >= 2 && tol >= 0.0 && phi <= (1.0 + tol) * phi_prev) {
      status = ORC_CONVERGED;
      break;
    }
    phi_prev = phi;
  }
  if (status == ORC_DEGENERATE || status == ORC_ZERO) {
    for (int64_t j = 0; j < p; ++j) x[j] = 0.0;
  }
  double evv = 0.0;
  double fv = 0.0;
  if (status == ORC_DEGENERATE || status == ORC_ZERO) {
    fv = 0.0;
    evv = 0.0;
  } else {
    fv = orc_objective(fid, A, n, p, lda, x, s_or_gamma, &evv);
  }
  if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)p);
  if (iters) *iters = k;
  if (f) *f = fv;
  if (ev) *ev = evv;
  free(x);
  free(w);
  free(v);
  free(u);
  return status;
}

typedef struct {
  const double* A;
  int64_t n, p, lda;
  int fid;
  double s_or_gamma;
  const double* X0;
  int32_t r;
  double tol;
  int32_t maxit;
  int nthreads;
  int tid;
  double* X_out;
  double* f_out;
  double* ev_out;
  double* phi_out;
  int32_t* iters_out;
  int32_t* status_out;
  double* f_all;
} multi_job_t;

static void* multi_worker(void* arg) {
  multi_job_t* jb = (multi_job_t*)arg;
  double* phi_trace =
      (double*)malloc(sizeof(double) * (size_t)(jb->maxit > 0 ? jb->maxit : 1));
  for (int32_t j = jb->tid; j < jb->r; j += jb->nthreads) {
    int32_t it = 0;
    double fv = 0.0, evv = 0.0;
    double* xo = jb->X_out ? jb->X_out + (int64_t)j * jb->p : NULL;
    int st = orc_am_single(jb->A, jb->n, jb->p, jb->lda, jb->fid,
                           jb->s_or_gamma, jb->X0 + (int64_t)j * jb->p,
                           jb->tol, jb->maxit, xo, phi_trace, &it, &fv, &evv);
    jb->f_all[j] = fv;
    if (jb->f_out) jb->f_out[j] = fv;
    if (jb->ev_out) jb->ev_out[j] = evv;
    if (jb->phi_out) jb->phi_out[j] = it > 0 ? phi_trace[it - 1] : 0.0;
    if (jb->iters_out) jb->iters_out[j] = it;
    if (jb->status_out) jb->status_out[j] = st;
  }
  free(phi_trace);
  return NULL;
}

int32_t orc_am_multi(const double* A, int64_t n, int64_t p, int64_t lda,
                     int fid, double s_or_gamma, const double* X0, int32_t r,
                     double tol, int32_t maxit, int nthreads, double* X_out,
                     double* f_out, double* ev_out, double* phi_out,
                     int32_t* iters_out, int32_t* status_out) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > r) nthreads = r;
  double* f_all = (double*)malloc(sizeof(double) * (size_t)r);
  multi_job_t* jobs = (multi_job_t*)malloc(sizeof(multi_job_t) * (size_t)nthreads);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
  for (int t = 0; t < nthreads; ++t) {
    multi_job_t jb = {A,  n,      p,      lda,       fid,     s_or_gamma,
                      X0, r,      tol,    maxit,     nthreads, t,
                      X_out, f_out, ev_out, phi_out, iters_out, status_out,
                      f_all};
    jobs[t] = jb;
  }
  for (int t = 1; t < nthreads; ++t)
    pthread_create(&th[t], NULL, multi_worker, &jobs[t]);
  multi_worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  /* best start: largest objective, ties to the lowest index */
  int32_t best = 0;
  for (int32_t j = 1; j < r; ++j)
    if (f_all[j] > f_all[best]) best = j;
  free(f_all);
  free(jobs);
  free(th);
  return best;
}

/* ------------------------------------------------------------------------ */
/* Sparsity-targeted warm-up (Section 4.1)                                  */
/* ------------------------------------------------------------------------ */

static int cmp_double_desc(const void* pa, const void* pb) {
  double a = *(const double*)pa, b = *(const double*)pb;
  return (a < b) - (a > b);
}

/* the (s+1)-th largest of |v_i| (or of v_i^2 when squared), 0 if s >= p */
static double target_threshold(const double* v, int64_t p, int64_t s, int squared) {
  if (s >= p) return 0.0;
  double* c = (double*)malloc(sizeof(double) * (size_t)p);
  for (int64_t i = 0; i < p; ++i) c[i] = squared ? v[i] * v[i] : fabs(v[i]);
  qsort(c, (size_t)p, sizeof(double), cmp_double_desc);
  double t = c[s];
  free(c);
  return t;
}

int orc_am_single_warm(const double* A, int64_t n, int64_t p, int64_t lda,
                       int fid, double s_or_gamma, int64_t target_s,
                       int32_t warm_iters, const double* x0, double tol,
                       int32_t maxit, double* x_out, int32_t* iters, double* f,
                       double* ev, double* param_out) {
  double* x = (double*)malloc(sizeof(double) * (size_t)p);
  double* w = (double*)malloc(sizeof(double) * (size_t)p);
  double* v = (double*)malloc(sizeof(double) * (size_t)p);
  double* u = (double*)malloc(sizeof(double) * (size_t)n);
  memcpy(x, x0, sizeof(double) * (size_t)p);
  const int lambda_kind = fid == 3 || fid == 4;
  /* the parameter in force: lambda (fid 3, 4) or gamma (fid 5..8) */
  double param = lambda_kind ? 0.0 : s_or_gamma;

  int status = ORC_MAXIT;
  double phi_prev = 0.0;
  int32_t k = 0;
  while (k < maxit) {
    matvec(A, n, p, lda, x, u);
    double unorm = norm2(u, n);
    if (unorm == 0.0) {
      status = ORC_DEGENERATE;
      break;
    }
    for (int64_t i = 0; i < n; ++i)
      u[i] = is_l1_variance(fid) ? sgn(u[i]) : u[i] / unorm;
    matvec_t(A, n, p, lda, u, v);
    ++k;
    const int warming = k <= warm_iters;
    double phi;
    if (lambda_kind) {
      if (warming || warm_iters == 0) param = orc_lambda_s(v, p, s_or_gamma);
      phi = param * sqrt(s_or_gamma) + orc_V_gamma(v, p, param, w);
    } else if (fid <= 2) {
      phi = orc_x_operator(fid, v, p, s_or_gamma, w);
    } else {
      const int l0pen = fid == 5 || fid == 6;
      if (warming) param = target_threshold(v, p, target_s, l0pen);
      phi = l0pen ? orc_U_gamma(v, p, param, w) : orc_V_gamma(v, p, param, w);
    }
    double wnorm = norm2(w, p);
    if (wnorm == 0.0) {
      status = ORC_ZERO;
      break;
    }
    for (int64_t j = 0; j < p; ++j) x[j] = w[j] / wnorm;
    if (k >= 2 && k >= warm_iters + 1 && tol >= 0.0 && phi <= (1.0 + tol) * phi_prev) {
      status = ORC_CONVERGED;
      break;
    }
    phi_prev = phi;
  }
  double evv = 0.0, fv = 0.0;
  if (status == ORC_DEGENERATE || status == ORC_ZERO) {
    for (int64_t j = 0; j < p; ++j) x[j] = 0.0;
  } else {
    fv = orc_objective(fid, A, n, p, lda, x, lambda_kind || fid <= 2 ? s_or_gamma : param,
                       &evv);
  }
  if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)p);
  if (iters) *iters = k;
  if (f) *f = fv;
  if (ev) *ev = evv;
  if (param_out) *param_out = param;
  free(x);
  free(w);
  free(v);
  free(u);
  return status;
}

typedef struct {
  const double* A;
  int64_t n, p, lda;
  int fid;
  double s_or_gamma;
  int64_t target_s;
  int32_t warm_iters;
  const double* X0;
  int32_t r;
  double tol;
  int32_t maxit;
  int nthreads, tid;
  double *X_out, *f_out, *ev_out, *param_out, *ev_all;
  int32_t *iters_out, *status_out;
} warm_job_t;

static void* warm_worker(void* arg) {
  warm_job_t* jb = (warm_job_t*)arg;
  for (int32_t j = jb->tid; j < jb->r; j += jb->nthreads) {
    int32_t it = 0;
    double fv = 0.0, evv = 0.0, par = 0.0;
    double* xo = jb->X_out ? jb->X_out + (int64_t)j * jb->p : NULL;
    int st = orc_am_single_warm(jb->A, jb->n, jb->p, jb->lda, jb->fid, jb->s_or_gamma,
                                jb->target_s, jb->warm_iters, jb->X0 + (int64_t)j * jb->p,
                                jb->tol, jb->maxit, xo, &it, &fv, &evv, &par);
    jb->ev_all[j] = evv;
    if (jb->f_out) jb->f_out[j] = fv;
    if (jb->ev_out) jb->ev_out[j] = evv;
    if (jb->param_out) jb->param_out[j] = par;
    if (jb->iters_out) jb->iters_out[j] = it;
    if (jb->status_out) jb->status_out[j] = st;
  }
  return NULL;
}

int32_t orc_am_multi_warm(const double* A, int64_t n, int64_t p, int64_t lda,
                          int fid, double s_or_gamma, int64_t target_s,
                          int32_t warm_iters, const double* X0, int32_t r,
                          double tol, int32_t maxit, int nthreads, double* X_out,
                          double* f_out, double* ev_out, double* param_out,
                          int32_t* iters_out, int32_t* status_out) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > r) nthreads = r;
  double* ev_all = (double*)malloc(sizeof(double) * (size_t)r);
  warm_job_t* jobs = (warm_job_t*)malloc(sizeof(warm_job_t) * (size_t)nthreads);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
  for (int t = 0; t < nthreads; ++t) {
    warm_job_t jb = {A, n, p, lda, fid, s_or_gamma, target_s, warm_iters, X0, r, tol,
                     maxit, nthreads, t, X_out, f_out, ev_out, param_out, ev_all,
                     iters_out, status_out};
    jobs[t] = jb;
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, warm_worker, &jobs[t]);
  warm_worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  int32_t best = 0;
  for (int32_t j = 1; j < r; ++j)
    if (ev_all[j] > ev_all[best]) best = j;
  free(ev_all);
  free(jobs);
  free(th);
  return best;
}

/* ------------------------------------------------------------------------ */
/* Sparse A in compressed sparse columns                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  const int64_t* cp;
  const int32_t* ri;
  const double* v;
  int64_t n, p;
} csc_t;

/* u = A x over the stored entries, column by column */
static void csc_matvec(const csc_t* M, const double* x, double* u) {
  for (int64_t i = 0; i < M->n; ++i) u[i] = 0.0;
  for (int64_t j = 0; j < M->p; ++j) {
    const double xj = x[j];
    for (int64_t k = M->cp[j]; k < M->cp[j + 1]; ++k) u[M->ri[k]] += M->v[k] * xj;
  }
}

/* v = A^T y */
static void csc_matvec_t(const csc_t* M, const double* y, double* v) {
  for (int64_t j = 0; j < M->p; ++j) {
    double acc = 0.0;
    for (int64_t k = M->cp[j]; k < M->cp[j + 1]; ++k) acc += M->v[k] * y[M->ri[k]];
    v[j] = acc;
  }
}

static int csc_am_single(const csc_t* M, int fid, double s_or_gamma, const double* x0,
                         double tol, int32_t maxit, double* x_out, int32_t* iters,
                         double* f, double* ev) {
  const int64_t n = M->n, p = M->p;
  double* x = (double*)malloc(sizeof(double) * (size_t)p);
  double* w = (double*)malloc(sizeof(double) * (size_t)p);
  double* v = (double*)malloc(sizeof(double) * (size_t)p);
  double* u = (double*)malloc(sizeof(double) * (size_t)n);
  memcpy(x, x0, sizeof(double) * (size_t)p);
  int status = ORC_MAXIT;
  double phi_prev = 0.0;
  int32_t k = 0;
  while (k < maxit) {
    csc_matvec(M, x, u);
    double unorm = norm2(u, n);
    if (unorm == 0.0) {
      status = ORC_DEGENERATE;
      break;
    }
    for (int64_t i = 0; i < n; ++i)
      u[i] = is_l1_variance(fid) ? sgn(u[i]) : u[i] / unorm;
    csc_matvec_t(M, u, v);
    double phi = orc_x_operator(fid, v, p, s_or_gamma, w);
    ++k;
    double wnorm = norm2(w, p);
    if (wnorm == 0.0) {
      status = ORC_ZERO;
      break;
    }
    for (int64_t j = 0; j < p; ++j) x[j] = w[j] / wnorm;
    if (k >= 2 && tol >= 0.0 && phi <= (1.0 + tol) * phi_prev) {
      status = ORC_CONVERGED;
      break;
    }
    phi_prev = phi;
  }
  double fv = 0.0, evv = 0.0;
  if (status == ORC_DEGENERATE || status == ORC_ZERO) {
    for (int64_t j = 0; j < p; ++j) x[j] = 0.0;
  } else {
    csc_matvec(M, x, u);
    double var = is_l1_variance(fid) ? norm1(u, n) : norm2(u, n);
    evv = is_l1_variance(fid) ? var : var * var;
    if (fid <= 4)
      fv = var;
    else if (fid <= 6)
      fv = var * var - s_or_gamma * norm0(x, p);
    else
      fv = var - s_or_gamma * norm1(x, p);
  }
  if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)p);
  if (iters) *iters = k;
  if (f) *f = fv;
  if (ev) *ev = evv;
  free(x);
  free(w);
  free(v);
  free(u);
  return status;
}

typedef struct {
  const csc_t* M;
  int fid;
  double s_or_gamma;
  const double* X0;
  int32_t r;
  double tol;
  int32_t maxit;
  int nthreads, tid;
  double *X_out, *f_out, *ev_out, *f_all;
  int32_t *iters_out, *status_out;
} csc_job_t;

static void* csc_worker(void* arg) {
  csc_job_t* jb = (csc_job_t*)arg;
  const int64_t p = jb->M->p;
  for (int32_t j = jb->tid; j < jb->r; j += jb->nthreads) {
    int32_t it = 0;
    double fv = 0.0, evv = 0.0;
    int st = csc_am_single(jb->M, jb->fid, jb->s_or_gamma, jb->X0 + (int64_t)j * p, jb->tol,
                           jb->maxit, jb->X_out ? jb->X_out + (int64_t)j * p : NULL, &it,
                           &fv, &evv);
    jb->f_all[j] = fv;
    if (jb->f_out) jb->f_out[j] = fv;
    if (jb->ev_out) jb->ev_out[j] = evv;
    if (jb->iters_out) jb->iters_out[j] = it;
    if (jb->status_out) jb->status_out[j] = st;
  }
  return NULL;
}

int32_t orc_am_multi_csc(const int64_t* col_ptr, const int32_t* row_idx,
                         const double* val, int64_t n, int64_t p, int fid,
                         double s_or_gamma, const double* X0, int32_t r, double tol,
                         int32_t maxit, int nthreads, double* X_out, double* f_out,
                         double* ev_out, int32_t* iters_out, int32_t* status_out) {
  csc_t M = {col_ptr, row_idx, val, n, p};
  if (nthreads < 1) nthreads = 1;
  if (nthreads > r) nthreads = r;
  double* f_all = (double*)malloc(sizeof(double) * (size_t)r);
  csc_job_t* jobs = (csc_job_t*)malloc(sizeof(csc_job_t) * (size_t)nthreads);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
  for (int t = 0; t < nthreads; ++t) {
    csc_job_t jb = {&M, fid, s_or_gamma, X0, r, tol, maxit, nthreads, t, X_out, f_out,
                    ev_out, f_all, iters_out, status_out};
    jobs[t] = jb;
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, csc_worker, &jobs[t]);
  csc_worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  int32_t best = 0;
  for (int32_t j = 1; j < r; ++j)
    if (f_all[j] > f_all[best]) best = j;
  free(f_all);
  free(jobs);
  free(th);
  return best;
}

void orc_deflate(const double* A, int64_t n, int64_t p, int64_t lda,
                 const double* x, double* out, int64_t ldo) {
  double* u = (double*)malloc(sizeof(double) * (size_t)n);
  matvec(A, n, p, lda, x, u);
  for (int64_t j = 0; j < p; ++j)
    for (int64_t i = 0; i < n; ++i) out[j * ldo + i] = A[j * lda + i] - u[i] * x[j];
  free(u);
}

int64_t orc_max_norm_column(const double* A, int64_t n, int64_t p,
                            int64_t lda) {
  int64_t best = 0;
  double best_sq = -1.0;
  for (int64_t j = 0; j < p; ++j) {
    double sq = 0.0;
    for (int64_t i = 0; i < n; ++i) sq += A[j * lda + i] * A[j * lda + i];
    if (sq > best_sq) {
      best_sq = sq;
      best = j;
    }
  }
  return best;
}
