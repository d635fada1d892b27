/*
 * CPU oracle for the Laplace-evidence hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of what the method computes, written
 * from the paper (arXiv 2601.19957, "SunBURST") and kept obviously correct:
 * plain loops, no BLAS, no blocking, no fusion.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may call it; the
 * product library never links, loads or calls anything here, and this file
 * shares no code with it.
 *
 * Functions whose results have no independent pin say "parity unpinned" in
 * their comment; every other one is checked against closed forms, brute
 * force, invariants or library routines by the CPU tests.
 *
 * Conventions: all arrays are row-major FP64; d is the dimension, K the
 * number of components.  Status codes use the same numeric values as the
 * product ABI (defined independently below).
 */
#ifndef SB_ORACLE_H
#define SB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OR_OK = 0, OR_E_INVAL = -1, OR_E_NOTPD = -2, OR_E_NOMEM = -3,
  OR_E_NOMODE = -5, OR_E_CAPACITY = -6, OR_E_UNSUPPORTED = -7
};
enum { OR_FAMILY_GAUSS_MIX = 0, OR_FAMILY_STUDENT_T = 1 };
enum { OR_NORM_PEAK_ZERO = 0, OR_NORM_DENSITY = 1 };
/* per-start optimiser outcome */
enum { OR_ST_ACTIVE = 0, OR_ST_CONVERGED = 1, OR_ST_STALLED = 2, OR_ST_MAXITER = 3,
       OR_ST_DEAD = 4 };

typedef struct {
  int32_t family, norm, d, K;
  const double *log_w; /* [K] or NULL (all weights 1) */
  const double *mu;    /* [K][d] */
  const double *prec;  /* [K][d][d] */
  double nu;           /* Student-t degrees of freedom */
  double logl_offset;  /* constant c added to the log-likelihood */
} or_problem;

typedef struct {
  int32_t n_rays, n_points, n_starts, m, max_iter, max_modes;
  double grad_tol;      /* L-BFGS stop: ||grad l||_inf <= grad_tol (<=0: 1e-10) */
  double dedup_tol;     /* final dedup radius (<=0: 1e-6 * max box width) */
  double dedup_tol_pre; /* pre-polish dedup radius (<=0: 0.25) */
  uint64_t seed;
  int32_t n_threads;    /* OpenMP threads for per-start work (<=0: all) */
  uint32_t problem;     /* problem index within a batch: Philox counter word 3 */
} or_config;

typedef struct {
  double log_z;
  int32_t n_modes;
  double *modes;      /* [max_modes][d] */
  double *mode_log_z; /* [max_modes] */
  double *mode_logl;  /* [max_modes] */
  double *log_det_h;  /* [max_modes] */
  int64_t n_logl_evals, n_grad_evals, n_hess_evals;
  int32_t iterations, n_rejected_nonpd, n_dead_starts, n_candidates, n_reps_pre;
} or_result;

/* ---- reductions (fixed order) ---- */
double or_pairwise_sum(const double *x, int64_t n);
double or_logsumexp(const double *x, int32_t n);

/* ---- dense linear algebra ---- */
/* A = L L^T; L lower-triangular (upper part zeroed).  Returns 0, or j+1 if the
 * pivot of column j is not positive (A not positive definite). */
int32_t or_cholesky(int32_t n, const double *A, double *L);
double or_logdet_from_chol(int32_t n, const double *L);
/* solve L L^T x = b */
void or_chol_solve(int32_t n, const double *L, const double *b, double *x);

/* ---- likelihood family ---- */
int32_t or_validate_problem(const or_problem *p);
/* per-component constants beta_k (and log det P_k); OR_E_NOTPD if a P_k fails */
int32_t or_prep(const or_problem *p, double *beta, double *logdet_prec);
/* log-likelihood (and gradient if grad != NULL) at B points X[B][d] */
void or_logl(const or_problem *p, const double *beta, int64_t B, const double *X, double *logl,
             double *grad);
/* Hessian-vector products of the log-likelihood: HV[b] = (nabla^2 l)(X[b]) V[b] */
void or_hvp(const or_problem *p, const double *beta, int64_t B, const double *X, const double *V,
            double *HV);
/* H = -nabla^2 l(x), [d][d] */
void or_neg_hessian(const or_problem *p, const double *beta, const double *x, double *H);

/* ---- counter-based RNG: Philox4x32-10 (Salmon et al., SC'11) ---- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t or_rng_word(uint64_t seed, uint32_t problem, uint32_t ray, uint32_t stream, uint32_t i);
double or_rng_uniform(uint64_t seed, uint32_t problem, uint32_t ray, uint32_t stream, uint32_t i);

/* ---- discovery ---- */
/* endpoints of R rays (four geometries, ray r uses geometry r mod 4) */
void or_rays(int32_t d, const double *lo, const double *hi, int32_t R, uint64_t seed,
             uint32_t problem, double *P0, double *P1);
/* evaluate l at R*n_pts ray points, per-ray argmax, top n_starts rays.
 * ray_best_l/j [R]; start_ray [n_starts]; X0 [n_starts][d]. */
int32_t or_discover(const or_problem *p, const double *beta, const double *lo, const double *hi,
                    int32_t R, int32_t n_pts, int32_t n_starts, uint64_t seed, uint32_t problem,
                    double *ray_best_l, int32_t *ray_best_j, int32_t *start_ray, double *X0);

/* ---- L-BFGS ---- */
/* Two-loop recursion.  S, Y: [cnt][d] in logical order (oldest first).
 * Returns the search direction p = -H_k^{-1} g (H_k the L-BFGS inverse estimate). */
void or_two_loop(int32_t d, int32_t cnt, const double *S, const double *Y, const double *g,
                 double *p);
/* Maximise l from x (in place).  Writes l, grad l, iterations, evals; returns OR_ST_*. */
int32_t or_lbfgs(const or_problem *p, const double *beta, double *x, int32_t m,
                 int32_t max_iter, double grad_tol, double *logl, double *grad,
                 int32_t *iters, int64_t *evals);
/* Newton polish with the exact Hessian; OR_E_NOTPD if H is not positive definite. */
int32_t or_newton(const or_problem *p, const double *beta, double *x, int32_t max_steps,
                  int32_t *steps);

/* ---- dedup: L-infinity leader clustering (highest l first, ties lower index) ----
 * valid[C] (nullable) excludes candidates.  rep_of[C] gets the representative's
 * candidate index (-1 for excluded); reps[] the representatives in creation order.
 * Returns the number of representatives. */
int32_t or_dedup(int32_t C, int32_t d, const double *X, const double *l, const uint8_t *valid,
                 double tau, int32_t *rep_of, int32_t *reps);

/* ---- Laplace combine ---- */
double or_log_volume(int32_t d, const double *lo, const double *hi);

/* ---- preprocessing: dimensional pathology detection ---- */
/* Section "Preprocessing: Dimensional Pathology Detection" (sensitivity
 * equation, flat and soft-nuisance criteria, analytical marginalisation,
 * algorithm summary).  Centre c_i = (a_i + b_i)/2, half-width
 * D_i = (b_i - a_i)/2, s_i = |l(c + D_i e_i) - l(c)| + |l(c - D_i e_i) - l(c)|
 * (2d + 1 evaluations).  cls[i] = 1 (flat) if s_i < eps_flat * median(s),
 * else 2 (soft nuisance) if s_i < eps_soft * max(s), else 0 (active).
 * *logz_marginal = sum over flat i of log(b_i - a_i) plus sum over soft i of
 * 1/2 log 2 pi + log(D_i / sqrt(s_i)), summed pairwise in index order (zero
 * for active i).  Readings: the median of an even count is the mean of the
 * two middle values; a flat coordinate's term is the integral of a constant
 * likelihood factor over its whole prior range, log(b_i - a_i) (the paper
 * writes log D_i); eps <= 0 selects the paper's defaults 1e-6 and 1e-3.
 * Returns OR_OK, or OR_E_INVAL for a bad box or a non-finite l at a probe. */
int32_t or_precheck(const or_problem *p, const double *beta, const double *lo, const double *hi,
                    double eps_flat, double eps_soft, double *s, int32_t *cls,
                    double *logz_marginal);
double or_mode_log_z(int32_t d, double logl, double log_det_h, double log_volume);

/* ---- the whole path ---- */
int32_t or_evidence(const or_problem *p, const double *lo, const double *hi, const or_config *cfg,
                    or_result *res);
/* the tail of or_evidence from given end points: pre-dedup, polish, filters, dedup, combine */
int32_t or_finish_points(const or_problem *p, const double *lo, const double *hi,
                         const or_config *cfg, int32_t n, const double *X, const double *l,
                         const uint8_t *valid, or_result *res);
/* reference mode set: Newton from each mu_k, then filters and dedup as in or_evidence */
int32_t or_reference_modes(const or_problem *p, const double *lo, const double *hi,
                           double dedup_tol, int32_t max_modes, or_result *res);

#ifdef __cplusplus
}
#endif
#endif
