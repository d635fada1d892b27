/*
 * sb.h -- C ABI of the MI355X (gfx950) Laplace-evidence library, version 1.
 *
 * The library computes the Bayesian evidence of a likelihood with a uniform
 * box prior by the mode-centric Laplace method of SunBURST (arXiv
 * 2601.19957):
 *
 *   log Z = logsumexp_k [ l(theta_k) + log pi(theta_k) + (d/2) log 2 pi
 *                         - (1/2) log det H_k ],    H_k = -nabla^2 l(theta_k)
 *
 * (Laplace approximation, appendix eq. "laplace"; mixture of Laplace
 * contributions, eq. "mixture-evidence"; problem statement in section 3,
 * uniform prior on the box with log pi = -log V).  Modes theta_k are found by
 * ray-bundle discovery (section "Ray Generation", "Two-Pass Sampling"),
 * batched L-BFGS (appendix "L-BFGS Optimization"), L-infinity
 * de-duplication (appendix "The L-infinity Metric") and a Newton polish
 * with the exact Hessian; log det H_k comes from a Cholesky factor
 * (appendix "Coordinate Whitening").
 *
 * Likelihood families (closed forms, theta in R^d):
 *   SB_FAMILY_GAUSS_MIX: l = c + logsumexp_k (beta_k - q_k/2),
 *       q_k = (theta-mu_k)^T P_k (theta-mu_k), beta_k = log w_k, plus
 *       (1/2) log det P_k - (d/2) log 2 pi when norm == SB_NORM_DENSITY.
 *   SB_FAMILY_STUDENT_T (K = 1): l = c + beta - ((nu+d)/2) log(1 + q/nu),
 *       beta = lgamma((nu+d)/2) - lgamma(nu/2) - (d/2) log(nu pi)
 *              + (1/2) log det P for SB_NORM_DENSITY, else 0.
 *
 * Conventions
 *  - Arrays are row-major.  Host entry points take host pointers and
 *    allocate their own device memory; *_dev entry points take device
 *    pointers, a caller-provided workspace and a HIP stream (passed as
 *    void*, hipStream_t), and never allocate.
 *  - Every call returns an sb_status.  No exception crosses the ABI.  On an
 *    error the outputs are untouched, except sb_result.log_z = NaN and, for
 *    SB_E_CAPACITY, sb_result.n_modes = the number of modes found.
 *  - Calls are deterministic: the same inputs, seed and GPU give bitwise
 *    identical outputs.  Calls on different streams are independent.
 *  - The caller owns every buffer.  sb_last_error() describes the last
 *    failure on the calling thread.
 *
 * Beyond the evidence path: the preprocessing probe for flat and weakly
 * constrained coordinates (sb_precheck_dev), the eigendecomposition-based
 * reduction at the modes for sampler handoff (sb_eig_reduce_dev), and
 * generic user likelihoods given as HIP source, compiled at run time, with
 * finite-difference derivatives and their own evidence path (sb_user_*),
 * and the building blocks of the ChiSao exploration cycle: stick detection,
 * the Hands Like Clouds and anti-convergence moves, the reseeding ray and
 * Golden Rooster's orthonormal directions (sb_chisao_*).
 */
#ifndef SB_H
#define SB_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SB_ABI_VERSION 1

typedef enum {
  SB_OK = 0,
  SB_E_INVAL = -1,       /* invalid argument (sizes, pointers, box, config) */
  SB_E_NOTPD = -2,       /* a precision matrix is asymmetric or not positive definite */
  SB_E_NOMEM = -3,       /* device allocation failed or workspace too small */
  SB_E_DEVICE = -4,      /* HIP runtime error, or no gfx950 device */
  SB_E_NOMODE = -5,      /* no mode passed the filters; log_z = -inf */
  SB_E_CAPACITY = -6,    /* more modes than max_modes; n_modes = modes found */
  SB_E_UNSUPPORTED = -7, /* valid but not supported (e.g. Student-t with K > 1) */
  SB_E_NOCONV = -8       /* an iteration stopped at its cap above its tolerance (outputs written) */
} sb_status;

typedef enum { SB_FAMILY_GAUSS_MIX = 0, SB_FAMILY_STUDENT_T = 1 } sb_family;
typedef enum { SB_NORM_PEAK_ZERO = 0, SB_NORM_DENSITY = 1 } sb_norm;
/* SB_PREC_FP64: every step in FP64.  SB_PREC_MIXED: discovery GEMM in BF16
 * with FP32 accumulation, L-BFGS bulk in FP32 (its history pairs rounded to
 * BF16 when m <= 8), then Newton polish, Hessian, Cholesky, log det and the
 * logsumexp combine in FP64. */
typedef enum { SB_PREC_FP64 = 0, SB_PREC_MIXED = 1 } sb_precision;
/* SB_DTYPE_F32_SPLIT: FP32 data whose contraction runs on the BF16 matrix
 * cores as three products of split operands (v = hi + lo, hi = bf16(v),
 * lo = bf16(v - hi); hi*hi + hi*lo + lo*hi with FP32 accumulation, about
 * 2^-16 relative per product); needs d a multiple of 8.
 * SB_DTYPE_F32_H16 (sb_lbfgs_dev, sb_lbfgs_timed_dev only): FP32 points,
 * gradients and directions with the L-BFGS history ring in BF16 (each pair
 * s, y rounded to BF16 when formed, then used and stored as rounded); m <= 8. */
typedef enum {
  SB_DTYPE_F64 = 0,
  SB_DTYPE_F32 = 1,
  SB_DTYPE_BF16 = 2,
  SB_DTYPE_F32_SPLIT = 3,
  SB_DTYPE_F32_H16 = 4
} sb_dtype;

/* Likelihood: family, normalisation and parameters.
 * log_w [K] (NULL: all weights 1), mu [K][d], prec [K][d][d] (symmetric
 * positive definite precision matrices P_k = Sigma_k^{-1}).  Host pointers
 * for sb_evidence / sb_evidence_batch, device pointers for *_dev calls. */
typedef struct {
  int32_t family, norm, d, K;
  const double *log_w;
  const double *mu;
  const double *prec;
  double nu;          /* Student-t degrees of freedom, > 0 */
  double logl_offset; /* constant c */
} sb_loglik;

/* Uniform prior box prod_i [lo_i, hi_i], lo_i < hi_i finite, [d] each. */
typedef struct {
  const double *lo, *hi;
} sb_box;

/* Run parameters.  Non-positive tolerances and max_iter select defaults:
 * grad_tol 1e-10 (FP64 bulk; the FP32 bulk of SB_PREC_MIXED stops at its
 * rounding floor), dedup_tol 1e-6 * max_i(hi_i - lo_i), dedup_tol_pre 0.25,
 * max_iter 10 d + 200.  Requires 1 <= m <= 32, 1 <= n_starts <= n_rays,
 * n_points >= 1, max_modes >= 1.  Memories up to 8 pairs are held in
 * registers during a step; larger ones are read from the history ring in
 * each loop of the two-loop recursion (same arithmetic, more traffic). */
typedef struct {
  int32_t n_rays, n_points, n_starts, m, max_iter, max_modes, precision;
  double grad_tol, dedup_tol, dedup_tol_pre;
  uint64_t seed;
} sb_config;

/* Results (host memory, caller-allocated arrays of max_modes entries; may be
 * NULL).  Modes are sorted by mode_log_z descending (ties: lexicographic). */
typedef struct {
  double log_z;
  int32_t n_modes;
  double *modes;      /* [max_modes][d] */
  double *mode_log_z; /* [max_modes] */
  double *mode_logl;  /* [max_modes] */
  double *log_det_h;  /* [max_modes], log det of H = -nabla^2 l at the mode */
  int64_t n_logl_evals; /* l-only evaluations (discovery) */
  int64_t n_grad_evals; /* l + gradient evaluations (L-BFGS, polish) */
  int64_t n_hess_evals; /* Hessian assemblies */
  int32_t iterations;   /* L-BFGS batch steps */
  int32_t n_rejected_nonpd, n_dead_starts, n_candidates, n_reps_pre;
  double seconds[8];    /* prep, discovery, bulk, dedup_pre, polish, hessian+chol, combine, total */
} sb_result;

/* ------------------------------------------------------------------ whole path */

/* Evidence of one problem (host buffers in and out).  Section 3 problem
 * statement; modules CarryTiger / GreenDragon / BendTheBow in order. */
int32_t sb_evidence(const sb_loglik *ll, const sb_box *box, const sb_config *cfg,
                    sb_result *res);

/* Evidence of n independent problems (uneven d and K), results in res[n].
 * Problem j uses ll[j], box[j] and cfg[j]; their ray/start kernels run as
 * one batch per phase. */
int32_t sb_evidence_batch(int32_t n, const sb_loglik *ll, const sb_box *box,
                          const sb_config *cfg, sb_result *res);

/* Device-resident variant of sb_evidence: ll and box hold device pointers,
 * the workspace (>= sb_evidence_workspace_bytes) is caller-owned device
 * memory; results are written to host memory in res.  The call allocates
 * nothing, on the device or the host: it launches each L-BFGS iteration
 * block directly and reads its 4-byte active count into a host stack word;
 * res->seconds holds only the total (seconds[7]).  The box is checked on the
 * device (SB_E_INVAL if some lo_i >= hi_i or a bound is not finite).  The
 * first call for a new shape runs the tile autotuner, which times its
 * candidates on this call's own workspace and keeps the choice in the
 * process-wide tile cache.  stream may be NULL (the null stream).
 * Synchronises stream. */
size_t sb_evidence_workspace_bytes(const sb_loglik *ll, const sb_config *cfg);
int32_t sb_evidence_dev(const sb_loglik *ll_dev, const sb_box *box_dev, const sb_config *cfg,
                        sb_result *res, void *workspace, size_t ws_bytes, void *stream);

/* The whole path with the ChiSao oscillation cycle as its convergence and,
 * optionally, the refinement pass of the two-pass ray sampling (section
 * "ChiSao Exploration": the oscillation cycle and CarryTiger's algorithm
 * summary; section "Two-Pass Sampling").  FP64 throughout (cfg->precision
 * must be SB_PREC_FP64, else SB_E_UNSUPPORTED).
 *
 * Discovery: the rays and coarse pass of sb_discover_dev; with n_ref > 0, per
 * ray the cells [t_j - h/2, t_j + h/2] (h = 1/n_points) of the coarse scores
 * above the ray's maximum minus ref_delta carry the density exp(l_j - l_max)
 * and n_ref more points sit at its quantiles (i + 1/2)/n_ref; each ray keeps
 * its best sample over both passes (ties: coarse first, lower index), and the
 * n_starts best rays seed the cycle.
 * Cycle, n_osc oscillations over the n_starts sample slots:
 *  1. convergence: L-BFGS (fresh history, memory cfg->m) on every active slot
 *     for at most n_conv accepted steps;
 *  2. stick detection (sb_chisao_stick_dev over the active slots, stick_tol);
 *  3. L-infinity leader dedup (radius cfg->dedup_tol_pre, default 0.25) of the
 *     stuck slots: a stuck slot in another's cluster is lost (emptied);
 *  4. not on the last oscillation, when slots were lost: with >= 5 active
 *     slots that did not converge, Repulse Monkey refills lost slot j with the
 *     best of n_reseed_pts samples on the ray (sb_chisao_reseed_dev) from
 *     unconverged slot j mod n_unconverged in a random direction; with fewer,
 *     Golden Rooster refills the lost slots round-robin over the distinct
 *     stuck peaks (l descending), each peak's slots taking QR-orthonormal
 *     directions (sb_chisao_orthonormal_dev, chunks of at most d rows) for rays
 *     from the peak; else the slots stay empty.  Golden Rooster switches off
 *     for good when the oscillation after one in which it refilled ends with no
 *     more distinct converged peaks than the one before;
 *  5. not on the last oscillation: the free slots (active, not stuck) take
 *     n_cloud Hands Like Clouds steps of n_smooth perturbations at scale sigma
 *     and n_anti anti-convergence steps (sb_chisao_explore_dev).
 * The last phase's active slots with a finite l then go through the tail of
 * sb_evidence_dev (pre-dedup, Newton polish, Hessian, Cholesky, filters,
 * dedup, combine).  Draws are Philox4x32-10 normals (cosine branch of
 * Box-Muller on the uniforms of two streams) keyed by cfg->seed, counter (slot,
 * block, 16 + 8 k + purpose, 0) on oscillation k, purpose 0 Repulse Monkey
 * directions, 2 Golden Rooster draws, 4 Hands Like Clouds perturbations
 * (index (c n_smooth + q) d + i).  With n_osc = 1 and n_ref = 0 the result is
 * that of sb_evidence_dev in FP64.  res->iterations counts the L-BFGS batch
 * steps of all phases, res->n_grad_evals also the moves' evaluations.  The
 * per-oscillation bookkeeping uses O(n_starts) bytes of host memory.
 * Workspace >= sb_evidence_chisao_workspace_bytes. */
typedef struct {
  int32_t n_osc;        /* oscillations, >= 1 (the paper's default is 3) */
  int32_t n_conv;       /* L-BFGS steps per convergence phase (<= 0: max_iter) */
  double stick_tol;     /* gradient L-infinity bound of stick detection (<= 0: 1e-6) */
  int32_t n_reseed_pts; /* samples along a reseeding ray (<= 0: 32) */
  int32_t n_cloud;      /* Hands Like Clouds steps (>= 0) */
  int32_t n_smooth;     /* perturbations per smoothed gradient (<= 0: 4) */
  double sigma;         /* smoothing scale; <= 0: half the median over coordinates of
                           the population standard deviation of the free slots */
  double alpha_cloud;   /* ascent step (<= 0: 0.01) */
  int32_t n_anti;       /* anti-convergence steps (>= 0) */
  double alpha_anti;    /* descent step (<= 0: 0.01) */
  double momentum;      /* in [0, 1) */
  int32_t n_ref;        /* refinement-pass points per ray (0: coarse pass only) */
  double ref_delta;     /* active region: l > l_max - ref_delta (<= 0: 10) */
} sb_chisao_config;
size_t sb_evidence_chisao_workspace_bytes(const sb_loglik *ll, const sb_config *cfg,
                                          const sb_chisao_config *cc);
int32_t sb_evidence_chisao_dev(const sb_loglik *ll_dev, const sb_box *box_dev,
                               const sb_config *cfg, const sb_chisao_config *cc,
                               sb_result *res, void *workspace, size_t ws_bytes, void *stream);

/* Execution context for repeated whole-path calls on one device (the
 * batching form: an iteration block of the L-BFGS bulk, 8 steps of step,
 * compaction, contraction and epilogue launches, replayed as one HIP graph).
 * sb_exec_create allocates, on the current device, a pinned host word for
 * the per-block count readback, ten timing events and room for four
 * instantiated block graphs; sb_exec_destroy frees them.
 * sb_evidence_exec_dev is sb_evidence_dev with that state: the block graph
 * for this call's buffers, model and box pointers, configuration, stream
 * and tiles is looked up in the context; a call that finds it captures and
 * instantiates nothing, a new combination captures the block once and
 * updates the least recently used executable in place (or instantiates one
 * when the update is refused).  res->seconds gets the phase times.  A NULL
 * stream cannot be captured: the blocks are then launched directly.  A
 * context is used by one call at a time (calls that share one race) and on
 * the device it was created on (else SB_E_INVAL).  sb_exec_stats writes
 * counts [4]: graphs captured, instantiated, updated in place, and block
 * graph launches, since creation. */
typedef struct sb_exec sb_exec;
int32_t sb_exec_create(sb_exec **out);
void sb_exec_destroy(sb_exec *ex);
int32_t sb_exec_stats(const sb_exec *ex, int32_t *counts);
int32_t sb_evidence_exec_dev(sb_exec *ex, const sb_loglik *ll_dev, const sb_box *box_dev,
                             const sb_config *cfg, sb_result *res, void *workspace,
                             size_t ws_bytes, void *stream);

/* --------------------------------------------------------------- single steps
 * Device pointers throughout; nothing allocates.  "model" arrays:
 *   beta [K] FP64 per-component constants written by sb_prep_dev;
 *   prec_lp, mu_lp: FP32 copies (dtype F32) or BF16 precision + FP32 mu
 *   (dtype BF16) written by sb_prep_dev when non-NULL. */
typedef struct {
  int32_t family, norm, d, K;
  const double *log_w, *mu, *prec; /* device, FP64 */
  double nu, logl_offset;
  const double *beta;              /* device [K], from sb_prep_dev */
  const void *prec_lp;             /* device [K][d][d] FP32 or BF16, or [2][K][d][d]
                                      BF16 hi then lo (dtype F32_SPLIT), or NULL */
  const float *mu_lp;              /* device [K][d] FP32, or NULL */
} sb_model_dev;

/* Problem prep (step A1): Cholesky of every P_k; writes beta[K] and
 * logdet_prec[K] (device FP64) and, when non-NULL, prec_f32 [K][d][d],
 * prec_bf16 [K][d][d] (uint16 bit patterns) and mu_f32 [K][d].
 * SB_E_NOTPD if a P_k is asymmetric (> 1e-12 relative) or not positive
 * definite.  Workspace >= sb_prep_workspace_bytes(d, K). */
size_t sb_prep_workspace_bytes(int32_t d, int32_t K);
int32_t sb_prep_dev(const sb_loglik *ll_dev, double *beta, double *logdet_prec, float *prec_f32,
                    uint16_t *prec_bf16, float *mu_f32, void *workspace, size_t ws_bytes,
                    void *stream);

/* Batched log-likelihood and gradient (step A3): for B points X [B][d]
 * (dtype F64: double; F32 or F32_SPLIT: float) writes logl [B] and, if grad != NULL,
 * grad [B][d] (same dtype).  One GEMM (X - mu_k) P_k on the matrix cores,
 * then the logsumexp / Student-t epilogue and the hand-written backward.
 * Workspace >= sb_logl_grad_workspace_bytes(d, K, B, dtype). */
size_t sb_logl_grad_workspace_bytes(int32_t d, int32_t K, int64_t B, int32_t dtype);
int32_t sb_logl_grad_dev(const sb_model_dev *m, int64_t B, const void *X, void *logl, void *grad,
                         int32_t dtype, void *workspace, size_t ws_bytes, void *stream);

/* sb_logl_grad_dev for callers that cannot allocate: code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc.  No workspace
 * argument: the contraction's scratch (Y rows and q partials, the bytes
 * sb_logl_grad_workspace_bytes(d, K, B, dtype) reports) lives in a static
 * device array of 32 MiB per GPU that the library holds until the process
 * ends (its address is looked up on the first call on each device).  Sizes
 * whose scratch exceeds 32 MiB are rejected with SB_E_NOMEM.  The call
 * allocates nothing and times no tiles (it takes the tile cached by an earlier
 * sb_logl_grad_dev of that shape, else a fixed heuristic).  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (on different
 * streams or threads) race; each call overwrites the scratch before reading
 * it, so nothing needs clearing between calls. */
int32_t sb_logl_grad_noalloc_dev(const sb_model_dev *m, int64_t B, const void *X, void *logl,
                                 void *grad, int32_t dtype, void *stream);

/* The contraction of step A3 alone, as used inside sb_logl_grad_dev and the
 * optimiser: Y [B][K*d] with Y[b][k*d + n] = sum_j P_k[n][j] (X[b][j] -
 * mu_k[j]) and per-tile partial quadratic forms qpart [B][K][*n_tiles]
 * (q_k = sum over tiles).  dtype F64, F32 or F32_SPLIT (Y, qpart FP64 or
 * FP32; *n_tiles gets the tiles' count, which depends on dtype).  qpart
 * must hold B*K*ceil(d/64) values.  For measurement and testing. */
int32_t sb_quadform_dev(const sb_model_dev *m, int64_t B, const void *X, int32_t dtype, void *Y,
                        void *qpart, int32_t *n_tiles, void *stream);

/* The contraction of listed (row, component) pairs, as the bulk's screened
 * mixture path runs it (dtype F32_SPLIT, 128 x 128 tiles): component k
 * multiplies the gcnt[k] rows listed at rows + k * cap of X [B][d] (FP32),
 * writing Y[r][k*d + n] and qpart[r][k][t] for those pairs only (Y, qpart as
 * for sb_quadform_dev; other entries untouched).  gcnt [K], rows [K][cap]
 * device int32, each row < B.  Gaussian mixtures only.  For measurement and
 * testing. */
int32_t sb_quadform_pairs_dev(const sb_model_dev *m, int64_t B, const void *X,
                              const int32_t *gcnt, const int32_t *rows, int64_t cap, void *Y,
                              void *qpart, int32_t *n_tiles, void *stream);

/* Split copy for the F32_SPLIT contraction: hi[i] = bf16(fp32(x[i])) and,
 * when lo != NULL, lo[i] = bf16(x[i] - hi[i]) (round to nearest even; uint16
 * bit patterns), for n device values.  A model's prec_lp for dtype
 * F32_SPLIT is hi of all K d x d precisions followed by lo. */
int32_t sb_split_bf16_dev(int64_t n, const double *x, uint16_t *hi, uint16_t *lo, void *stream);

/* Batched Hessian-vector product (step A3'): HV[b] = nabla^2 l(X[b]) V[b],
 * FP64.  Workspace >= sb_hvp_workspace_bytes(d, K, B). */
size_t sb_hvp_workspace_bytes(int32_t d, int32_t K, int64_t B);
int32_t sb_hvp_dev(const sb_model_dev *m, int64_t B, const double *X, const double *V, double *HV,
                   void *workspace, size_t ws_bytes, void *stream);

/* Ray-bundle discovery (step A2, section "Ray Generation" and the coarse
 * pass): R rays of the four geometries (ray r uses r mod 4) from Philox4x32-10
 * keyed by seed; l at t_j = (j + 1/2)/n_pts; per-ray argmax (ties: lowest j);
 * the n_starts rays with the highest maxima (ties: lowest ray).  dtype F64
 * evaluates in FP64, BF16 runs the GEMM in BF16 with FP32 accumulation.
 * Outputs (device): P0, P1 [R][d] FP64 endpoints (may be NULL), ray_best_l
 * [R] FP64, ray_best_j [R], start_ray [n_starts], X0 [n_starts][d] FP64.
 * Workspace >= sb_discover_workspace_bytes(d, K, R, n_pts, dtype). */
size_t sb_discover_workspace_bytes(int32_t d, int32_t K, int32_t R, int32_t n_pts, int32_t dtype);
int32_t sb_discover_dev(const sb_model_dev *m, const double *lo, const double *hi, int32_t R,
                        int32_t n_pts, int32_t n_starts, uint64_t seed, int32_t dtype,
                        double *P0, double *P1, double *ray_best_l, int32_t *ray_best_j,
                        int32_t *start_ray, double *X0, void *workspace, size_t ws_bytes,
                        void *stream);

/* Preprocessing probe (section "Preprocessing: Dimensional Pathology
 * Detection": its sensitivity equation, flat and soft-nuisance criteria,
 * analytical marginalisation and algorithm summary).  With the prior centre
 * c_i = (lo_i + hi_i)/2 and half-widths D_i = (hi_i - lo_i)/2, the model's l
 * is evaluated in FP64 at c and at c +- D_i e_i (2d + 1 points in one batch):
 * s [d] (device) gets s_i = |l(c + D_i e_i) - l(c)| + |l(c - D_i e_i) - l(c)|,
 * cls [d] (device) 1 where s_i < eps_flat * median(s) (flat), else 2 where
 * s_i < eps_soft * max(s) (soft nuisance), else 0 (active); *logz_marginal
 * (device) the sum over flat i of log(hi_i - lo_i) and over soft i of
 * 1/2 log 2 pi + log(D_i / sqrt(s_i)).  The median of an even count is the
 * mean of the middle two.  eps <= 0 selects the defaults 1e-6 (flat) and
 * 1e-3 (soft).  n_flagged [2] (host, nullable) gets the flat and soft counts.
 * lo, hi [d] are device FP64 arrays with lo < hi (not checked here: the
 * caller validates the box).  SB_E_INVAL if l is not finite at a probe point
 * (then *logz_marginal is NaN).  The call synchronises the stream.
 * Workspace >= sb_precheck_workspace_bytes(d, K). */
size_t sb_precheck_workspace_bytes(int32_t d, int32_t K);
int32_t sb_precheck_dev(const sb_model_dev *m, const double *lo, const double *hi,
                        double eps_flat, double eps_soft, double *s, int32_t *cls,
                        double *logz_marginal, int32_t *n_flagged, void *workspace,
                        size_t ws_bytes, void *stream);

/* Dimensional reduction for sampler handoff (section "Module 4:
 * GraspBirdsTail": eigendecomposition, direction classes, reduced likelihood
 * and algorithm summary).  For C symmetric n x n matrices H [C][n][n]
 * (device, FP64; H = -grad^2 l at a mode, e.g. from sb_hessian_dev; only the
 * symmetric part (H + H^T)/2 is used, H is not modified): eigval [C][n]
 * (device) the eigenvalues in descending order, V [C][n][n] (device,
 * row-major) with column i the unit eigenvector of eigval i (sign
 * arbitrary), by cyclic Jacobi in FP64 to an off-diagonal norm of at most
 * 4 n eps |H|_F.  cls [C][n] (device): 0 informative (lambda > eps_inform),
 * 1 nuisance (eps_nuisance < lambda <= eps_inform), 2 degenerate
 * (lambda <= eps_nuisance).  logz_marginal [C] (device): the sum over
 * nuisance directions of 1/2 log(2 pi / lambda) and over degenerate
 * directions of the log of the box's extent along the direction,
 * log sum_j |V_ji| (hi_j - lo_j) (lo, hi [n] device).  d_eff [C] (host,
 * nullable): informative counts; *sweeps (host, nullable): Jacobi sweeps
 * used.  The reduced likelihood of a mode theta* is
 * l(theta* + V_inform phi) on the d_eff informative coordinates phi.
 * SB_E_INVAL for bad sizes, thresholds outside 0 <= eps_nuisance <=
 * eps_inform < inf, or non-finite H; SB_E_NOCONV when some matrix is still
 * above the off-diagonal bound after 40 sweeps (every output written from the
 * last sweep, *sweeps = 40).  The call synchronises the stream.
 * Workspace >= sb_eig_reduce_workspace_bytes(C, n). */
size_t sb_eig_reduce_workspace_bytes(int32_t C, int32_t n);
int32_t sb_eig_reduce_dev(int32_t C, int32_t n, const double *H, const double *lo,
                          const double *hi, double eps_inform, double eps_nuisance,
                          double *eigval, double *V, int32_t *cls, double *logz_marginal,
                          int32_t *d_eff, int32_t *sweeps, void *workspace, size_t ws_bytes,
                          void *stream);

/* The reduced likelihood for sampler handoff (section "Module 4:
 * GraspBirdsTail": compacted likelihood, algorithm summary and exports):
 * l_red(phi) = l(theta* + V_inform phi), V_inform the first r columns of V
 * [d][ldv] (device, row-major; column i a direction, e.g. the informative
 * eigenvectors sb_eig_reduce_dev returns first, r = d_eff), theta* [d]
 * (device) the mode, phi [B][r] (device) points in the reduced coordinates.
 * Writes logl [B] (device) and, if grad_phi != NULL, grad_phi [B][r] =
 * V_inform^T grad l (device).  FP64 throughout: the points by one FP64
 * matrix-core product, then sb_logl_grad_dev's FP64 path, then the chain rule
 * by a second product.  0 <= r <= d, ldv >= max(r, 1); the model needs its
 * FP64 data.  SB_E_INVAL for bad sizes or NULL arrays, SB_E_NOMEM for a
 * short workspace.  Workspace >= sb_reduced_logl_workspace_bytes(d, K, B). */
size_t sb_reduced_logl_workspace_bytes(int32_t d, int32_t K, int64_t B);
int32_t sb_reduced_logl_dev(const sb_model_dev *m, const double *theta_star, const double *V,
                            int32_t ldv, int32_t r, int64_t B, const double *phi, double *logl,
                            double *grad_phi, void *workspace, size_t ws_bytes, void *stream);

/* Bounds of the reduced box (section "Module 4: GraspBirdsTail", exports):
 * for each of the first r columns v of V [d][ldv] (device) the interval
 * [phi_lo_i, phi_hi_i] (device [r]) of t with theta* + t v inside the box
 * [lo, hi] (device [d]): the intersection over the coordinates j with v_j != 0
 * of the t where lo_j <= theta*_j + t v_j <= hi_j (a column of zeros gives
 * [-inf, inf]; theta* outside the box an empty interval, lo > hi).  Exact
 * IEEE divisions, minima and maxima: no rounding beyond the divisions.
 * SB_E_INVAL for bad sizes or NULL arrays.  No workspace. */
int32_t sb_reduced_bounds_dev(int32_t d, const double *theta_star, const double *V, int32_t ldv,
                              int32_t r, const double *lo, const double *hi, double *phi_lo,
                              double *phi_hi, void *stream);

/* ChiSao stick detection (section "ChiSao Exploration": the oscillation
 * cycle's stick step and the CarryTiger algorithm summary).  For B samples
 * with values logl [B] and gradients grad [B][d] (device FP64), stuck [B]
 * (device) gets 1 where max_j |grad_bj| < grad_tol and logl_b >= l_max +
 * log 0.1, l_max being the largest finite logl of the batch, else 0; a
 * non-finite logl or gradient entry gives 0.  SB_E_INVAL for B < 0, d < 1,
 * a non-finite grad_tol or NULL arrays (B > 0).  Workspace >= 8 bytes. */
int32_t sb_chisao_stick_dev(int64_t B, int32_t d, const double *logl, const double *grad,
                            double grad_tol, uint8_t *stuck, void *workspace, size_t ws_bytes,
                            void *stream);

/* ChiSao reseeding ray (section "ChiSao Exploration": the Repulse Monkey /
 * Golden Rooster step shoots rays from existing samples; they are sampled as
 * the coarse pass of section "Ray Generation" samples a ray).  For each of B
 * samples X [B][d] (device FP64, in place) and direction U [B][d] (device
 * FP64, chosen by the caller: random for Repulse Monkey, orthonormal for
 * Golden Rooster), the ray runs from x to where it leaves the box [lo, hi]:
 * t_exit = min over u_i != 0 of (hi_i - x_i)/u_i (u_i > 0) or (lo_i - x_i)/u_i
 * (u_i < 0), at least 0, and 0 for u = 0.  l is evaluated in FP64 at
 * x + (t_j t_exit) u, t_j = (j + 1/2)/n_pts, and the first point of highest
 * finite l replaces x (none finite: x stays); best_l [B] (device, nullable)
 * gets that l or NaN.  SB_E_INVAL for B < 0, n_pts < 1 or NULL arrays.
 * Workspace >= sb_chisao_reseed_workspace_bytes(d, K, B, n_pts). */
size_t sb_chisao_reseed_workspace_bytes(int32_t d, int32_t K, int64_t B, int32_t n_pts);
int32_t sb_chisao_reseed_dev(const sb_model_dev *m, const double *lo, const double *hi,
                             int64_t B, double *X, const double *U, int32_t n_pts,
                             double *best_l, void *workspace, size_t ws_bytes, void *stream);

/* Golden Rooster's orthonormal ray directions (section "ChiSao Exploration":
 * the near-exhaustion refill from converged peaks uses directions made
 * orthonormal by QR).  For each of C peaks the n rows of G [C][n][d] (device
 * FP64, in place; Gaussian draws chosen by the caller) become the rows of Q in
 * G_c^T = Q R with R's diagonal positive (modified Gram-Schmidt with a second
 * projection pass, one workgroup per peak; 2 n^2 d multiply-adds per peak).  A row whose norm after removing
 * its projections on the earlier rows is at most 8 n eps (eps = 2^-52) of its
 * own norm (it depends on them), or not finite, becomes NaN, and so does every
 * later row.  SB_E_INVAL
 * unless C >= 0 and 1 <= n <= d; G may be NULL when C = 0. */
int32_t sb_chisao_orthonormal_dev(int32_t C, int32_t n, int32_t d, double *G, void *stream);

/* ChiSao moves of the samples that are not stuck (section "ChiSao
 * Exploration": the Hands Like Clouds smoothed gradient and the momentum
 * equation of the anti-convergence phase), in place on X [B][d] (device
 * FP64), stuck [B] (device, nonzero = frozen).  First n_cloud Hands Like
 * Clouds steps: step c evaluates the model's gradient at the n_smooth points
 * x + sigma z for z = Z[c][k][b] (Z [n_cloud][n_smooth][B][d] device FP64
 * standard normal draws, drawn by the caller) and moves x by alpha_cloud
 * times their mean.  Then n_anti anti-convergence steps v <- mu v - alpha
 * grad l(x), x <- x + v from v = 0.  Each move is clipped to the box
 * [lo, hi] (device [d]).  Gradients run through the FP64 path of
 * sb_logl_grad_dev (the model needs its FP64 data only).  SB_E_INVAL for
 * negative counts, n_cloud > 0 with n_smooth < 1 or Z NULL, sigma < 0 or
 * non-finite parameters; B = 0 or no steps is a no-op.  Workspace >=
 * sb_chisao_explore_workspace_bytes(d, K, B, n_smooth). */
size_t sb_chisao_explore_workspace_bytes(int32_t d, int32_t K, int64_t B, int32_t n_smooth);
int32_t sb_chisao_explore_dev(const sb_model_dev *m, const double *lo, const double *hi,
                              int64_t B, double *X, const uint8_t *stuck, int32_t n_cloud,
                              int32_t n_smooth, const double *Z, double sigma, double alpha_cloud,
                              int32_t n_anti, double alpha, double mu, void *workspace,
                              size_t ws_bytes, void *stream);

/* Generic user log-likelihoods without an analytic backward (the paper's
 * general case: any l, derivatives by finite differences; appendix "Gradient
 * and Hessian Computation" for the stencils, "Rotation Detection" for the
 * off-diagonal probe).  sb_user_compile compiles `source`, which must define
 *   __device__ double NAME(const double *x, int d, const double *params);
 * (x: one point, params: the caller's device array, may be NULL), for gfx950
 * with hipRTC on the current device and returns a handle in *out (release
 * with sb_user_release).  SB_E_INVAL if `name` is not a C identifier or the
 * source does not compile (the compiler's message is in sb_last_error);
 * SB_E_DEVICE if the code object does not load.  A handle is used on the
 * device it was compiled on.  The user function must not fault: it is run as
 * given. */
typedef struct sb_user_fn sb_user_fn;
int32_t sb_user_compile(const char *source, const char *name, sb_user_fn **out);
void sb_user_release(sb_user_fn *fn);
/* l [B] (device) = NAME(X + b d, d, params) for the rows of X [B][d] (device). */
int32_t sb_user_logl_dev(const sb_user_fn *fn, int64_t B, int32_t d, const double *X,
                         const double *params, double *l, void *stream);
/* Central finite differences at the rows of X [B][d] with step eps > 0: all
 * perturbed points of the batch in one launch of the user function, then
 * l [B], grad [B][d] ((f(x + eps e_i) - f(x - eps e_i)) / (2 eps)), hdiag [B][d]
 * ((f(x + eps e_i) - 2 f(x) + f(x - eps e_i)) / eps^2), probe_b [B]
 * ((v^T H v - mean H_ii) / (d - 1) with v = (1..1)/sqrt(d) and v^T H v the
 * second difference along v; 0 for d = 1), and, when H is not NULL, the full
 * Hessian H [B][d][d] with H_ij = (f_{++} - f_{+-} - f_{-+} + f_{--}) /
 * (4 eps^2), f_{+-} = f(x + eps e_i - eps e_j), diagonal hdiag (2d^2 + 3
 * evaluations per point; 2d + 3 without H).  Every output but H may be NULL.
 * Workspace >= sb_user_fd_workspace_bytes(B, d, H != NULL). */
size_t sb_user_fd_workspace_bytes(int64_t B, int32_t d, int32_t full);
int32_t sb_user_fd_dev(const sb_user_fn *fn, int64_t B, int32_t d, const double *X,
                       const double *params, double eps, double *l, double *grad, double *hdiag,
                       double *H, double *probe_b, void *workspace, size_t ws_bytes,
                       void *stream);
/* Laplace evidence of a user likelihood at n given modes [n][d] (device),
 * with finite-difference curvature (the geometry detection and evidence
 * calculation of module BendTheBow): per mode the diagonal H_ii and the probe
 * b from one batch (2d + 3 evaluations); where |b| > rot_tol |mean H_ii| the
 * full FD Hessian (2d^2 + 3 evaluations) and log det(-H) by Cholesky, else
 * sum log(-H_ii).  Writes logl [n], logdet [n] (device), full_used [n] (host,
 * nullable: 1 where the full Hessian was taken), then the combine of
 * sb_combine_dev: order [n], mode_log_z [n] (sorted descending), log_z [1]
 * (device), with lo, hi [d] (device) the box.  SB_E_NOTPD if -H is not
 * positive definite at some mode (outputs written, that logdet NaN).  The
 * call synchronises the stream.
 * Workspace >= sb_user_mode_evidence_workspace_bytes(n, d). */
/* The evidence path for a user likelihood, all in FP64 on the device: ray
 * discovery (the rays of sb_discover_dev, l at every sample point, per-ray
 * argmax, top n_starts rays), batched L-BFGS of sb_lbfgs_dev on central
 * finite-difference gradients with step eps (2d + 3 user evaluations per
 * row), leader de-duplication of the starts that converged inside the box,
 * and the Laplace evidence of sb_user_mode_evidence_geo_dev at the
 * representatives: both steps of the geometry detection with the default
 * sb_geometry_config (its seeds on FD gradients of step eps with cfg's m
 * and grad_tol, the probe threshold rot_tol), the curvature with step
 * eps_hess (second differences divide rounding by eps^2, so their step is
 * larger).  cfg as for
 * sb_evidence (precision ignored); defaults here: grad_tol 1e-6 (FD
 * gradients carry rounding of order eps_mach |l| / eps), dedup_tol
 * 1e-4 max_i(hi_i - lo_i).  lo, hi [d] are device arrays.  Fills res as
 * sb_evidence does (no seconds, no Newton polish: the modes are the L-BFGS end
 * points); SB_E_NOMODE if no start converged, SB_E_CAPACITY beyond
 * max_modes, SB_E_NOTPD if a representative is not a maximum.
 * Workspace >= sb_user_evidence_workspace_bytes(d, cfg). */
size_t sb_user_evidence_workspace_bytes(int32_t d, const sb_config *cfg);
int32_t sb_user_evidence_dev(const sb_user_fn *fn, int32_t d, const double *params,
                             const double *lo, const double *hi, const sb_config *cfg,
                             double eps, double eps_hess, double rot_tol, sb_result *res,
                             void *workspace, size_t ws_bytes, void *stream);
size_t sb_user_mode_evidence_workspace_bytes(int32_t n, int32_t d);
int32_t sb_user_mode_evidence_dev(const sb_user_fn *fn, int32_t n, int32_t d,
                                  const double *modes, const double *params, const double *lo,
                                  const double *hi, double eps, double rot_tol, double *logl,
                                  double *logdet, int32_t *full_used, int32_t *order,
                                  double *mode_log_z, double *log_z, void *workspace,
                                  size_t ws_bytes, void *stream);

/* Geometry detection in two steps (section "Automatic Geometry Detection",
 * the algorithm "BendTheBow Evidence Calculation" and the appendix "Rotation
 * Detection").  Step 1, the TrajectoryBank: GreenDragon's seeds of each mode,
 * theta* +- 0.9 w_i e_i (2d per mode; w_i = 1/sqrt(-H_ii) from the FD diagonal
 * at the mode; seed 2i is +, 2i + 1 is -), run batched L-BFGS on central-FD
 * gradients (step eps, memory m, n_iter steps or grad_tol); for every
 * accepted step of a seed's trajectory, in coordinates whitened by
 * sqrt(-H_ii) (du = sqrt(h) dtheta, gradient g / sqrt(h) at the step's start),
 * f_perp = |du perpendicular to the gradient| / |du|; a step counts while the
 * whitened gradient at its start is at least 1e-3 of the seed's first.  A
 * mode's f_perp is the largest over its seeds' counted steps (NaN if none).
 * f_perp > eps_rot: rotated; f_perp <= eps_axis: axis-aligned; otherwise, or
 * NaN, Step 2: the probe b of sb_user_fd_dev decides (|b| > rot_tol |mean
 * H_ii|: rotated).  Rotated modes take the full FD Hessian and its Cholesky
 * log det, the others sum log(-H_ii). */
typedef struct {
  int32_t n_iter;  /* seeds' L-BFGS steps (<= 0: max(10, 3 ceil(log2 d))) */
  int32_t m;       /* their memory (<= 0: 8; at most 32) */
  double grad_tol; /* their stopping gradient (<= 0: 1e-6) */
  double eps_axis; /* f_perp at most this: axis-aligned (<= 0: 1e-4) */
  double eps_rot;  /* f_perp above this: rotated (<= 0: 1e-2) */
  double rot_tol;  /* Step 2 threshold (>= 0) */
} sb_geometry_config;
/* Step 1 alone for n modes [n][d] with the FD diagonal hdiag [n][d] (device,
 * negative at a maximum): fperp [n] (device).  Xbank, Gbank (device, both
 * or neither; [n][2d][n_iter + 1][d]) get each seed's start and accepted
 * points and the gradients of l there, bank_len [n][2d] (device, nullable)
 * the number recorded.  Workspace >= sb_user_trajectories_workspace_bytes. */
size_t sb_user_trajectories_workspace_bytes(int32_t n, int32_t d, int32_t m);
int32_t sb_user_trajectories_dev(const sb_user_fn *fn, int32_t n, int32_t d, const double *modes,
                                 const double *params, const double *hdiag, double eps,
                                 int32_t n_iter, int32_t m, double grad_tol, double *fperp,
                                 double *Xbank, double *Gbank, int32_t *bank_len,
                                 void *workspace, size_t ws_bytes, void *stream);
/* sb_user_mode_evidence_dev with both steps: FD gradients of the
 * trajectories with step eps_grad, the diagonal, probe and full Hessian with
 * eps_hess; fperp [n] (device, nullable) and decision [n] (host, nullable: 0
 * axis-aligned by the trajectories, 1 rotated by them, 2 axis-aligned by the
 * probe, 3 rotated by it).  SB_E_NOTPD if some H_ii >= 0 or a full -H is not
 * positive definite.  Workspace >= sb_user_mode_evidence_geo_workspace_bytes. */
size_t sb_user_mode_evidence_geo_workspace_bytes(int32_t n, int32_t d,
                                                 const sb_geometry_config *gc);
int32_t sb_user_mode_evidence_geo_dev(const sb_user_fn *fn, int32_t n, int32_t d,
                                      const double *modes, const double *params,
                                      const double *lo, const double *hi, double eps_grad,
                                      double eps_hess, const sb_geometry_config *gc,
                                      double *logl, double *logdet, double *fperp,
                                      int32_t *decision, int32_t *order, double *mode_log_z,
                                      double *log_z, void *workspace, size_t ws_bytes,
                                      void *stream);

/* L-BFGS two-loop direction (appendix "L-BFGS Optimization") for B
 * independent histories: S, Y [B][m][d] in logical order (oldest first),
 * cnt [B] pairs used (0 <= cnt <= m, clamped), G [B][d] gradient of f.
 * Writes the direction P [B][d] = -H_k G.  FP64 (dtype F64) or FP32 (dtype
 * F32); 1 <= m <= 32, 1 <= d <= 4096 (SB_E_INVAL / SB_E_UNSUPPORTED). */
int32_t sb_lbfgs_direction_dev(int64_t B, int32_t d, int32_t m, const int32_t *cnt,
                               const void *S, const void *Y, const void *G, void *P,
                               int32_t dtype, void *stream);

/* Batched L-BFGS on f = -l (steps A4-A5) from X [B][d] (in place).  The
 * Armijo line search (c1 = 1e-4, halving up to 40 times), curvature skip
 * s^T y <= 1e-10 |s||y|, history reset on failure, stop at
 * ||grad l||_inf <= grad_tol or max_iter accepted steps.  Writes logl [B],
 * grad [B][d] at the final points, status [B] (1 converged, 2 stalled,
 * 3 max-iter, 4 dead) and iters [B]; *n_evals (host) gets the number of
 * l+grad evaluations.  dtype F64, F32 or F32_H16 (FP32 with the BF16 history
 * ring, m <= 8; SB_E_UNSUPPORTED beyond); the model needs prec_lp/mu_lp for
 * the FP32 forms.  Workspace >= sb_lbfgs_workspace_bytes(d, K, B, m, dtype). */
size_t sb_lbfgs_workspace_bytes(int32_t d, int32_t K, int64_t B, int32_t m, int32_t dtype);
int32_t sb_lbfgs_dev(const sb_model_dev *mdl, int64_t B, void *X, int32_t m, int32_t max_iter,
                     double grad_tol, int32_t dtype, void *logl, void *grad, int32_t *status,
                     int32_t *iters, int64_t *n_evals, void *workspace, size_t ws_bytes,
                     void *stream);

/* sb_lbfgs_dev with per-launch timing of the L-BFGS step (step A4), for
 * measuring that kernel against the HBM roofline.  Same arguments and
 * results, plus: for each of the first n_timed batch steps, step_us [n_timed]
 * (host) gets the duration of the step kernel's launch in microseconds, from
 * HIP events recorded on `stream` around it, step_rows [n_timed] (host) the
 * number of starts active when it began (B for the first step), step_full
 * [n_timed] (host) the number of starts that accepted their trial point in it
 * and end it active with a full history ring (each read and wrote the same
 * (2m + 6) d-vectors), and step_back [n_timed] (host) the number that halved
 * their step instead (each read two d-vectors and wrote one).  Entries past
 * the last step are 0.  step_bytes [n_timed] (host, nullable) gets the
 * launch's algorithmic bytes when every start active entering it accepted or
 * halved: 3 d per halving start; per accepting start with c history pairs,
 * 2 c d (ring) + 6 d plus 2 d (ring) when the new pair is stored, and
 * 2 m d (ring) + 6 d with the ring full (d-vectors of the dtype's size, ring
 * vectors of the ring's: BF16 for F32_H16); -1 for the first step and for a
 * step in which some start reset its history or stopped.  The host
 * synchronises after every timed step.  SB_E_INVAL if n_timed < 0 or, with
 * n_timed > 0, one of the four counting arrays is NULL. */
int32_t sb_lbfgs_timed_dev(const sb_model_dev *mdl, int64_t B, void *X, int32_t m,
                           int32_t max_iter, double grad_tol, int32_t dtype, void *logl,
                           void *grad, int32_t *status, int32_t *iters, int64_t *n_evals,
                           void *workspace, size_t ws_bytes, void *stream, int32_t n_timed,
                           float *step_us, int32_t *step_rows, int32_t *step_full,
                           int32_t *step_back, double *step_bytes);

/* L-infinity leader de-duplication (step A7): candidates X [C][d] (FP64 or
 * FP32 per dtype) with values l [C] (same dtype) and valid [C] (nullable,
 * nonzero = candidate).  Visiting order l descending, ties lower index;
 * each candidate joins the first representative within tau, else founds
 * one.  Writes rep_of [C] (representative index, -1 if invalid) and reps
 * [max_reps]; *n_reps (host) = representatives found (SB_E_CAPACITY if more
 * than max_reps).  Workspace >= sb_dedup_workspace_bytes(C). */
size_t sb_dedup_workspace_bytes(int32_t C);
int32_t sb_dedup_dev(int32_t C, int32_t d, const void *X, const void *l, const uint8_t *valid,
                     double tau, int32_t dtype, int32_t *rep_of, int32_t *reps, int32_t max_reps,
                     int32_t *n_reps, void *workspace, size_t ws_bytes, void *stream);

/* Hessian assembly (step A8): H [C][d][d] = -nabla^2 l at X [C][d], FP64,
 * symmetrised; assembled from the same GEMM and epilogue as sb_hvp_dev with
 * V = I.  Workspace >= sb_hessian_workspace_bytes(d, K, C). */
size_t sb_hessian_workspace_bytes(int32_t d, int32_t K, int32_t C);
int32_t sb_hessian_dev(const sb_model_dev *m, int32_t C, const double *X, double *H,
                       void *workspace, size_t ws_bytes, void *stream);

/* Batched FP64 Cholesky and log det (step A9): A [C][n][n] SPD (read; only
 * the lower triangle is used) -> L [C][n][n] lower factor (may alias A),
 * logdet [C] = 2 sum log L_ii (pairwise), info [C] = 0 or the 1-based column
 * whose pivot was not positive (then logdet = NaN). */
int32_t sb_cholesky_logdet_dev(int32_t C, int32_t n, const double *A, double *L, double *logdet,
                               int32_t *info, void *stream);
/* Solve L L^T x = b for C right-hand sides b [C][n] with factors L [C][n][n]. */
int32_t sb_cholesky_solve_dev(int32_t C, int32_t n, const double *L, const double *b, double *x,
                              void *stream);

/* Laplace combine (step A10): log Z_k = logl_k - log V + (d/2) log 2 pi -
 * (1/2) logdet_k for n modes, sorted descending (ties: lexicographic in
 * modes [n][d]), log Z = logsumexp in that order.  Device inputs; writes
 * order [n] (sorted position -> input index), mode_log_z [n] (sorted) and
 * log_z [1]. */
int32_t sb_combine_dev(int32_t n, int32_t d, const double *lo, const double *hi,
                       const double *logl, const double *logdet, const double *modes,
                       int32_t *order, double *mode_log_z, double *log_z, void *stream);

/* ------------------------------------------------------------------- misc */
const char *sb_status_string(int32_t status);
const char *sb_last_error(void); /* thread-local; "" if none */
int32_t sb_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SB_H */
