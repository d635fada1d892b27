/*
 * CPU oracle for the Laplace-evidence hot path -- TEST INFRASTRUCTURE ONLY
 * (see oracle.h).  Plain FP64 loops written from the paper's definitions;
 * every function names the passage it follows.  Never linked into, loaded
 * by, or called from the product library.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LOG_2PI 1.8378770664093454835606594728112

/* ------------------------------------------------------------------ sums */

/* Pairwise summation: blocks of <= 8 summed left to right, halves added. */
double or_pairwise_sum(const double *x, int64_t n) {
  if (n <= 8) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i];
    return s;
  }
  int64_t h = n / 2;
  return or_pairwise_sum(x, h) + or_pairwise_sum(x + h, n - h);
}

/* Stable log-sum-exp (appendix "Log-Sum-Exp Stability"): x_max + log sum e^(x - x_max),
 * the sum taken in the order given. */
double or_logsumexp(const double *x, int32_t n) {
  if (n <= 0) return -INFINITY;
  double mx = -INFINITY;
  for (int32_t i = 0; i < n; ++i)
    if (x[i] > mx) mx = x[i];
  if (mx == -INFINITY || mx == INFINITY) return mx;
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += exp(x[i] - mx);
  return mx + log(s);
}

static double norm_inf(int32_t n, const double *x) {
  double m = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    double a = fabs(x[i]);
    if (!(a <= m)) m = a; /* NaN propagates */
  }
  return m;
}

static double dot(int32_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* --------------------------------------------------------- linear algebra */

/* Cholesky A = L L^T, column by column (the whitening factor of the appendix
 * "Coordinate Whitening"; log det from its diagonal). */
int32_t or_cholesky(int32_t n, const double *A, double *L) {
  memset(L, 0, sizeof(double) * (size_t)n * (size_t)n);
  for (int32_t j = 0; j < n; ++j) {
    const double *Lj = L + (size_t)j * n;
    double s = A[(size_t)j * n + j];
    for (int32_t k = 0; k < j; ++k) s -= Lj[k] * Lj[k];
    if (!(s > 0.0)) return j + 1;
    double ljj = sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int32_t i = j + 1; i < n; ++i) {
      const double *Li = L + (size_t)i * n;
      double t = A[(size_t)i * n + j];
      for (int32_t k = 0; k < j; ++k) t -= Li[k] * Lj[k];
      L[(size_t)i * n + j] = t / ljj;
    }
  }
  return 0;
}

/* log det A = 2 sum_i log L_ii (pairwise sum of the logs). */
double or_logdet_from_chol(int32_t n, const double *L) {
  double *lg = (double *)malloc(sizeof(double) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) lg[i] = log(L[(size_t)i * n + i]);
  double s = or_pairwise_sum(lg, n);
  free(lg);
  return 2.0 * s;
}

void or_chol_solve(int32_t n, const double *L, const double *b, double *x) {
  /* forward: L z = b */
  for (int32_t i = 0; i < n; ++i) {
    double t = b[i];
    for (int32_t k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * x[k];
    x[i] = t / L[(size_t)i * n + i];
  }
  /* backward: L^T x = z */
  for (int32_t i = n - 1; i >= 0; --i) {
    double t = x[i];
    for (int32_t k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * x[k];
    x[i] = t / L[(size_t)i * n + i];
  }
}

/* ------------------------------------------------------ likelihood family */

int32_t or_validate_problem(const or_problem *p) {
  if (!p) return OR_E_INVAL;
  if (p->d < 1 || p->K < 1) return OR_E_INVAL;
  if (p->family != OR_FAMILY_GAUSS_MIX && p->family != OR_FAMILY_STUDENT_T) return OR_E_INVAL;
  if (p->norm != OR_NORM_PEAK_ZERO && p->norm != OR_NORM_DENSITY) return OR_E_INVAL;
  if (!p->mu || !p->prec) return OR_E_INVAL;
  if (p->family == OR_FAMILY_STUDENT_T) {
    if (p->K != 1) return OR_E_UNSUPPORTED;
    if (!(p->nu > 0.0) || !isfinite(p->nu)) return OR_E_INVAL;
  }
  if (!isfinite(p->logl_offset)) return OR_E_INVAL;
  const int64_t d = p->d;
  for (int64_t i = 0; i < (int64_t)p->K * d; ++i)
    if (!isfinite(p->mu[i])) return OR_E_INVAL;
  if (p->log_w)
    for (int32_t k = 0; k < p->K; ++k)
      if (!isfinite(p->log_w[k])) return OR_E_INVAL;
  for (int32_t k = 0; k < p->K; ++k) {
    const double *P = p->prec + (size_t)k * d * d;
    double mx = 0.0;
    for (int64_t i = 0; i < d * d; ++i) {
      if (!isfinite(P[i])) return OR_E_INVAL;
      if (fabs(P[i]) > mx) mx = fabs(P[i]);
    }
    for (int64_t i = 0; i < d; ++i)
      for (int64_t j = i + 1; j < d; ++j)
        if (fabs(P[i * d + j] - P[j * d + i]) > 1e-12 * mx) return OR_E_NOTPD;
  }
  return OR_OK;
}

/* Per-component constants.  Gaussian mixture: l = c + logsumexp_k(beta_k - q_k/2)
 * with q_k = (x-mu_k)^T P_k (x-mu_k) and beta_k = log w_k plus, for a normalised
 * density, (1/2) log det P_k - (d/2) log 2 pi.  Student-t (density):
 * beta = lgamma((nu+d)/2) - lgamma(nu/2) - (d/2) log(nu pi) + (1/2) log det P. */
int32_t or_prep(const or_problem *p, double *beta, double *logdet_prec) {
  const int32_t d = p->d;
  double *L = (double *)malloc(sizeof(double) * (size_t)d * d);
  if (!L) return OR_E_NOMEM;
  for (int32_t k = 0; k < p->K; ++k) {
    if (or_cholesky(d, p->prec + (size_t)k * d * d, L) != 0) {
      free(L);
      return OR_E_NOTPD;
    }
    double ld = or_logdet_from_chol(d, L);
    if (logdet_prec) logdet_prec[k] = ld;
    double b = 0.0;
    if (p->family == OR_FAMILY_GAUSS_MIX) {
      b = p->log_w ? p->log_w[k] : 0.0;
      if (p->norm == OR_NORM_DENSITY) b += 0.5 * ld - 0.5 * d * LOG_2PI;
    } else if (p->norm == OR_NORM_DENSITY) {
      b = lgamma(0.5 * (p->nu + d)) - lgamma(0.5 * p->nu) - 0.5 * d * log(p->nu * M_PI) + 0.5 * ld;
    }
    beta[k] = b;
  }
  free(L);
  return OR_OK;
}

/* u = P (x - mu), q = (x-mu)^T u, for one component. delta = x - mu formed first. */
static double quad_form(int32_t d, const double *P, const double *mu, const double *x,
                        double *delta, double *u) {
  for (int32_t i = 0; i < d; ++i) delta[i] = x[i] - mu[i];
  for (int32_t i = 0; i < d; ++i) u[i] = dot(d, P + (size_t)i * d, delta);
  return dot(d, delta, u);
}

/* l and nabla l at one point.  Work arrays: a[K], U[K][d], delta[d]. */
static double logl_one(const or_problem *p, const double *beta, const double *x, double *grad,
                       double *a, double *U, double *delta, double *r) {
  const int32_t d = p->d, K = p->K;
  if (p->family == OR_FAMILY_STUDENT_T) {
    double q = quad_form(d, p->prec, p->mu, x, delta, U);
    double nd = p->nu + d;
    double l = p->logl_offset + beta[0] - 0.5 * nd * log1p(q / p->nu);
    if (grad) {
      double s = nd / (p->nu + q);
      for (int32_t i = 0; i < d; ++i) grad[i] = -s * U[i];
    }
    return l;
  }
  for (int32_t k = 0; k < K; ++k) {
    double q = quad_form(d, p->prec + (size_t)k * d * d, p->mu + (size_t)k * d, x, delta,
                         U + (size_t)k * d);
    a[k] = beta[k] - 0.5 * q;
  }
  double lse = or_logsumexp(a, K);
  if (grad) {
    for (int32_t k = 0; k < K; ++k) r[k] = exp(a[k] - lse);
    for (int32_t i = 0; i < d; ++i) {
      double s = 0.0;
      for (int32_t k = 0; k < K; ++k) s += r[k] * U[(size_t)k * d + i];
      grad[i] = -s;
    }
  }
  return p->logl_offset + lse;
}

typedef struct {
  double *a, *U, *delta, *r, *g;
} work_t;

static int work_alloc(work_t *w, int32_t d, int32_t K) {
  w->a = (double *)malloc(sizeof(double) * K);
  w->r = (double *)malloc(sizeof(double) * K);
  w->U = (double *)malloc(sizeof(double) * (size_t)K * d);
  w->delta = (double *)malloc(sizeof(double) * d);
  w->g = (double *)malloc(sizeof(double) * d);
  return w->a && w->r && w->U && w->delta && w->g;
}
static void work_free(work_t *w) {
  free(w->a); free(w->r); free(w->U); free(w->delta); free(w->g);
}

void or_logl(const or_problem *p, const double *beta, int64_t B, const double *X, double *logl,
             double *grad) {
  work_t w;
  work_alloc(&w, p->d, p->K);
  for (int64_t b = 0; b < B; ++b)
    logl[b] = logl_one(p, beta, X + b * p->d, grad ? grad + b * p->d : NULL, w.a, w.U, w.delta,
                       w.r);
  work_free(&w);
}

/* nabla^2 l at x applied to v:
 *  mixture:   sum_k r_k (u_k u_k^T v - P_k v) - g g^T v   (u_k = P_k (x-mu_k), g = nabla l)
 *  Student-t: -((nu+d)/(nu+q)) P v + (2(nu+d)/(nu+q)^2) u u^T v */
static void hvp_one(const or_problem *p, const double *beta, const double *x, const double *v,
                    double *hv, work_t *w) {
  const int32_t d = p->d, K = p->K;
  if (p->family == OR_FAMILY_STUDENT_T) {
    double q = quad_form(d, p->prec, p->mu, x, w->delta, w->U);
    double nd = p->nu + d, den = p->nu + q;
    double uv = dot(d, w->U, v);
    for (int32_t i = 0; i < d; ++i) {
      double pv = dot(d, p->prec + (size_t)i * d, v);
      hv[i] = -(nd / den) * pv + (2.0 * nd / (den * den)) * w->U[i] * uv;
    }
    return;
  }
  logl_one(p, beta, x, w->g, w->a, w->U, w->delta, w->r);
  double gv = dot(d, w->g, v);
  for (int32_t i = 0; i < d; ++i) hv[i] = -w->g[i] * gv;
  for (int32_t k = 0; k < K; ++k) {
    const double *Pk = p->prec + (size_t)k * d * d;
    const double *uk = w->U + (size_t)k * d;
    double uv = dot(d, uk, v);
    for (int32_t i = 0; i < d; ++i) hv[i] += w->r[k] * (uk[i] * uv - dot(d, Pk + (size_t)i * d, v));
  }
}

void or_hvp(const or_problem *p, const double *beta, int64_t B, const double *X, const double *V,
            double *HV) {
  work_t w;
  work_alloc(&w, p->d, p->K);
  for (int64_t b = 0; b < B; ++b)
    hvp_one(p, beta, X + b * p->d, V + b * p->d, HV + b * p->d, &w);
  work_free(&w);
}

/* H = -nabla^2 l(x): the observed information at a mode (Laplace section). */
void or_neg_hessian(const or_problem *p, const double *beta, const double *x, double *H) {
  const int32_t d = p->d, K = p->K;
  work_t w;
  work_alloc(&w, d, K);
  if (p->family == OR_FAMILY_STUDENT_T) {
    double q = quad_form(d, p->prec, p->mu, x, w.delta, w.U);
    double nd = p->nu + d, den = p->nu + q;
    for (int32_t i = 0; i < d; ++i)
      for (int32_t j = 0; j < d; ++j)
        H[(size_t)i * d + j] = (nd / den) * p->prec[(size_t)i * d + j] -
                               (2.0 * nd / (den * den)) * w.U[i] * w.U[j];
  } else {
    logl_one(p, beta, x, w.g, w.a, w.U, w.delta, w.r);
    for (int32_t i = 0; i < d; ++i)
      for (int32_t j = 0; j < d; ++j) {
        double s = w.g[i] * w.g[j];
        for (int32_t k = 0; k < K; ++k) {
          const double *uk = w.U + (size_t)k * d;
          s += w.r[k] * (p->prec[(size_t)k * d * d + (size_t)i * d + j] - uk[i] * uk[j]);
        }
        H[(size_t)i * d + j] = s;
      }
  }
  /* symmetrise */
  for (int32_t i = 0; i < d; ++i)
    for (int32_t j = i + 1; j < d; ++j) {
      double s = 0.5 * (H[(size_t)i * d + j] + H[(size_t)j * d + i]);
      H[(size_t)i * d + j] = s;
      H[(size_t)j * d + i] = s;
    }
  work_free(&w);
}

/* ------------------------------------------------------------------- RNG */

/* Philox4x32-10: ten rounds of two 32x32->64 multiplies and xors, the key
 * bumped by the Weyl constants between rounds (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Word i of stream `stream` for ray `ray`: counter (ray, i/4, stream, problem),
 * key (seed low, seed high), output word i%4. */
uint32_t or_rng_word(uint64_t seed, uint32_t problem, uint32_t ray, uint32_t stream, uint32_t i) {
  uint32_t ctr[4] = {ray, i / 4u, stream, problem};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  or_philox4x32_10(ctr, key, out);
  return out[i % 4u];
}

/* Uniform double in [0,1) from the two words of half-block i (53 random bits). */
double or_rng_uniform(uint64_t seed, uint32_t problem, uint32_t ray, uint32_t stream, uint32_t i) {
  uint32_t ctr[4] = {ray, i / 2u, stream, problem};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  or_philox4x32_10(ctr, key, out);
  uint32_t a = out[2u * (i % 2u)], b = out[2u * (i % 2u) + 1u];
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------- discovery */

/* Ray endpoints (section "Ray Generation"): geometry r mod 4:
 *  0 vertex-to-vertex, 1 vertex-to-edge-midpoint, 2 wall-to-wall along a
 *  random axis, 3 sunburst from the box centre along a uniform direction to
 *  the box boundary.  Randomness: streams 0 and 1 for the two endpoints,
 *  stream 2 word 0 for the axis. */
void or_rays(int32_t d, const double *lo, const double *hi, int32_t R, uint64_t seed,
             uint32_t problem, double *P0, double *P1) {
  for (int32_t r = 0; r < R; ++r) {
    double *p = P0 + (size_t)r * d, *q = P1 + (size_t)r * d;
    int g = r % 4;
    uint32_t axis = (uint32_t)(((uint64_t)or_rng_word(seed, problem, r, 2, 0) * (uint64_t)d) >> 32);
    if (g == 0 || g == 1) {
      for (int32_t i = 0; i < d; ++i) {
        p[i] = (or_rng_word(seed, problem, r, 0, i) & 1u) ? hi[i] : lo[i];
        q[i] = (or_rng_word(seed, problem, r, 1, i) & 1u) ? hi[i] : lo[i];
      }
      if (g == 1) q[axis] = 0.5 * (lo[axis] + hi[axis]);
    } else if (g == 2) {
      for (int32_t i = 0; i < d; ++i) {
        p[i] = lo[i] + or_rng_uniform(seed, problem, r, 0, i) * (hi[i] - lo[i]);
        q[i] = lo[i] + or_rng_uniform(seed, problem, r, 1, i) * (hi[i] - lo[i]);
      }
      p[axis] = lo[axis];
      q[axis] = hi[axis];
    } else {
      double nrm2 = 0.0;
      for (int32_t i = 0; i < d; ++i) {
        double u1 = or_rng_uniform(seed, problem, r, 0, i);
        double u2 = or_rng_uniform(seed, problem, r, 1, i);
        double z = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2); /* Box-Muller */
        q[i] = z;
        nrm2 += z * z;
      }
      double nrm = sqrt(nrm2);
      double texit = INFINITY;
      for (int32_t i = 0; i < d; ++i) {
        double c = 0.5 * (lo[i] + hi[i]);
        double u = nrm > 0.0 ? q[i] / nrm : (i == 0 ? 1.0 : 0.0);
        q[i] = u;
        double t = INFINITY;
        if (u > 0.0) t = (hi[i] - c) / u;
        else if (u < 0.0) t = (lo[i] - c) / u;
        if (t < texit) texit = t;
      }
      for (int32_t i = 0; i < d; ++i) {
        double c = 0.5 * (lo[i] + hi[i]);
        double u = q[i];
        p[i] = c;
        q[i] = c + texit * u;
      }
    }
  }
}

typedef struct {
  double key;
  int32_t idx;
} keyidx_t;

/* descending key, ascending index; NaN sorts last */
static int cmp_desc(const void *A, const void *B) {
  const keyidx_t *a = (const keyidx_t *)A, *b = (const keyidx_t *)B;
  double ka = isnan(a->key) ? -INFINITY : a->key, kb = isnan(b->key) ? -INFINITY : b->key;
  if (ka > kb) return -1;
  if (ka < kb) return 1;
  return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Coarse pass (section "Two-Pass Sampling"): l at t_j = (j+1/2)/n_pts along
 * each ray; keep each ray's argmax (ties: lowest j) and seed from the
 * n_starts rays with the highest maxima (ties: lowest ray index). */
int32_t or_discover(const or_problem *p, const double *beta, const double *lo, const double *hi,
                    int32_t R, int32_t n_pts, int32_t n_starts, uint64_t seed, uint32_t problem,
                    double *ray_best_l, int32_t *ray_best_j, int32_t *start_ray, double *X0) {
  const int32_t d = p->d;
  if (n_starts > R) return OR_E_INVAL;
  double *P0 = (double *)malloc(sizeof(double) * (size_t)R * d);
  double *P1 = (double *)malloc(sizeof(double) * (size_t)R * d);
  keyidx_t *ki = (keyidx_t *)malloc(sizeof(keyidx_t) * (size_t)R);
  if (!P0 || !P1 || !ki) {
    free(P0); free(P1); free(ki);
    return OR_E_NOMEM;
  }
  or_rays(d, lo, hi, R, seed, problem, P0, P1);
#pragma omp parallel
  {
    work_t w;
    work_alloc(&w, d, p->K);
    double *x = (double *)malloc(sizeof(double) * d);
#pragma omp for schedule(static)
    for (int32_t r = 0; r < R; ++r) {
      const double *a = P0 + (size_t)r * d, *b = P1 + (size_t)r * d;
      double best = -INFINITY;
      int32_t bj = 0;
      for (int32_t j = 0; j < n_pts; ++j) {
        double t = (j + 0.5) / n_pts;
        for (int32_t i = 0; i < d; ++i) x[i] = a[i] + t * (b[i] - a[i]);
        double l = logl_one(p, beta, x, NULL, w.a, w.U, w.delta, w.r);
        if (l > best) {
          best = l;
          bj = j;
        }
      }
      ray_best_l[r] = best;
      ray_best_j[r] = bj;
    }
    free(x);
    work_free(&w);
  }
  for (int32_t r = 0; r < R; ++r) {
    ki[r].key = ray_best_l[r];
    ki[r].idx = r;
  }
  qsort(ki, (size_t)R, sizeof(keyidx_t), cmp_desc);
  for (int32_t s = 0; s < n_starts; ++s) {
    int32_t r = ki[s].idx;
    start_ray[s] = r;
    double t = (ray_best_j[r] + 0.5) / n_pts;
    const double *a = P0 + (size_t)r * d, *b = P1 + (size_t)r * d;
    for (int32_t i = 0; i < d; ++i) X0[(size_t)s * d + i] = a[i] + t * (b[i] - a[i]);
  }
  free(P0); free(P1); free(ki);
  return OR_OK;
}

/* ---------------------------------------------------------------- L-BFGS */

/* Two-loop recursion exactly as in the appendix "L-BFGS Optimization":
 * backward loop (newest to oldest) alpha_i = rho_i s_i^T q, q -= alpha_i y_i;
 * r = gamma q with gamma = s^T y / y^T y of the newest pair; forward loop
 * beta = rho_i y_i^T r, r += s_i (alpha_i - beta); direction p = -r. */
void or_two_loop(int32_t d, int32_t cnt, const double *S, const double *Y, const double *g,
                 double *p) {
  double *q = (double *)malloc(sizeof(double) * d);
  double alpha[64], rho[64];
  for (int32_t i = 0; i < d; ++i) q[i] = g[i];
  for (int32_t j = cnt - 1; j >= 0; --j) {
    const double *s = S + (size_t)j * d, *y = Y + (size_t)j * d;
    rho[j] = 1.0 / dot(d, y, s);
    alpha[j] = rho[j] * dot(d, s, q);
    for (int32_t i = 0; i < d; ++i) q[i] -= alpha[j] * y[i];
  }
  double gamma = 1.0;
  if (cnt > 0) {
    const double *s = S + (size_t)(cnt - 1) * d, *y = Y + (size_t)(cnt - 1) * d;
    gamma = dot(d, s, y) / dot(d, y, y);
  }
  for (int32_t i = 0; i < d; ++i) q[i] *= gamma; /* q now holds r */
  for (int32_t j = 0; j < cnt; ++j) {
    const double *s = S + (size_t)j * d, *y = Y + (size_t)j * d;
    double b = rho[j] * dot(d, y, q);
    for (int32_t i = 0; i < d; ++i) q[i] += s[i] * (alpha[j] - b);
  }
  for (int32_t i = 0; i < d; ++i) p[i] = -q[i];
  free(q);
}

/* L-BFGS on f = -l (appendix "L-BFGS Optimization", batched in the paper;
 * here one start at a time).  Readings where the paper is silent: the first
 * step (or a step after a history reset) is -grad f / max(1, ||grad f||_inf);
 * Armijo sufficient decrease with c1 = 1e-4, alpha = 1, 1/2, ..., 2^-40; a
 * failed search clears the history and retries steepest descent once, then
 * the start is stalled; a pair is stored only if s^T y > 1e-10 |s| |y|; stop
 * when ||grad l||_inf <= grad_tol or after max_iter accepted steps. */
int32_t or_lbfgs(const or_problem *p, const double *beta, double *x, int32_t m,
                 int32_t max_iter, double grad_tol, double *logl, double *grad,
                 int32_t *iters, int64_t *evals) {
  const int32_t d = p->d;
  work_t w;
  work_alloc(&w, d, p->K);
  double *S = (double *)malloc(sizeof(double) * (size_t)m * d);
  double *Y = (double *)malloc(sizeof(double) * (size_t)m * d);
  double *g = (double *)malloc(sizeof(double) * d);   /* grad f */
  double *gl = (double *)malloc(sizeof(double) * d);  /* grad l at x */
  double *pd = (double *)malloc(sizeof(double) * d);
  double *xt = (double *)malloc(sizeof(double) * d);
  double *glt = (double *)malloc(sizeof(double) * d);
  double *sv = (double *)malloc(sizeof(double) * d);
  double *yv = (double *)malloc(sizeof(double) * d);
  int32_t cnt = 0, it = 0, status = OR_ST_MAXITER;
  int64_t ev = 0;
  double l = logl_one(p, beta, x, gl, w.a, w.U, w.delta, w.r);
  ++ev;
  if (!isfinite(l) || !isfinite(norm_inf(d, gl))) {
    status = OR_ST_DEAD;
    goto done;
  }
  double f = -l;
  for (int32_t i = 0; i < d; ++i) g[i] = -gl[i];
  for (;;) {
    double gn = norm_inf(d, gl);
    if (gn <= grad_tol) {
      status = OR_ST_CONVERGED;
      break;
    }
    if (it >= max_iter) {
      status = OR_ST_MAXITER;
      break;
    }
    double gtp;
    if (cnt > 0) {
      or_two_loop(d, cnt, S, Y, g, pd);
      gtp = dot(d, g, pd);
    } else {
      gtp = 0.0;
    }
    if (cnt == 0 || !(gtp < 0.0)) {
      cnt = 0;
      double sc = 1.0 / (gn > 1.0 ? gn : 1.0);
      for (int32_t i = 0; i < d; ++i) pd[i] = -g[i] * sc;
      gtp = dot(d, g, pd);
    }
    int accepted = 0;
    double alpha = 1.0, lt = 0.0;
    for (int32_t ls = 0; ls <= 40; ++ls) {
      for (int32_t i = 0; i < d; ++i) xt[i] = x[i] + alpha * pd[i];
      lt = logl_one(p, beta, xt, glt, w.a, w.U, w.delta, w.r);
      ++ev;
      double ft = -lt;
      if (isfinite(ft) && ft <= f + 1e-4 * alpha * gtp) {
        accepted = 1;
        break;
      }
      alpha *= 0.5;
    }
    if (!accepted) {
      if (cnt > 0) {
        cnt = 0;
        continue;
      }
      status = OR_ST_STALLED;
      break;
    }
    /* s = xt - x, y = grad f(xt) - grad f(x), with grad f = -grad l */
    for (int32_t i = 0; i < d; ++i) {
      sv[i] = xt[i] - x[i];
      yv[i] = -glt[i] - g[i];
    }
    double sy = dot(d, sv, yv), ss = dot(d, sv, sv), yy = dot(d, yv, yv);
    if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
      if (cnt == m) { /* drop the oldest pair */
        memmove(S, S + d, sizeof(double) * (size_t)(m - 1) * d);
        memmove(Y, Y + d, sizeof(double) * (size_t)(m - 1) * d);
        cnt = m - 1;
      }
      memcpy(S + (size_t)cnt * d, sv, sizeof(double) * d);
      memcpy(Y + (size_t)cnt * d, yv, sizeof(double) * d);
      ++cnt;
    }
    for (int32_t i = 0; i < d; ++i) {
      gl[i] = glt[i];
      g[i] = -glt[i];
    }
    memcpy(x, xt, sizeof(double) * d);
    f = -lt;
    l = lt;
    ++it;
  }
done:
  if (logl) *logl = l;
  if (grad) memcpy(grad, gl, sizeof(double) * d);
  if (iters) *iters = it;
  if (evals) *evals = ev;
  free(S); free(Y); free(g); free(gl); free(pd); free(xt); free(glt); free(sv); free(yv);
  work_free(&w);
  return status;
}

/* Newton polish with the exact H = -nabla^2 l: x += H^{-1} nabla l until
 * ||dx||_inf <= 1e-14 max(1, ||x||_inf), at most max_steps steps. */
int32_t or_newton(const or_problem *p, const double *beta, double *x, int32_t max_steps,
                  int32_t *steps) {
  const int32_t d = p->d;
  double *H = (double *)malloc(sizeof(double) * (size_t)d * d);
  double *L = (double *)malloc(sizeof(double) * (size_t)d * d);
  double *g = (double *)malloc(sizeof(double) * d);
  double *dx = (double *)malloc(sizeof(double) * d);
  double l;
  int32_t st = OR_OK, it;
  for (it = 0; it < max_steps; ++it) {
    or_logl(p, beta, 1, x, &l, g);
    or_neg_hessian(p, beta, x, H);
    if (or_cholesky(d, H, L) != 0) {
      st = OR_E_NOTPD;
      break;
    }
    or_chol_solve(d, L, g, dx);
    for (int32_t i = 0; i < d; ++i) x[i] += dx[i];
    double xn = norm_inf(d, x);
    if (norm_inf(d, dx) <= 1e-14 * (xn > 1.0 ? xn : 1.0)) {
      ++it;
      break;
    }
  }
  if (steps) *steps = it;
  free(H); free(L); free(g); free(dx);
  return st;
}

/* ----------------------------------------------------------------- dedup */

/* L-infinity leader clustering (ChiSao dedup, GreenDragon dedup; appendix
 * "The L-infinity Metric"): candidates visited by l descending (ties: lower
 * index); each joins the first representative within tau, else founds one. */
int32_t or_dedup(int32_t C, int32_t d, const double *X, const double *l, const uint8_t *valid,
                 double tau, int32_t *rep_of, int32_t *reps) {
  keyidx_t *ki = (keyidx_t *)malloc(sizeof(keyidx_t) * (size_t)(C > 0 ? C : 1));
  int32_t n = 0;
  for (int32_t c = 0; c < C; ++c) {
    rep_of[c] = -1;
    if (valid && !valid[c]) continue;
    ki[n].key = l[c];
    ki[n].idx = c;
    ++n;
  }
  qsort(ki, (size_t)n, sizeof(keyidx_t), cmp_desc);
  int32_t nrep = 0;
  for (int32_t t = 0; t < n; ++t) {
    int32_t c = ki[t].idx, joined = -1;
    for (int32_t r = 0; r < nrep && joined < 0; ++r) {
      const double *a = X + (size_t)c * d, *b = X + (size_t)reps[r] * d;
      double dist = 0.0;
      for (int32_t i = 0; i < d; ++i) {
        double e = fabs(a[i] - b[i]);
        if (e > dist) dist = e;
      }
      if (dist <= tau) joined = reps[r];
    }
    if (joined < 0) {
      reps[nrep++] = c;
      rep_of[c] = c;
    } else {
      rep_of[c] = joined;
    }
  }
  free(ki);
  return nrep;
}

/* --------------------------------------------------------------- combine */

/* log V = sum_i log(b_i - a_i), pairwise. */
double or_log_volume(int32_t d, const double *lo, const double *hi) {
  double *t = (double *)malloc(sizeof(double) * d);
  for (int32_t i = 0; i < d; ++i) t[i] = log(hi[i] - lo[i]);
  double s = or_pairwise_sum(t, d);
  free(t);
  return s;
}

/* Laplace evidence of one mode with the uniform prior (appendix eq. for
 * log Z with log pi; prior density 1/V):
 *   log Z_k = l(theta*) - log V + (d/2) log 2 pi - (1/2) log det H. */
/* ------------------------------------------------------- preprocessing */

static int cmp_double(const void *A, const void *B) {
  const double a = *(const double *)A, b = *(const double *)B;
  return (a > b) - (a < b);
}

/* Section "Preprocessing: Dimensional Pathology Detection", in the order of
 * its algorithm summary: the centre, l there, the two boundary probes of each
 * coordinate, the median and maximum of the sensitivities, the two classes,
 * the marginal log-evidence of the flagged coordinates. */
int32_t or_precheck(const or_problem *p, const double *beta, const double *lo, const double *hi,
                    double eps_flat, double eps_soft, double *s, int32_t *cls,
                    double *logz_marginal) {
  const int32_t d = p->d;
  for (int32_t i = 0; i < d; ++i)
    if (!(isfinite(lo[i]) && isfinite(hi[i]) && lo[i] < hi[i])) return OR_E_INVAL;
  if (eps_flat <= 0.0) eps_flat = 1e-6;
  if (eps_soft <= 0.0) eps_soft = 1e-3;
  double *c = malloc(sizeof(double) * d), *x = malloc(sizeof(double) * d);
  double *half = malloc(sizeof(double) * d), *sorted = malloc(sizeof(double) * d);
  double *term = malloc(sizeof(double) * d);
  int32_t st = OR_OK;
  for (int32_t i = 0; i < d; ++i) {
    c[i] = 0.5 * (lo[i] + hi[i]);
    half[i] = 0.5 * (hi[i] - lo[i]);
  }
  double l0, lp, lm;
  or_logl(p, beta, 1, c, &l0, NULL);
  if (!isfinite(l0)) st = OR_E_INVAL;
  for (int32_t i = 0; i < d && st == OR_OK; ++i) {
    memcpy(x, c, sizeof(double) * d);
    x[i] = c[i] + half[i];
    or_logl(p, beta, 1, x, &lp, NULL);
    x[i] = c[i] - half[i];
    or_logl(p, beta, 1, x, &lm, NULL);
    if (!isfinite(lp) || !isfinite(lm)) st = OR_E_INVAL;
    s[i] = fabs(lp - l0) + fabs(lm - l0);
  }
  if (st == OR_OK) {
    memcpy(sorted, s, sizeof(double) * d);
    qsort(sorted, d, sizeof(double), cmp_double);
    const double med = (d % 2) ? sorted[d / 2] : 0.5 * (sorted[d / 2 - 1] + sorted[d / 2]);
    const double mx = sorted[d - 1];
    for (int32_t i = 0; i < d; ++i) {
      if (s[i] < eps_flat * med) {
        cls[i] = 1;
        term[i] = log(hi[i] - lo[i]);
      } else if (s[i] < eps_soft * mx) {
        cls[i] = 2;
        term[i] = 0.5 * LOG_2PI + log(half[i] / sqrt(s[i]));
      } else {
        cls[i] = 0;
        term[i] = 0.0;
      }
    }
    *logz_marginal = or_pairwise_sum(term, d);
  }
  free(c);
  free(x);
  free(half);
  free(sorted);
  free(term);
  return st;
}

double or_mode_log_z(int32_t d, double logl, double log_det_h, double log_volume) {
  return logl - log_volume + 0.5 * d * LOG_2PI - 0.5 * log_det_h;
}

/* ------------------------------------------------------------ whole path */

static int32_t validate_all(const or_problem *p, const double *lo, const double *hi,
                            const or_config *c) {
  int32_t st = or_validate_problem(p);
  if (st) return st;
  if (!lo || !hi || !c) return OR_E_INVAL;
  for (int32_t i = 0; i < p->d; ++i)
    if (!isfinite(lo[i]) || !isfinite(hi[i]) || !(lo[i] < hi[i])) return OR_E_INVAL;
  if (c->m < 1 || c->m > 32) return OR_E_INVAL;
  if (c->n_rays < 1 || c->n_points < 1 || c->n_starts < 1 || c->n_starts > c->n_rays)
    return OR_E_INVAL;
  if (c->max_modes < 1) return OR_E_INVAL;
  return OR_OK;
}

typedef struct {
  double lz;
  int32_t idx;
  int32_t d;
  const double *x;
} mode_key_t;

/* log Z_k descending, ties lexicographic in theta */
static int cmp_modes(const void *A, const void *B) {
  const mode_key_t *a = (const mode_key_t *)A, *b = (const mode_key_t *)B;
  if (a->lz > b->lz) return -1;
  if (a->lz < b->lz) return 1;
  for (int32_t i = 0; i < a->d; ++i) {
    if (a->x[i] < b->x[i]) return -1;
    if (a->x[i] > b->x[i]) return 1;
  }
  return 0;
}

/* Polish candidates, apply the filters (stationary, inside the box, H
 * positive definite), dedup, Laplace per mode, sort and combine. */
static int32_t finish_modes(const or_problem *p, const double *beta, const double *lo,
                            const double *hi, double tau, int32_t max_modes, int32_t nc,
                            double *Xc, int32_t n_threads, or_result *res) {
  const int32_t d = p->d;
  double *lc = (double *)malloc(sizeof(double) * (nc > 0 ? nc : 1));
  double *ldh = (double *)malloc(sizeof(double) * (nc > 0 ? nc : 1));
  uint8_t *ok = (uint8_t *)malloc((size_t)(nc > 0 ? nc : 1));
  int32_t *rep_of = (int32_t *)malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
  int32_t *reps = (int32_t *)malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
  int32_t nrej = 0;
#pragma omp parallel for schedule(dynamic) num_threads(n_threads) reduction(+ : nrej)
  for (int32_t c = 0; c < nc; ++c) {
    double *x = Xc + (size_t)c * d;
    ok[c] = 0;
    int32_t steps = 0;
    int32_t st = or_newton(p, beta, x, 20, &steps);
    if (st != OR_OK) {
      ++nrej;
      continue;
    }
    double *g = (double *)malloc(sizeof(double) * d);
    double *H = (double *)malloc(sizeof(double) * (size_t)d * d);
    double *L = (double *)malloc(sizeof(double) * (size_t)d * d);
    or_logl(p, beta, 1, x, &lc[c], g);
    int inside = 1;
    for (int32_t i = 0; i < d; ++i)
      if (!(x[i] >= lo[i] && x[i] <= hi[i])) inside = 0;
    or_neg_hessian(p, beta, x, H);
    int pd = or_cholesky(d, H, L) == 0;
    if (!pd) ++nrej;
    if (pd && inside && isfinite(lc[c]) && norm_inf(d, g) <= 1e-8) {
      ok[c] = 1;
      ldh[c] = or_logdet_from_chol(d, L);
    }
    free(g); free(H); free(L);
  }
  int32_t nm = or_dedup(nc, d, Xc, lc, ok, tau, rep_of, reps);
  double logv = or_log_volume(d, lo, hi);
  mode_key_t *mk = (mode_key_t *)malloc(sizeof(mode_key_t) * (nm > 0 ? nm : 1));
  for (int32_t i = 0; i < nm; ++i) {
    int32_t c = reps[i];
    mk[i].lz = or_mode_log_z(d, lc[c], ldh[c], logv);
    mk[i].idx = c;
    mk[i].d = d;
    mk[i].x = Xc + (size_t)c * d;
  }
  qsort(mk, (size_t)nm, sizeof(mode_key_t), cmp_modes);
  res->n_rejected_nonpd = nrej;
  res->n_modes = nm;
  int32_t status = OR_OK;
  if (nm == 0) {
    res->log_z = -INFINITY;
    status = OR_E_NOMODE;
  } else if (nm > max_modes) {
    res->log_z = NAN;
    status = OR_E_CAPACITY;
  } else {
    double *lz = (double *)malloc(sizeof(double) * (size_t)(nm > 0 ? nm : 1));
    for (int32_t i = 0; i < nm; ++i) {
      int32_t c = mk[i].idx;
      lz[i] = mk[i].lz;
      if (res->modes) memcpy(res->modes + (size_t)i * d, Xc + (size_t)c * d, sizeof(double) * d);
      if (res->mode_log_z) res->mode_log_z[i] = mk[i].lz;
      if (res->mode_logl) res->mode_logl[i] = lc[c];
      if (res->log_det_h) res->log_det_h[i] = ldh[c];
    }
    res->log_z = or_logsumexp(lz, nm);
    free(lz);
  }
  res->n_hess_evals += nc;
  free(lc); free(ldh); free(ok); free(rep_of); free(reps); free(mk);
  return status;
}

int32_t or_evidence(const or_problem *p, const double *lo, const double *hi, const or_config *cfg,
                    or_result *res) {
  int32_t st = validate_all(p, lo, hi, cfg);
  if (st) {
    if (res) res->log_z = NAN;
    return st;
  }
  const int32_t d = p->d, ns = cfg->n_starts;
  int32_t nt = cfg->n_threads;
#ifdef _OPENMP
  if (nt <= 0) nt = omp_get_max_threads();
#else
  nt = 1;
#endif
  double *beta = (double *)malloc(sizeof(double) * p->K);
  st = or_prep(p, beta, NULL);
  if (st) {
    free(beta);
    res->log_z = NAN;
    return st;
  }
  const int32_t R = cfg->n_rays;
  double *rbl = (double *)malloc(sizeof(double) * R);
  int32_t *rbj = (int32_t *)malloc(sizeof(int32_t) * R);
  int32_t *sray = (int32_t *)malloc(sizeof(int32_t) * ns);
  double *X = (double *)malloc(sizeof(double) * (size_t)ns * d);
  double *lv = (double *)malloc(sizeof(double) * ns);
  int32_t *stat = (int32_t *)malloc(sizeof(int32_t) * ns);
  int32_t *its = (int32_t *)malloc(sizeof(int32_t) * ns);
  int64_t *evs = (int64_t *)malloc(sizeof(int64_t) * ns);
  uint8_t *valid = (uint8_t *)malloc((size_t)ns);
  int32_t *rep_of = (int32_t *)malloc(sizeof(int32_t) * ns);
  int32_t *reps = (int32_t *)malloc(sizeof(int32_t) * ns);
  res->n_logl_evals = (int64_t)R * cfg->n_points;
  res->n_grad_evals = 0;
  res->n_hess_evals = 0;
  st = or_discover(p, beta, lo, hi, R, cfg->n_points, ns, cfg->seed, cfg->problem, rbl, rbj, sray,
                   X);
  if (st == OR_OK) {
    const int32_t max_iter = cfg->max_iter > 0 ? cfg->max_iter : 10 * d + 200;
    const double tol = cfg->grad_tol > 0 ? cfg->grad_tol : 1e-10;
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int32_t s = 0; s < ns; ++s)
      stat[s] = or_lbfgs(p, beta, X + (size_t)s * d, cfg->m, max_iter, tol, &lv[s], NULL,
                         &its[s], &evs[s]);
    int32_t ndead = 0, maxit = 0, ncand = 0;
    for (int32_t s = 0; s < ns; ++s) {
      res->n_grad_evals += evs[s];
      if (its[s] > maxit) maxit = its[s];
      valid[s] = (uint8_t)(stat[s] != OR_ST_DEAD && isfinite(lv[s]));
      if (stat[s] == OR_ST_DEAD) ++ndead;
      ncand += valid[s];
    }
    res->iterations = maxit;
    res->n_dead_starts = ndead;
    res->n_candidates = ncand;
    /* pre-polish dedup of the optimiser's end points */
    double tau_pre = cfg->dedup_tol_pre > 0 ? cfg->dedup_tol_pre : 0.25;
    int32_t nr = or_dedup(ns, d, X, lv, valid, tau_pre, rep_of, reps);
    res->n_reps_pre = nr;
    double *Xr = (double *)malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1) * d);
    for (int32_t i = 0; i < nr; ++i)
      memcpy(Xr + (size_t)i * d, X + (size_t)reps[i] * d, sizeof(double) * d);
    double wmax = 0.0;
    for (int32_t i = 0; i < d; ++i)
      if (hi[i] - lo[i] > wmax) wmax = hi[i] - lo[i];
    double tau = cfg->dedup_tol > 0 ? cfg->dedup_tol : 1e-6 * wmax;
    st = finish_modes(p, beta, lo, hi, tau, cfg->max_modes, nr, Xr, nt, res);
    free(Xr);
  } else {
    res->log_z = NAN;
  }
  free(beta); free(rbl); free(rbj); free(sray); free(X); free(lv); free(stat); free(its);
  free(evs); free(valid); free(rep_of); free(reps);
  return st;
}

/* The tail of or_evidence from given optimiser end points X [n][d] with their
 * l [n] and validity [n]: pre-polish dedup (tau_pre), then finish_modes
 * (Newton polish, filters, final dedup, Laplace combine).  The ChiSao cycle's
 * end points enter the same steps as the single convergence phase's. */
int32_t or_finish_points(const or_problem *p, const double *lo, const double *hi,
                         const or_config *cfg, int32_t n, const double *X, const double *l,
                         const uint8_t *valid, or_result *res) {
  int32_t st = validate_all(p, lo, hi, cfg);
  if (st) {
    if (res) res->log_z = NAN;
    return st;
  }
  const int32_t d = p->d;
  int32_t nt = cfg->n_threads;
#ifdef _OPENMP
  if (nt <= 0) nt = omp_get_max_threads();
#else
  nt = 1;
#endif
  double *beta = (double *)malloc(sizeof(double) * p->K);
  st = or_prep(p, beta, NULL);
  if (st) {
    free(beta);
    res->log_z = NAN;
    return st;
  }
  int32_t *rep_of = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  int32_t *reps = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  int32_t ncand = 0;
  for (int32_t s = 0; s < n; ++s) ncand += valid[s] ? 1 : 0;
  res->n_candidates = ncand;
  double tau_pre = cfg->dedup_tol_pre > 0 ? cfg->dedup_tol_pre : 0.25;
  int32_t nr = or_dedup(n, d, X, l, valid, tau_pre, rep_of, reps);
  res->n_reps_pre = nr;
  double *Xr = (double *)malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1) * d);
  for (int32_t i = 0; i < nr; ++i)
    memcpy(Xr + (size_t)i * d, X + (size_t)reps[i] * d, sizeof(double) * d);
  double wmax = 0.0;
  for (int32_t i = 0; i < d; ++i)
    if (hi[i] - lo[i] > wmax) wmax = hi[i] - lo[i];
  double tau = cfg->dedup_tol > 0 ? cfg->dedup_tol : 1e-6 * wmax;
  st = finish_modes(p, beta, lo, hi, tau, cfg->max_modes, nr, Xr, nt, res);
  free(Xr);
  free(rep_of);
  free(reps);
  free(beta);
  return st;
}

int32_t or_reference_modes(const or_problem *p, const double *lo, const double *hi,
                           double dedup_tol, int32_t max_modes, or_result *res) {
  int32_t st = or_validate_problem(p);
  if (st) return st;
  const int32_t d = p->d, K = p->K;
  double *beta = (double *)malloc(sizeof(double) * K);
  st = or_prep(p, beta, NULL);
  if (st) {
    free(beta);
    return st;
  }
  double *X = (double *)malloc(sizeof(double) * (size_t)K * d);
  memcpy(X, p->mu, sizeof(double) * (size_t)K * d);
  double wmax = 0.0;
  for (int32_t i = 0; i < d; ++i)
    if (hi[i] - lo[i] > wmax) wmax = hi[i] - lo[i];
  double tau = dedup_tol > 0 ? dedup_tol : 1e-6 * wmax;
  res->n_hess_evals = 0;
  st = finish_modes(p, beta, lo, hi, tau, max_modes, K, X, 1, res);
  free(X);
  free(beta);
  return st;
}
