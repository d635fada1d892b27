// ChiSao moves of the exploration samples (section "ChiSao Exploration"):
// stick detection, the Hands Like Clouds smoothed-gradient ascent and the
// momentum anti-convergence phase, on FP64 samples [B][d].
//
// Stick detection: sample b sticks when max_j |g_bj| < grad_tol and
// l_b >= l_max + log 0.1 (l_max the largest finite l of the batch); a
// non-finite l or gradient entry never sticks.  One workgroup finds l_max,
// then one wave per sample reduces its gradient row.
//
// Hands Like Clouds: per step, the n_smooth perturbed copies x + sigma z_k of
// every sample (z_k standard normal, supplied by the caller) go through the
// FP64 contraction and backward in one batch; the mean of their gradients
// (summed in k order, then divided by n_smooth) times alpha_cloud moves each
// free sample.  Anti-convergence: v <- mu v - alpha grad l(x), x <- x + v,
// starting from v = 0.  Every move is clipped to the prior box; stuck samples
// keep their coordinates.  Reseeding (Repulse Monkey / Golden Rooster): from
// each sample along a given direction to where the ray leaves the box, n_pts
// points at t_j = (j + 1/2)/n_pts of that span, l in one FP64 batch, and the
// first point of highest finite l replaces the sample.  The elementwise
// kernels round each operation separately (no contraction into FMAs), in the
// order the steps are written.
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "internal.h"

namespace sb {

// log 0.1 = -ln 10, correctly rounded (not the logarithm of the double nearest 0.1)
constexpr double kLogTenth = -2.3025850929940456840179914546844;

// One workgroup of 1024 threads: the largest finite l (-inf if none).
__global__ __launch_bounds__(1024) void stick_lmax_kernel(int64_t B, const double *l,
                                                          double *lmax) {
  __shared__ double part[16];
  double m = -INFINITY;
  for (int64_t i = threadIdx.x; i < B; i += 1024) {
    const double v = l[i];
    if (isfinite(v)) m = fmax(m, v);
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = part[0];
    for (int w = 1; w < 16; ++w) r = fmax(r, part[w]);
    *lmax = r;
  }
}

// One wave per sample: the gradient row's largest magnitude and finiteness,
// then both conditions.
__global__ __launch_bounds__(256) void stick_mask_kernel(int64_t B, int d, const double *l,
                                                         const double *G, double grad_tol,
                                                         const double *lmax, uint8_t *stuck) {
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  const double *g = G + b * d;
  double m = 0.0;
  int bad = 0;
  for (int j = lane; j < d; j += 64) {
    const double v = g[j];
    bad |= !isfinite(v);
    m = fmax(m, fabs(v));
  }
  m = wave_max(m);
  bad = __any(bad);
  if (lane == 0) {
    const double lb = l[b];
    const double thr = *lmax + kLogTenth;
    stuck[b] = (isfinite(lb) && !bad && m < grad_tol && lb >= thr) ? 1 : 0;
  }
}

// P[k][b][:] = X[b][:] + sigma Z[k][b][:] over n = n_smooth B d values.
__global__ __launch_bounds__(256) void cloud_points_kernel(int64_t n, int64_t bd, const double *X,
                                                           const double *Z, double sigma,
                                                           double *P) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double dz = sigma * Z[e];
  P[e] = X[e % bd] + dz;
}

__device__ inline double clip_box(double x, double lo, double hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

// x <- clip(x + alpha (sum_k G[k] / n_smooth)) for free samples.
__global__ __launch_bounds__(256) void cloud_move_kernel(int64_t bd, int d, int n_smooth,
                                                         const double *G, const uint8_t *stuck,
                                                         const double *lo, const double *hi,
                                                         double alpha, double *X) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= bd) return;
  if (stuck[e / d]) return;
  double acc = 0.0;
  for (int k = 0; k < n_smooth; ++k) acc = acc + G[(int64_t)k * bd + e];
  const double mean = acc / (double)n_smooth;
  const double step = alpha * mean;
  const int j = (int)(e % d);
  X[e] = clip_box(X[e] + step, lo[j], hi[j]);
}

// v <- mu v - alpha g (v = 0 before the first step); free samples x <- clip(x + v).
__global__ __launch_bounds__(256) void anti_move_kernel(int64_t bd, int d, const double *G,
                                                        const uint8_t *stuck, const double *lo,
                                                        const double *hi, double alpha, double mu,
                                                        int first, double *V, double *X) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= bd) return;
  const double v0 = first ? 0.0 : V[e];
  const double mv = mu * v0;
  const double ag = alpha * G[e];
  const double v = mv - ag;
  V[e] = v;
  if (stuck[e / d]) return;
  const int j = (int)(e % d);
  X[e] = clip_box(X[e] + v, lo[j], hi[j]);
}


// Reseeding rays: t_exit per sample (one wave), then the n_pts points per ray,
// then the best of them.  te[b] = min over u_i != 0 of the distance parameter
// to the face u points at, at least 0; 0 when u = 0.
__global__ __launch_bounds__(256) void reseed_exit_kernel(int64_t B, int d, const double *X,
                                                          const double *U, const double *lo,
                                                          const double *hi, double *te) {
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  double m = INFINITY;
  for (int i = lane; i < d; i += 64) {
    const double u = U[b * d + i], x = X[b * d + i];
    if (u > 0.0) m = fmin(m, (hi[i] - x) / u);
    else if (u < 0.0) m = fmin(m, (lo[i] - x) / u);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
  if (lane == 0) te[b] = isinf(m) ? 0.0 : fmax(m, 0.0);
}

// P[b][j][i] = x_bi + ((j + 1/2)/n_pts * te_b) u_bi, each operation rounded.
__global__ __launch_bounds__(256) void reseed_points_kernel(int64_t B, int d, int n_pts,
                                                            const double *X, const double *U,
                                                            const double *te, double *P) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= B * n_pts * d) return;
  const int i = (int)(e % d);
  const int64_t r = e / d;
  const int j = (int)(r % n_pts);
  const int64_t b = r / n_pts;
  const double tj = ((double)j + 0.5) / (double)n_pts;
  const double s = tj * te[b];
  const double su = s * U[b * d + i];
  P[e] = X[b * d + i] + su;
}

// One wave per sample: the first point of highest finite l replaces x.
__global__ __launch_bounds__(256) void reseed_pick_kernel(int64_t B, int d, int n_pts,
                                                          const double *P, const double *L,
                                                          double *X, double *best_l) {
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  int jb = -1;
  double lb = 0.0;
  for (int j = 0; j < n_pts; ++j) {
    const double v = L[b * n_pts + j];
    if (isfinite(v) && (jb < 0 || v > lb)) {
      jb = j;
      lb = v;
    }
  }
  if (jb >= 0)
    for (int i = lane; i < d; i += 64) X[b * d + i] = P[(b * n_pts + jb) * d + i];
  if (lane == 0 && best_l) best_l[b] = jb >= 0 ? lb : (double)NAN;
}

// Golden Rooster's orthonormal directions: modified Gram-Schmidt with
// re-orthogonalisation in FP64, one workgroup per peak, rows of G [C][n][d] in
// place.  Row k loses its projection on each earlier (already normalised) row
// in turn, twice, then is
// divided by its norm, so the triangular factor's diagonal is positive.  A
// row whose remaining norm is at most 8 n eps of its own norm (eps = 2^-52:
// below the rounding residue of n projections it carries no direction of its
// own, so it depends on the earlier rows), or not finite, becomes NaN, and so
// does every later row.  Each thread owns the coordinates i = tid (mod 256)
// of every row.
__device__ void mgs_block(int n, int d, double *V, double *red) {
  for (int k = 0; k < n; ++k) {
    double *v = V + (int64_t)k * d;
    double p0 = 0.0;
    for (int i = threadIdx.x; i < d; i += 256) p0 += v[i] * v[i];
    const double nrm0 = sqrt(block_sum<256>(p0, red));
    // two passes of projections (re-orthogonalisation): one pass leaves the
    // rounding of the projections, a fraction ~eps/residual of the residual
    // itself, in the earlier directions; the second removes it, so the rows
    // stay orthonormal to rounding even for nearly dependent draws
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < k; ++j) {
        const double *q = V + (int64_t)j * d;
        double p = 0.0;
        for (int i = threadIdx.x; i < d; i += 256) p += q[i] * v[i];
        const double dot = block_sum<256>(p, red);
        for (int i = threadIdx.x; i < d; i += 256) v[i] -= dot * q[i];
      }
    double p = 0.0;
    for (int i = threadIdx.x; i < d; i += 256) p += v[i] * v[i];
    const double nrm = sqrt(block_sum<256>(p, red));
    const bool ok = nrm > 8.0 * n * 2.220446049250313e-16 * nrm0 && isfinite(nrm);
    for (int i = threadIdx.x; i < d; i += 256) v[i] = ok ? v[i] / nrm : (double)NAN;
    if (!ok) {
      for (int r = k + 1; r < n; ++r)
        for (int i = threadIdx.x; i < d; i += 256) V[(int64_t)r * d + i] = (double)NAN;
      return;
    }
  }
}

__global__ __launch_bounds__(256) void mgs_rows_kernel(int n, int d, double *G) {
  __shared__ double red[4];
  mgs_block(n, d, G + (int64_t)blockIdx.x * n * d, red);
}

// The same for chunks of uneven size: chunk c is the cnt[c] rows starting at
// row off[c] of U [*][d] (cnt[c] <= d).
__global__ __launch_bounds__(256) void mgs_chunks_kernel(int d, const int32_t *off,
                                                         const int32_t *cnt, double *U) {
  __shared__ double red[4];
  mgs_block(cnt[blockIdx.x], d, U + (int64_t)off[blockIdx.x] * d, red);
}

int launch_mgs_chunks(int n_chunks, int d, const int32_t *off, const int32_t *cnt, double *U,
                      hipStream_t s) {
  if (n_chunks <= 0) return SB_OK;
  hipLaunchKernelGGL(mgs_chunks_kernel, dim3((unsigned)n_chunks), dim3(256), 0, s, d, off, cnt,
                     U);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb

using namespace sb;

static int fail(int st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  char buf[512];
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  set_error("%s", buf);
  return st;
}

extern "C" {

int32_t sb_chisao_stick_dev(int64_t B, int32_t d, const double *logl, const double *grad,
                            double grad_tol, uint8_t *stuck, void *workspace, size_t ws_bytes,
                            void *stream) {
  if (B < 0 || d < 1) return fail(SB_E_INVAL, "stick detection: bad B or d");
  if (!std::isfinite(grad_tol)) return fail(SB_E_INVAL, "grad_tol must be finite");
  if (B == 0) return SB_OK;
  if (!logl || !grad || !stuck) return fail(SB_E_INVAL, "stick detection: NULL array");
  if (B > (int64_t)4 * INT32_MAX) return fail(SB_E_INVAL, "stick detection: B too large");
  if (!workspace || ws_bytes < sizeof(double)) return fail(SB_E_NOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  double *lmax = (double *)workspace;
  hipLaunchKernelGGL(stick_lmax_kernel, dim3(1), dim3(1024), 0, s, B, logl, lmax);
  SB_LAUNCH_CHECK();
  hipLaunchKernelGGL(stick_mask_kernel, dim3((unsigned)ceil_div(B, 4)), dim3(256), 0, s, B, d,
                     logl, grad, grad_tol, lmax, stuck);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

size_t sb_chisao_explore_workspace_bytes(int32_t d, int32_t K, int64_t B, int32_t n_smooth) {
  if (d < 1 || K < 1 || B < 1) return 0;
  const int64_t rows = B * (n_smooth > 1 ? n_smooth : 1);
  return 2 * align_up(8ull * rows * d) + align_up(8ull * rows) + align_up(8ull * B * d) +
         sb_logl_grad_workspace_bytes(d, K, rows, SB_DTYPE_F64) + 1024;
}

int32_t sb_chisao_explore_dev(const sb_model_dev *m, const double *lo, const double *hi,
                              int64_t B, double *X, const uint8_t *stuck, int32_t n_cloud,
                              int32_t n_smooth, const double *Z, double sigma, double alpha_cloud,
                              int32_t n_anti, double alpha, double mu, void *workspace,
                              size_t ws_bytes, void *stream) {
  if (!m) return fail(SB_E_INVAL, "model is NULL");
  if (B < 0 || n_cloud < 0 || n_anti < 0) return fail(SB_E_INVAL, "negative B or step count");
  if (n_cloud > 0 && (n_smooth < 1 || !Z))
    return fail(SB_E_INVAL, "Hands Like Clouds needs n_smooth >= 1 and Z");
  if (!std::isfinite(sigma) || sigma < 0.0 || !std::isfinite(alpha_cloud) ||
      !std::isfinite(alpha) || !std::isfinite(mu))
    return fail(SB_E_INVAL, "sigma, step sizes and momentum must be finite (sigma >= 0)");
  if (B == 0 || (n_cloud == 0 && n_anti == 0)) return SB_OK;
  if (!X || !stuck || !lo || !hi) return fail(SB_E_INVAL, "NULL X, stuck or box");
  const int d = m->d;
  if (d < 1) return fail(SB_E_INVAL, "model d must be >= 1");
  const int ns = n_cloud > 0 ? n_smooth : 1;
  if (!workspace || ws_bytes < sb_chisao_explore_workspace_bytes(d, m->K, B, ns))
    return fail(SB_E_NOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const int64_t bd = B * d, rows = B * ns;
  if (rows * d > ((int64_t)1 << 38)) return fail(SB_E_INVAL, "too many perturbed values");
  Arena ar(workspace, ws_bytes);
  double *P = ar.take<double>((size_t)(rows * d));
  double *G = ar.take<double>((size_t)(rows * d));
  double *L = ar.take<double>((size_t)rows);
  double *V = ar.take<double>((size_t)bd);
  const size_t gws_bytes = sb_logl_grad_workspace_bytes(d, m->K, rows, SB_DTYPE_F64);
  void *gws = ar.take<char>(gws_bytes);
  if (!ar.ok()) return fail(SB_E_NOMEM, "workspace too small");
  int st;
  for (int c = 0; c < n_cloud; ++c) {
    const double *Zc = Z + (int64_t)c * rows * d;
    hipLaunchKernelGGL(cloud_points_kernel, dim3((unsigned)ceil_div(rows * d, 256)), dim3(256),
                       0, s, rows * d, bd, X, Zc, sigma, P);
    SB_LAUNCH_CHECK();
    if ((st = sb_logl_grad_dev(m, rows, P, L, G, SB_DTYPE_F64, gws, gws_bytes, stream))) return st;
    hipLaunchKernelGGL(cloud_move_kernel, dim3((unsigned)ceil_div(bd, 256)), dim3(256), 0, s, bd,
                       d, ns, G, stuck, lo, hi, alpha_cloud, X);
    SB_LAUNCH_CHECK();
  }
  for (int t = 0; t < n_anti; ++t) {
    if ((st = sb_logl_grad_dev(m, B, X, L, G, SB_DTYPE_F64, gws, gws_bytes, stream))) return st;
    hipLaunchKernelGGL(anti_move_kernel, dim3((unsigned)ceil_div(bd, 256)), dim3(256), 0, s, bd, d,
                       G, stuck, lo, hi, alpha, mu, t == 0 ? 1 : 0, V, X);
    SB_LAUNCH_CHECK();
  }
  return SB_OK;
}

size_t sb_chisao_reseed_workspace_bytes(int32_t d, int32_t K, int64_t B, int32_t n_pts) {
  if (d < 1 || K < 1 || B < 1 || n_pts < 1) return 0;
  const int64_t rows = B * n_pts;
  return align_up(8ull * rows * d) + align_up(8ull * rows) + align_up(8ull * B) +
         sb_logl_grad_workspace_bytes(d, K, rows, SB_DTYPE_F64) + 1024;
}

int32_t sb_chisao_reseed_dev(const sb_model_dev *m, const double *lo, const double *hi,
                             int64_t B, double *X, const double *U, int32_t n_pts,
                             double *best_l, void *workspace, size_t ws_bytes, void *stream) {
  if (!m) return fail(SB_E_INVAL, "model is NULL");
  if (B < 0 || n_pts < 1) return fail(SB_E_INVAL, "reseeding needs B >= 0 and n_pts >= 1");
  if (B == 0) return SB_OK;
  if (!X || !U || !lo || !hi) return fail(SB_E_INVAL, "NULL X, U or box");
  const int d = m->d;
  if (d < 1) return fail(SB_E_INVAL, "model d must be >= 1");
  const int64_t rows = B * n_pts;
  if (rows * d > ((int64_t)1 << 38) || B > (int64_t)4 * INT32_MAX)
    return fail(SB_E_INVAL, "too many ray points");
  if (!workspace || ws_bytes < sb_chisao_reseed_workspace_bytes(d, m->K, B, n_pts))
    return fail(SB_E_NOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  Arena ar(workspace, ws_bytes);
  double *P = ar.take<double>((size_t)(rows * d));
  double *L = ar.take<double>((size_t)rows);
  double *te = ar.take<double>((size_t)B);
  const size_t gws_bytes = sb_logl_grad_workspace_bytes(d, m->K, rows, SB_DTYPE_F64);
  void *gws = ar.take<char>(gws_bytes);
  if (!ar.ok()) return fail(SB_E_NOMEM, "workspace too small");
  hipLaunchKernelGGL(reseed_exit_kernel, dim3((unsigned)ceil_div(B, 4)), dim3(256), 0, s, B, d,
                     X, U, lo, hi, te);
  SB_LAUNCH_CHECK();
  hipLaunchKernelGGL(reseed_points_kernel, dim3((unsigned)ceil_div(rows * d, 256)), dim3(256), 0,
                     s, B, d, n_pts, X, U, te, P);
  SB_LAUNCH_CHECK();
  int st = sb_logl_grad_dev(m, rows, P, L, nullptr, SB_DTYPE_F64, gws, gws_bytes, stream);
  if (st) return st;
  hipLaunchKernelGGL(reseed_pick_kernel, dim3((unsigned)ceil_div(B, 4)), dim3(256), 0, s, B, d,
                     n_pts, P, L, X, best_l);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int32_t sb_chisao_orthonormal_dev(int32_t C, int32_t n, int32_t d, double *G, void *stream) {
  if (C < 0 || n < 1 || d < 1 || n > d) return fail(SB_E_INVAL, "need C >= 0 and 1 <= n <= d");
  if (C == 0) return SB_OK;
  if (!G) return fail(SB_E_INVAL, "G is NULL");
  hipLaunchKernelGGL(mgs_rows_kernel, dim3((unsigned)C), dim3(256), 0, (hipStream_t)stream, n, d,
                     G);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // extern "C"
