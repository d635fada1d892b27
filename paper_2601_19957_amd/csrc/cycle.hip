// Kernels of the ChiSao oscillation cycle and of the two-pass ray sampling
// (section "ChiSao Exploration": the oscillation cycle and CarryTiger's
// algorithm summary; section "Two-Pass Sampling": coarse and refinement
// passes).  The cycle's decisions (which slots were lost, which reseeding
// rule applies) are taken on the host from small readbacks; every per-sample
// and per-coordinate computation runs here.
#include <algorithm>

#include "internal.h"
#include "rng.h"

namespace sb {

// out[j * ld + i] = normal i0 + i of counter row rows[j] (j when rows is
// NULL) on `stream`, for j < n, i < d.
__global__ __launch_bounds__(256) void normal_rows_kernel(uint64_t seed, uint32_t problem,
                                                          uint32_t stream, int64_t n, int d,
                                                          const int32_t *rows, uint32_t i0,
                                                          double *out, int64_t ld) {
  const int64_t j = blockIdx.x;
  if (j >= n) return;
  const uint32_t row = rows ? (uint32_t)rows[j] : (uint32_t)j;
  for (int i = threadIdx.x; i < d; i += 256)
    out[j * ld + i] = rng_normal(seed, problem, row, stream, i0 + (uint32_t)i);
}

int launch_normal_rows(uint64_t seed, uint32_t problem, uint32_t stream, int64_t n, int d,
                       const int32_t *rows, uint32_t i0, double *out, int64_t ld, hipStream_t s) {
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(normal_rows_kernel, dim3((unsigned)n), dim3(256), 0, s, seed, problem,
                     stream, n, d, rows, i0, out, ld);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// U[j] <- U[j] / |U[j]| (a zero row stays zero).
__global__ __launch_bounds__(256) void normalize_rows_kernel(int d, double *U) {
  __shared__ double red[4];
  double *u = U + (int64_t)blockIdx.x * d;
  double p = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) p += u[i] * u[i];
  const double nrm = sqrt(block_sum<256>(p, red));
  if (nrm > 0.0)
    for (int i = threadIdx.x; i < d; i += 256) u[i] = u[i] / nrm;
}

int launch_normalize_rows(int64_t n, int d, double *U, hipStream_t s) {
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(normalize_rows_kernel, dim3((unsigned)n), dim3(256), 0, s, d, U);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// out[j] = X[src[j]] (rows of d doubles).
__global__ void gather_idx_kernel(int d, const int32_t *src, const double *X, double *out) {
  const int64_t j = blockIdx.x;
  const int64_t r = src[j];
  for (int i = threadIdx.x; i < d; i += blockDim.x) out[j * d + i] = X[r * d + i];
}
// X[dst[j]] = in[j].
__global__ void scatter_idx_kernel(int d, const int32_t *dst, const double *in, double *X) {
  const int64_t j = blockIdx.x;
  const int64_t r = dst[j];
  for (int i = threadIdx.x; i < d; i += blockDim.x) X[r * d + i] = in[j * d + i];
}

int launch_gather_idx(int64_t n, int d, const int32_t *src, const double *X, double *out,
                      hipStream_t s) {
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(gather_idx_kernel, dim3((unsigned)n), dim3(256), 0, s, d, src, X, out);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int launch_scatter_idx(int64_t n, int d, const int32_t *dst, const double *in, double *X,
                       hipStream_t s) {
  if (n <= 0) return SB_OK;
  hipLaunchKernelGGL(scatter_idx_kernel, dim3((unsigned)n), dim3(256), 0, s, d, dst, in, X);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Per-sample flags after a convergence phase: conv = active and converged,
// lmask = l where active (NaN elsewhere, so that inactive slots never stick
// and stay out of l_max).
__global__ void cycle_flags_kernel(int64_t B, const uint8_t *active, const int32_t *status,
                                   const double *l, uint8_t *conv, double *lmask) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const bool a = active[b] != 0;
  conv[b] = (uint8_t)(a && status[b] == 1);  // 1: converged
  lmask[b] = a ? l[b] : (double)NAN;
}

int launch_cycle_flags(int64_t B, const uint8_t *active, const int32_t *status, const double *l,
                       uint8_t *conv, double *lmask, hipStream_t s) {
  if (B <= 0) return SB_OK;
  hipLaunchKernelGGL(cycle_flags_kernel, dim3((unsigned)ceil_div(B, 256)), dim3(256), 0, s, B,
                     active, status, l, conv, lmask);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// The L-BFGS states of empty slots: status dead (4), so the step kernel skips
// them and the compaction leaves them out.
__global__ void mask_dead_kernel(int64_t B, const uint8_t *active, int32_t *status) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B && !active[b]) status[b] = 4;
}

int launch_mask_dead(int64_t B, const uint8_t *active, int32_t *status, hipStream_t s) {
  if (B <= 0) return SB_OK;
  hipLaunchKernelGGL(mask_dead_kernel, dim3((unsigned)ceil_div(B, 256)), dim3(256), 0, s, B,
                     active, status);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Population standard deviation of each coordinate over the rows with
// free[b] != 0 (mean first, then the mean squared deviation); 0 with no free
// row.  One thread per coordinate, rows in order.
__global__ void coord_spread_kernel(int64_t B, int d, const double *X, const uint8_t *free,
                                    double *sd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d) return;
  double sum = 0.0;
  int64_t n = 0;
  for (int64_t b = 0; b < B; ++b)
    if (free[b]) {
      sum += X[b * d + i];
      ++n;
    }
  if (n == 0) {
    sd[i] = 0.0;
    return;
  }
  const double mean = sum / (double)n;
  double ss = 0.0;
  for (int64_t b = 0; b < B; ++b)
    if (free[b]) {
      const double e = X[b * d + i] - mean;
      ss += e * e;
    }
  sd[i] = sqrt(ss / (double)n);
}

int launch_coord_spread(int64_t B, int d, const double *X, const uint8_t *free, double *sd,
                        hipStream_t s) {
  hipLaunchKernelGGL(coord_spread_kernel, dim3((unsigned)ceil_div(d, 256)), dim3(256), 0, s, B,
                     d, X, free, sd);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// ------------------------------------------------------ two-pass sampling

// Refinement pass of ray r from its coarse scores lc [R][n_pts] (t_j =
// (j + 1/2)/n_pts): the active cells [t_j - h/2, t_j + h/2] (h = 1/n_pts) of
// the finite scores above l_max - delta carry the density exp(l_j - l_max);
// refined point i sits at the quantile (i + 1/2)/n_ref of that piecewise
// constant density.  A ray without a finite score gets NaN points.
__global__ void refine_t_kernel(int R, int n_pts, int n_ref, double delta, const double *lc,
                                double *tref) {
#pragma clang fp contract(off)
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const double *l = lc + (int64_t)r * n_pts;
  double *t = tref + (int64_t)r * n_ref;
  double lmax = -INFINITY;
  bool any = false;
  for (int j = 0; j < n_pts; ++j)
    if (isfinite(l[j])) {
      any = true;
      lmax = fmax(lmax, l[j]);
    }
  if (!any) {
    for (int i = 0; i < n_ref; ++i) t[i] = (double)NAN;
    return;
  }
  const double h = 1.0 / (double)n_pts;
  double tot = 0.0;  // the total weight, accumulated in cell order
  for (int j = 0; j < n_pts; ++j)
    if (isfinite(l[j]) && l[j] > lmax - delta) tot += exp(l[j] - lmax) * h;
  // walk the cells and the quantiles together: quantile i lies in the first
  // active cell whose cumulative weight exceeds it
  int j = 0;
  double cw = 0.0, w = 0.0;
  int last = -1;
  for (int i = 0; i < n_ref; ++i) {
    const double u = ((double)i + 0.5) / (double)n_ref * tot;
    while (true) {
      if (last >= 0 && u < cw + w) break;
      // advance to the next active cell (keep the last one when none is left)
      int nx = (last < 0) ? 0 : last + 1;
      while (nx < n_pts && !(isfinite(l[nx]) && l[nx] > lmax - delta)) ++nx;
      if (nx >= n_pts) break;
      if (last >= 0) cw += w;
      last = nx;
      w = exp(l[nx] - lmax) * h;
    }
    j = last;
    const double tc = ((double)j + 0.5) / (double)n_pts;
    t[i] = tc - 0.5 * h + (u - cw) / w * h;
  }
}

int launch_refine_t(int R, int n_pts, int n_ref, double delta, const double *lc, double *tref,
                    hipStream_t s) {
  if (R <= 0 || n_ref <= 0) return SB_OK;
  hipLaunchKernelGGL(refine_t_kernel, dim3((unsigned)ceil_div(R, 64)), dim3(64), 0, s, R, n_pts,
                     n_ref, delta, lc, tref);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Points P0 + t (P1 - P0) of the refined samples, rows r * n_ref + i.
__global__ void refine_points_kernel(int n_ref, int d, const double *P0, const double *P1,
                                     const double *tref, double *Xr) {
#pragma clang fp contract(off)
  const int64_t row = blockIdx.x;
  const int64_t r = row / n_ref;
  const double t = tref[row];
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    const double a = P0[r * d + i], b = P1[r * d + i];
    Xr[row * d + i] = a + t * (b - a);
  }
}

int launch_refine_points(int R, int n_ref, int d, const double *P0, const double *P1,
                         const double *tref, double *Xr, hipStream_t s) {
  if (R <= 0 || n_ref <= 0) return SB_OK;
  hipLaunchKernelGGL(refine_points_kernel, dim3((unsigned)((int64_t)R * n_ref)), dim3(256), 0, s,
                     n_ref, d, P0, P1, tref, Xr);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Best sample of each ray over its coarse scores lc [R][n_pts] and refined
// scores lr [R][n_ref] at tref: highest finite l (ties: coarse before
// refined, then the lower index); NaN and t = 0 when no score is finite.
__global__ void refine_best_kernel(int R, int n_pts, int n_ref, const double *lc,
                                   const double *lr, const double *tref, double *best_l,
                                   double *best_t) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double bl = -INFINITY, bt = 0.0;
  bool any = false;
  for (int j = 0; j < n_pts; ++j) {
    const double v = lc[(int64_t)r * n_pts + j];
    if (isfinite(v) && (!any || v > bl)) {
      any = true;
      bl = v;
      bt = ((double)j + 0.5) / (double)n_pts;
    }
  }
  for (int i = 0; i < n_ref; ++i) {
    const double v = lr[(int64_t)r * n_ref + i];
    if (isfinite(v) && (!any || v > bl)) {
      any = true;
      bl = v;
      bt = tref[(int64_t)r * n_ref + i];
    }
  }
  best_l[r] = any ? bl : (double)NAN;
  best_t[r] = bt;
}

int launch_refine_best(int R, int n_pts, int n_ref, const double *lc, const double *lr,
                       const double *tref, double *best_l, double *best_t, hipStream_t s) {
  if (R <= 0) return SB_OK;
  hipLaunchKernelGGL(refine_best_kernel, dim3((unsigned)ceil_div(R, 256)), dim3(256), 0, s, R,
                     n_pts, n_ref, lc, lr, tref, best_l, best_t);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Start s = the point at best_t of ray start_ray[s].
__global__ void gather_starts_t_kernel(int d, const int32_t *start_ray, const double *best_t,
                                       const double *P0, const double *P1, double *X0) {
#pragma clang fp contract(off)
  const int64_t sidx = blockIdx.x;
  const int64_t r = start_ray[sidx];
  const double t = best_t[r];
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    const double a = P0[r * d + i], b = P1[r * d + i];
    X0[sidx * d + i] = a + t * (b - a);
  }
}

int launch_gather_starts_t(int d, int n_starts, const int32_t *start_ray, const double *best_t,
                           const double *P0, const double *P1, double *X0, hipStream_t s) {
  if (n_starts <= 0) return SB_OK;
  hipLaunchKernelGGL(gather_starts_t_kernel, dim3((unsigned)n_starts), dim3(256), 0, s, d,
                     start_ray, best_t, P0, P1, X0);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
