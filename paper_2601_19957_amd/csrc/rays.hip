// Ray-bundle discovery (CarryTiger's ray generation and coarse pass).
//
// Ray r uses geometry r mod 4: vertex-to-vertex, vertex-to-edge-midpoint,
// wall-to-wall along a random axis, and sunburst from the box centre along a
// uniform direction on the sphere to the boundary (section "Ray Generation").
// Randomness is Philox4x32-10 (Salmon et al., SC'11): counter (ray, block,
// stream, problem), key (seed low word, seed high word); coordinate i of a
// stream uses word i%4 of block i/4, a uniform uses the two words of half
// block i%2 of block i/2 (53 bits).  Points t_j = (j + 1/2)/n_pts along each
// ray are scored by the likelihood GEMM; each ray keeps its argmax (ties:
// lowest j) and the rays with the highest maxima seed the optimiser (ties:
// lowest ray index).
#include <algorithm>

#include "internal.h"
#include "rng.h"

namespace sb {

__global__ __launch_bounds__(256) void rays_kernel(int d, const double *lo, const double *hi,
                                                   uint64_t seed, uint32_t problem, double *P0,
                                                   double *P1, float *P0f, float *P1f) {
#pragma clang fp contract(off)
  const uint32_t r = blockIdx.x;
  const int g = (int)(r & 3u);
  double *p = P0 + (size_t)r * d, *q = P1 + (size_t)r * d;
  __shared__ double red[4];
  const uint32_t axis =
      (uint32_t)(((uint64_t)rng_word(seed, problem, r, 2, 0) * (uint64_t)d) >> 32);
  if (g == 0 || g == 1) {
    for (int i = threadIdx.x; i < d; i += 256) {
      p[i] = (rng_word(seed, problem, r, 0, i) & 1u) ? hi[i] : lo[i];
      double qi = (rng_word(seed, problem, r, 1, i) & 1u) ? hi[i] : lo[i];
      if (g == 1 && (uint32_t)i == axis) qi = 0.5 * (lo[i] + hi[i]);
      q[i] = qi;
    }
  } else if (g == 2) {
    for (int i = threadIdx.x; i < d; i += 256) {
      double pi = lo[i] + rng_uniform(seed, problem, r, 0, i) * (hi[i] - lo[i]);
      double qi = lo[i] + rng_uniform(seed, problem, r, 1, i) * (hi[i] - lo[i]);
      if ((uint32_t)i == axis) {
        pi = lo[i];
        qi = hi[i];
      }
      p[i] = pi;
      q[i] = qi;
    }
  } else {
    // z ~ N(0, I) by Box-Muller (cosine branch), u = z / |z|, exit where the
    // ray from the centre leaves the box.
    double n2 = 0.0;
    for (int i = threadIdx.x; i < d; i += 256) {
      double u1 = rng_uniform(seed, problem, r, 0, i);
      double u2 = rng_uniform(seed, problem, r, 1, i);
      double z = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
      q[i] = z;
      n2 += z * z;
    }
    n2 = block_sum<256>(n2, red);
    const double nrm = sqrt(n2);
    double tmin = INFINITY;
    for (int i = threadIdx.x; i < d; i += 256) {
      double c = 0.5 * (lo[i] + hi[i]);
      double u = nrm > 0.0 ? q[i] / nrm : (i == 0 ? 1.0 : 0.0);
      q[i] = u;
      double t = INFINITY;
      if (u > 0.0)
        t = (hi[i] - c) / u;
      else if (u < 0.0)
        t = (lo[i] - c) / u;
      tmin = fmin(tmin, t);
    }
    __syncthreads();
    tmin = -block_max<256>(-tmin, red);
    for (int i = threadIdx.x; i < d; i += 256) {
      double c = 0.5 * (lo[i] + hi[i]);
      p[i] = c;
      q[i] = c + tmin * q[i];
    }
  }
  if (P0f) {
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += 256) {
      P0f[(size_t)r * d + i] = (float)p[i];
      P1f[(size_t)r * d + i] = (float)q[i];
    }
  }
}

int launch_rays(int d, const double *lo, const double *hi, int R, uint64_t seed, uint32_t problem,
                double *P0, double *P1, float *P0f, float *P1f, hipStream_t s) {
  if (R <= 0) return SB_OK;
  hipLaunchKernelGGL(rays_kernel, dim3(R), dim3(256), 0, s, d, lo, hi, seed, problem, P0, P1, P0f,
                     P1f);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Per-ray argmax over the n_pts scores (strict >, so ties keep the lowest j;
// NaN never wins).
template <typename T>
__global__ void ray_argmax_kernel(int R, int n_pts, const T *l, double *best_l, int32_t *best_j) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double best = -INFINITY;
  int bj = 0;
  for (int j = 0; j < n_pts; ++j) {
    double v = (double)l[(size_t)r * n_pts + j];
    if (v > best) {
      best = v;
      bj = j;
    }
  }
  best_l[r] = best;
  best_j[r] = bj;
}

int launch_ray_argmax(int R, int n_pts, int dtype, const void *l, double *best_l, int32_t *best_j,
                      hipStream_t s) {
  if (R <= 0) return SB_OK;
  dim3 grid((unsigned)ceil_div(R, 256));
  if (dtype == DT_F64)
    hipLaunchKernelGGL(ray_argmax_kernel<double>, grid, dim3(256), 0, s, R, n_pts,
                       (const double *)l, best_l, best_j);
  else
    hipLaunchKernelGGL(ray_argmax_kernel<float>, grid, dim3(256), 0, s, R, n_pts,
                       (const float *)l, best_l, best_j);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Rank of each ray by (best l descending, index ascending), NaN as -inf; the
// first n_starts ranks name the starts.  A workgroup ranks 64 rays: lane l of
// every wave holds ray 64 b + l, and wave w counts the rays of the w-th
// sixteenth of the array that precede it (the compared key is the same for
// the whole wave, a broadcast read); the 16 partial counts are added in LDS.
constexpr int TOPN_PARTS = 16;
__global__ __launch_bounds__(64 * TOPN_PARTS) void topn_kernel(int R, int n_starts,
                                                               const double *best_l,
                                                               int32_t *start_ray) {
  __shared__ int part[TOPN_PARTS][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + lane;
  double key = -INFINITY;
  if (r < R) {
    key = best_l[r];
    if (key != key) key = -INFINITY;
  }
  const int seg = (R + TOPN_PARTS - 1) / TOPN_PARTS;
  const int t0 = w * seg, t1 = min(R, t0 + seg);
  int cnt = 0;
  for (int t = t0; t < t1; ++t) {
    double v = best_l[t];
    if (v != v) v = -INFINITY;
    cnt += (v > key) || (v == key && t < r);
  }
  part[w][lane] = cnt;
  __syncthreads();
  if (w == 0 && r < R) {
    int rank = 0;
#pragma unroll
    for (int q = 0; q < TOPN_PARTS; ++q) rank += part[q][lane];
    if (rank < n_starts) start_ray[rank] = r;
  }
}

int launch_topn(int R, int n_starts, const double *best_l, int32_t *start_ray, hipStream_t s) {
  if (R <= 0) return SB_OK;
  hipLaunchKernelGGL(topn_kernel, dim3((unsigned)ceil_div(R, 64)), dim3(64 * TOPN_PARTS), 0, s, R,
                     n_starts, best_l, start_ray);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

__global__ void gather_starts_kernel(int d, int n_pts, int n_starts, const int32_t *start_ray,
                                     const int32_t *best_j, const double *P0, const double *P1,
                                     double *X0) {
#pragma clang fp contract(off)
  const int sidx = blockIdx.x;
  const int r = start_ray[sidx];
  const double t = ((double)best_j[r] + 0.5) / (double)n_pts;
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    double a = P0[(size_t)r * d + i], b = P1[(size_t)r * d + i];
    X0[(size_t)sidx * d + i] = a + t * (b - a);
  }
}

int launch_gather_starts(int d, int n_pts, int n_starts, const int32_t *start_ray,
                         const int32_t *best_j, const double *P0, const double *P1, double *X0,
                         hipStream_t s) {
  if (n_starts <= 0) return SB_OK;
  hipLaunchKernelGGL(gather_starts_kernel, dim3(n_starts), dim3(256), 0, s, d, n_pts, n_starts,
                     start_ray, best_j, P0, P1, X0);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb

// ====================================================================
// Batches: rays of every problem in one launch (ray r of problem p uses
// Philox counter word 3 = p's index), per-problem argmax / top-n / starts.
namespace sb {

__device__ inline int find_ray_prob(const BatchProb *probs, int n, int64_t r) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].r0 <= r)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void rays_group_kernel(BatchDev b, double *P0, double *P1,
                                                         float *P0f, float *P1f) {
#pragma clang fp contract(off)
  const int64_t rg = blockIdx.x;
  const int pidx = find_ray_prob(b.probs, b.n, rg);
  const BatchProb pr = b.probs[pidx];
  const uint32_t r = (uint32_t)(rg - pr.r0);
  const int d = pr.d, dp = pr.dp;
  const double *lo = b.lo + pr.box_off, *hi = b.hi + pr.box_off;
  const uint64_t seed = pr.seed;
  const uint32_t problem = (uint32_t)pr.index;
  const int g = (int)(r & 3u);
  double *p = P0 + pr.roff0 + (size_t)r * dp, *q = P1 + pr.roff0 + (size_t)r * dp;
  __shared__ double red[4];
  const uint32_t axis =
      (uint32_t)(((uint64_t)rng_word(seed, problem, r, 2, 0) * (uint64_t)d) >> 32);
  if (g == 0 || g == 1) {
    for (int i = threadIdx.x; i < d; i += 256) {
      p[i] = (rng_word(seed, problem, r, 0, i) & 1u) ? hi[i] : lo[i];
      double qi = (rng_word(seed, problem, r, 1, i) & 1u) ? hi[i] : lo[i];
      if (g == 1 && (uint32_t)i == axis) qi = 0.5 * (lo[i] + hi[i]);
      q[i] = qi;
    }
  } else if (g == 2) {
    for (int i = threadIdx.x; i < d; i += 256) {
      double pi = lo[i] + rng_uniform(seed, problem, r, 0, i) * (hi[i] - lo[i]);
      double qi = lo[i] + rng_uniform(seed, problem, r, 1, i) * (hi[i] - lo[i]);
      if ((uint32_t)i == axis) {
        pi = lo[i];
        qi = hi[i];
      }
      p[i] = pi;
      q[i] = qi;
    }
  } else {
    double n2 = 0.0;
    for (int i = threadIdx.x; i < d; i += 256) {
      double u1 = rng_uniform(seed, problem, r, 0, i);
      double u2 = rng_uniform(seed, problem, r, 1, i);
      double z = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
      q[i] = z;
      n2 += z * z;
    }
    n2 = block_sum<256>(n2, red);
    const double nrm = sqrt(n2);
    double tmin = INFINITY;
    for (int i = threadIdx.x; i < d; i += 256) {
      double c = 0.5 * (lo[i] + hi[i]);
      double u = nrm > 0.0 ? q[i] / nrm : (i == 0 ? 1.0 : 0.0);
      q[i] = u;
      double t = INFINITY;
      if (u > 0.0)
        t = (hi[i] - c) / u;
      else if (u < 0.0)
        t = (lo[i] - c) / u;
      tmin = fmin(tmin, t);
    }
    __syncthreads();
    tmin = -block_max<256>(-tmin, red);
    for (int i = threadIdx.x; i < d; i += 256) {
      double c = 0.5 * (lo[i] + hi[i]);
      p[i] = c;
      q[i] = c + tmin * q[i];
    }
  }
  for (int i = d + threadIdx.x; i < dp; i += 256) {  // zero padding
    p[i] = 0.0;
    q[i] = 0.0;
  }
  if (P0f) {
    __syncthreads();
    for (int i = threadIdx.x; i < dp; i += 256) {
      P0f[pr.roff0 + (size_t)r * dp + i] = (float)p[i];
      P1f[pr.roff0 + (size_t)r * dp + i] = (float)q[i];
    }
  }
}

int launch_rays_group(const BatchDev &b, double *P0, double *P1, float *P0f, float *P1f,
                      hipStream_t s) {
  if (b.Rtot <= 0) return SB_OK;
  hipLaunchKernelGGL(rays_group_kernel, dim3((unsigned)b.Rtot), dim3(256), 0, s, b, P0, P1, P0f,
                     P1f);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Per ray (global index): argmax over its n_pts scores at rows pt0 + r*n_pts.
template <typename T>
__global__ void ray_argmax_group_kernel(BatchDev b, const T *l, double *best_l, int32_t *best_j) {
  const int64_t rg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rg >= b.Rtot) return;
  const BatchProb pr = b.probs[find_ray_prob(b.probs, b.n, rg)];
  const int64_t r = rg - pr.r0;
  double best = -INFINITY;
  int bj = 0;
  for (int j = 0; j < pr.n_pts; ++j) {
    const double v = (double)l[pr.pt0 + r * pr.n_pts + j];
    if (v > best) {
      best = v;
      bj = j;
    }
  }
  best_l[rg] = best;
  best_j[rg] = bj;
}

int launch_ray_argmax_group(const BatchDev &b, int dtype, const void *l, double *best_l,
                            int32_t *best_j, hipStream_t s) {
  if (b.Rtot <= 0) return SB_OK;
  dim3 grid((unsigned)ceil_div(b.Rtot, 256));
  if (dtype == DT_F64)
    hipLaunchKernelGGL(ray_argmax_group_kernel<double>, grid, dim3(256), 0, s, b,
                       (const double *)l, best_l, best_j);
  else
    hipLaunchKernelGGL(ray_argmax_group_kernel<float>, grid, dim3(256), 0, s, b,
                       (const float *)l, best_l, best_j);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Rank of each ray among its problem's rays (best l descending, index
// ascending; NaN as -inf); the first B_p ranks are problem p's starts:
// start_ray[s0 + rank] = local ray index.
__global__ __launch_bounds__(256) void topn_group_kernel(BatchDev b, const double *best_l,
                                                         int32_t *start_ray) {
  const int64_t rg = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (rg >= b.Rtot) return;
  const BatchProb pr = b.probs[find_ray_prob(b.probs, b.n, rg)];
  const int64_t r = rg - pr.r0;
  double key = best_l[rg];
  if (key != key) key = -INFINITY;
  // each thread scans its own problem's rays (a block may span two problems)
  int64_t rank = 0;
  for (int64_t t = 0; t < pr.R; ++t) {
    double w = best_l[pr.r0 + t];
    if (w != w) w = -INFINITY;
    rank += (w > key) || (w == key && t < r);
  }
  if (rank < pr.B) start_ray[pr.s0 + rank] = (int32_t)r;
}

int launch_topn_group(const BatchDev &b, const double *best_l, int32_t *start_ray,
                      hipStream_t s) {
  if (b.Rtot <= 0) return SB_OK;
  hipLaunchKernelGGL(topn_group_kernel, dim3((unsigned)ceil_div(b.Rtot, 256)), dim3(256), 0, s, b,
                     best_l, start_ray);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// X0 of start s (global): its ray's best point, written at voff0 + local*dp.
template <typename T>
__global__ void gather_starts_group_kernel(BatchDev b, const int32_t *start_ray,
                                           const int32_t *best_j, const double *P0,
                                           const double *P1, T *X0) {
#pragma clang fp contract(off)
  const int64_t sg = blockIdx.x;
  int lo = 0, hi = b.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.probs[mid].s0 <= sg)
      lo = mid;
    else
      hi = mid - 1;
  }
  const BatchProb pr = b.probs[lo];
  const int64_t sl = sg - pr.s0;
  const int r = start_ray[sg];
  const double t = ((double)best_j[pr.r0 + r] + 0.5) / (double)pr.n_pts;
  const double *a = P0 + pr.roff0 + (size_t)r * pr.dp, *c = P1 + pr.roff0 + (size_t)r * pr.dp;
  T *x = X0 + pr.voff0 + sl * pr.dp;
  for (int i = threadIdx.x; i < pr.dp; i += blockDim.x) {
    const double v = a[i] + t * (c[i] - a[i]);
    x[i] = (T)v;
  }
}

int launch_gather_starts_group(const BatchDev &b, const int32_t *start_ray, const int32_t *best_j,
                               const double *P0, const double *P1, void *X0, int dtype,
                               hipStream_t s) {
  if (b.Btot <= 0) return SB_OK;
  if (dtype == DT_F64)
    hipLaunchKernelGGL(gather_starts_group_kernel<double>, dim3((unsigned)b.Btot), dim3(128), 0,
                       s, b, start_ray, best_j, P0, P1, (double *)X0);
  else
    hipLaunchKernelGGL(gather_starts_group_kernel<float>, dim3((unsigned)b.Btot), dim3(128), 0, s,
                       b, start_ray, best_j, P0, P1, (float *)X0);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
