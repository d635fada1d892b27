// Preprocessing probe: dimensional pathology detection (section
// "Preprocessing: Dimensional Pathology Detection").
//
// From the prior centre c_i = (a_i + b_i)/2 with half-widths D_i =
// (b_i - a_i)/2, the likelihood is evaluated at c and at c +- D_i e_i for
// every coordinate (2d + 1 rows through the FP64 contraction and epilogue of
// the logL path), giving the sensitivities
//   s_i = |l(c + D_i e_i) - l(c)| + |l(c - D_i e_i) - l(c)|.
// Coordinates with s_i < eps_flat * median(s) are flat, the others with
// s_i < eps_soft * max(s) soft nuisance; the flagged ones contribute
// log(b_i - a_i) (flat: the integral of a constant likelihood factor over the
// prior range) or 1/2 log 2 pi + log(D_i / sqrt(s_i)) (soft: a Gaussian factor
// of width D_i / sqrt(s_i)) to the marginal log-evidence.
//
// The median comes from the ranks of the sensitivities (rank of s_i = number
// of j with (s_j, j) before (s_i, i), non-finite values last), which place
// every value at its sorted position with no sort kernel: O(d^2) compares,
// a few microseconds at d = 1024.
#include "internal.h"

namespace sb {

// Row 0: the centre; row 1 + 2i: coordinate i at c_i + D_i; row 2 + 2i: at
// c_i - D_i.  No contraction into FMAs: the points are the two-rounding
// expressions the definition gives.
__global__ __launch_bounds__(256) void precheck_points_kernel(int d, const double *lo,
                                                              const double *hi, double *X) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)(2 * d + 1) * d;
  if (e >= n) return;
  const int64_t row = e / d;
  const int j = (int)(e % d);
  const double c = 0.5 * (lo[j] + hi[j]);
  double v = c;
  if (row > 0 && (int)((row - 1) / 2) == j) {
    const double h = 0.5 * (hi[j] - lo[j]);
    v = ((row - 1) % 2 == 0) ? c + h : c - h;
  }
  X[e] = v;
}

__device__ inline double rank_key(double v) { return isfinite(v) ? v : INFINITY; }

// s_i from the probe values, then its rank among all s; sorted[rank] = s_i.
__global__ __launch_bounds__(256) void precheck_rank_kernel(int d, const double *l, double *s,
                                                            double *sorted) {
  __shared__ double tile[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double l0 = l[0];
  double si = 0.0;
  if (i < d) {
    si = fabs(l[1 + 2 * i] - l0) + fabs(l[2 + 2 * i] - l0);
    s[i] = si;
  }
  const double ki = rank_key(si);
  int rank = 0;
  for (int j0 = 0; j0 < d; j0 += 256) {
    const int j = j0 + threadIdx.x;
    // recompute s_j (the kernel's own writes of s are not visible across blocks)
    tile[threadIdx.x] = j < d ? rank_key(fabs(l[1 + 2 * j] - l0) + fabs(l[2 + 2 * j] - l0)) : 0.0;
    __syncthreads();
    const int nj = min(256, d - j0);
    for (int t = 0; t < nj; ++t) {
      const double kj = tile[t];
      rank += (kj < ki || (kj == ki && j0 + t < i)) ? 1 : 0;
    }
    __syncthreads();
  }
  if (i < d) sorted[rank] = si;
}

// One workgroup: median and maximum, the classes, the marginal terms and
// their sum (strided per-thread sums, then a fixed tree), and the counts
// (active, flat, soft, non-finite).
__global__ __launch_bounds__(256) void precheck_classify_kernel(int d, const double *lo,
                                                                const double *hi, double eps_flat,
                                                                double eps_soft, const double *s,
                                                                const double *sorted,
                                                                int32_t *cls, double *logz,
                                                                int32_t *counts) {
  __shared__ int cnt[4];
  __shared__ double part[256];
  if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
  __syncthreads();
  const double med = (d % 2) ? sorted[d / 2] : 0.5 * (sorted[d / 2 - 1] + sorted[d / 2]);
  const double mx = sorted[d - 1];
  int na = 0, nf = 0, ns = 0, nb = 0;
  double acc = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double si = s[i];
    int c = 0;
    double t = 0.0;
    if (!isfinite(si)) {
      ++nb;
    } else if (si < eps_flat * med) {
      c = 1;
      t = log(hi[i] - lo[i]);
    } else if (si < eps_soft * mx) {
      c = 2;
      t = 0.5 * 1.8378770664093454835606594728112 + log(0.5 * (hi[i] - lo[i]) / sqrt(si));
    }
    na += c == 0;
    nf += c == 1;
    ns += c == 2;
    cls[i] = c;
    acc += t;
  }
  // the terms' sum: per-thread strided partial sums, then a fixed tree
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  na = wave_sum(na);
  nf = wave_sum(nf);
  ns = wave_sum(ns);
  nb = wave_sum(nb);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&cnt[0], na);
    atomicAdd(&cnt[1], nf);
    atomicAdd(&cnt[2], ns);
    atomicAdd(&cnt[3], nb);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *logz = cnt[3] ? (double)NAN : part[0];
    for (int k = 0; k < 4; ++k) counts[k] = cnt[k];
  }
}

size_t precheck_ws_bytes(int d, int K) {
  const size_t rows = 2ull * d + 1;
  return align_up(8 * rows * d) + align_up(8 * rows) + align_up(8 * rows * K * ceil_div(d, 64)) +
         3 * align_up(8ull * d) + align_up(16) + 1024;
}

int run_precheck(const Model &m, const double *lo, const double *hi, double eps_flat,
                 double eps_soft, double *s, int32_t *cls, double *logz, int32_t *counts_host,
                 void *workspace, size_t ws_bytes, hipStream_t st) {
  const int d = m.d;
  const int64_t rows = 2ll * d + 1;
  Arena ar(workspace, ws_bytes);
  double *X = ar.take<double>((size_t)rows * d);
  double *l = ar.take<double>(rows);
  double *qp = ar.take<double>((size_t)rows * m.K * ceil_div(d, 64));
  double *sorted = ar.take<double>(d);
  ar.take<double>(2 * (size_t)d);
  int32_t *counts = ar.take<int32_t>(4);
  if (!ar.ok()) {
    set_error("precheck: workspace too small");
    return SB_E_NOMEM;
  }
  hipLaunchKernelGGL(precheck_points_kernel, dim3((unsigned)ceil_div(rows * d, 256)), dim3(256),
                     0, st, d, lo, hi, X);
  SB_LAUNCH_CHECK();
  ASrc a;
  a.kind = 0;
  a.X = X;
  a.ldx = d;
  QuadOut o;
  o.Y = nullptr;
  o.ldy = (int64_t)m.K * d;
  o.qpart = qp;
  const TuneProbe pr{a, o};
  const TileCfg t = autotune_tiles(DT_F64, m, rows, st, &pr);
  int r = launch_quad_gemm(DT_F64, m, a, rows, nullptr, o, t, st);
  if (r) return r;
  FinishArgs f;
  f.M = rows;
  f.qpart = qp;
  f.ntn = o.ntn;
  f.logl = l;
  f.logl_f64 = true;
  if ((r = launch_finish(DT_F64, m, f, st))) return r;
  hipLaunchKernelGGL(precheck_rank_kernel, dim3((unsigned)ceil_div(d, 256)), dim3(256), 0, st, d,
                     l, s, sorted);
  SB_LAUNCH_CHECK();
  hipLaunchKernelGGL(precheck_classify_kernel, dim3(1), dim3(256), 0, st, d, lo, hi, eps_flat,
                     eps_soft, s, sorted, cls, logz, counts);
  SB_LAUNCH_CHECK();
  SB_HIP(hipMemcpyAsync(counts_host, counts, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SB_HIP(hipStreamSynchronize(st));
  return SB_OK;
}

}  // namespace sb
