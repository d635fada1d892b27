// Batched FP64 Cholesky factorisation, log-determinant and solves.
//
// H = L L^T (the whitening factor of the paper's appendix "Coordinate
// Whitening"); log det H = 2 sum_i log L_ii.  A failed pivot means H is not
// positive definite, i.e. the candidate is not a maximum (saddle filter of
// GreenDragon, generalised).  Blocked right-looking factorisation with 64-wide
// panels: diagonal block in registers, triangular solve of the panel below
// it, symmetric rank-64 update of the trailing lower triangle.  One launch
// per stage covers every matrix of the batch.
#include <algorithm>

#include "internal.h"

namespace sb {

constexpr int NB = 64;

// The 64 x 64 blocks below are held as a 16 x 16 grid of 4 x 4 register
// tiles, thread t owning tile (t / 16, t % 16), and processed four columns
// (one tile column) at a time.  Every element receives the subtractions of
// the columns before it one at a time in column order and is scaled by the
// reciprocal of its pivot last (one division per pivot instead of one per
// element: the serial pivot chain is the kernels' critical path).

// Factor the diagonal block [j0, j0+nb)^2 of every matrix.  Step s: the
// owner of diagonal tile s factors it (left-looking within the tile), the
// tiles below it solve against it, and the trailing tiles take the rank-4
// update.  Rows and columns past nb are padded with the identity.
__global__ __launch_bounds__(256) void chol_diag_kernel(int n, int j0, double *L,
                                                        int32_t *info) {
  const int c = blockIdx.x;
  if (info[c] != 0) return;
  double *A = L + (size_t)c * n * n;
  const int nb = min(NB, n - j0);
  const int tid = threadIdx.x, ti = tid >> 4, tk = tid & 15;
  const bool low = ti >= tk;
  __shared__ double Dg[2][4][4];   // factor of the step's diagonal tile
  __shared__ double Dr[2][4];      // reciprocals of its diagonal
  __shared__ double Pn[2][NB][4];  // the step's solved tile column
  __shared__ int fail;
  double a[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * ti + u, k = 4 * tk + v;
      a[u][v] = (i < nb && k < nb) ? (k <= i ? A[(size_t)(j0 + i) * n + j0 + k] : 0.0)
                                   : (i == k ? 1.0 : 0.0);
    }
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int s = 0; s < NB / 4; ++s) {
    const int b = s & 1;
    if (ti == s && tk == s) {
      int f = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double p = a[v][v];
#pragma unroll
        for (int w = 0; w < v; ++w) p -= a[v][w] * a[v][w];
        if (!(p > 0.0) && f == 0) f = 4 * s + v + 1;
        const double d = sqrt(p), r = 1.0 / d;
        a[v][v] = d;
        Dr[b][v] = r;
#pragma unroll
        for (int u = v + 1; u < 4; ++u) {
          double t = a[u][v];
#pragma unroll
          for (int w = 0; w < v; ++w) t -= a[u][w] * a[v][w];
          a[u][v] = t * r;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) Dg[b][u][v] = (v <= u) ? a[u][v] : 0.0;
      if (f) fail = f;
    }
    __syncthreads();
    if (fail) break;
    if (tk == s && ti > s) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double t = a[u][v];
#pragma unroll
          for (int w = 0; w < v; ++w) t -= a[u][w] * Dg[b][v][w];
          a[u][v] = t * Dr[b][v];
          Pn[b][4 * ti + u][v] = a[u][v];
        }
    }
    __syncthreads();
    // Pn[b] and Dg[b] are next written at step s + 2, after every thread
    // has passed the first barrier of step s + 1
    if (low && tk > s) {
      double pi[4][4], pk[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          pi[u][w] = Pn[b][4 * ti + u][w];
          pk[u][w] = Pn[b][4 * tk + u][w];
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int w = 0; w < 4; ++w) a[u][v] -= pi[u][w] * pk[v][w];
    }
  }
  if (fail) {
    if (tid == 0) info[c] = j0 + fail;
    return;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * ti + u, k = 4 * tk + v;
      if (i < nb && k < nb) A[(size_t)(j0 + i) * n + j0 + k] = (k <= i) ? a[u][v] : 0.0;
    }
}

// Rows i >= j0+nb: L[i][j0:j0+nb] = A[i][j0:j0+nb] L_jj^{-T}, 64 rows per
// workgroup.  Step s: the threads of tile column s finish their tiles by
// substitution against diagonal tile s, then the tiles to the right
// subtract their products with L_jj's tile row.
__global__ __launch_bounds__(256) void chol_trsm_kernel(int n, int j0, double *L,
                                                        const int32_t *info) {
  const int c = blockIdx.y;
  if (info[c] != 0) return;
  double *A = L + (size_t)c * n * n;
  const int nb = min(NB, n - j0);
  const int rb = j0 + nb + blockIdx.x * 64;
  const int tid = threadIdx.x, ti = tid >> 4, tk = tid & 15;
  __shared__ double D[NB][NB + 1];  // L_jj, identity-padded past nb
  __shared__ double Rd[NB];         // reciprocals of its diagonal
  __shared__ double Xc[2][64][4];   // the step's solved tile column
  {
    // every load issued before the first LDS store
    const int k = tid & 63;
    double dv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = (tid >> 6) + 4 * q;
      dv[q] = (i < nb && k < nb) ? (k <= i ? A[(size_t)(j0 + i) * n + j0 + k] : 0.0)
                                 : (i == k ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) D[(tid >> 6) + 4 * q][k] = dv[q];
  }
  if (tid < NB) Rd[tid] = tid < nb ? 1.0 / A[(size_t)(j0 + tid) * n + j0 + tid] : 1.0;
  double a[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rb + 4 * ti + u, k = 4 * tk + v;
      a[u][v] = (i < n && k < nb) ? A[(size_t)i * n + j0 + k] : 0.0;
    }
  __syncthreads();
  for (int s = 0; s < NB / 4; ++s) {
    const int b = s & 1;
    if (tk == s) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double t = a[u][v];
#pragma unroll
          for (int w = 0; w < v; ++w) t -= a[u][w] * D[4 * s + v][4 * s + w];
          a[u][v] = t * Rd[4 * s + v];
          Xc[b][4 * ti + u][v] = a[u][v];
        }
    }
    __syncthreads();
    // Xc[b] is next written at step s + 2, after this step's readers have
    // passed the barrier of step s + 1
    if (tk > s) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int w = 0; w < 4; ++w) a[u][v] -= Xc[b][4 * ti + u][w] * D[4 * tk + v][4 * s + w];
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rb + 4 * ti + u, k = 4 * tk + v;
      if (i < n && k < nb) A[(size_t)i * n + j0 + k] = a[u][v];
    }
}

// Trailing update A[i][k] -= sum_c L[i][j0+c] L[k][j0+c] for r0 <= k <= i < n,
// 64x64 tiles of the lower triangle, 4x4 outputs per thread.
__global__ __launch_bounds__(256) void chol_syrk_kernel(int n, int j0, double *L,
                                                        const int32_t *info) {
  const int c = blockIdx.y;
  if (info[c] != 0) return;
  double *A = L + (size_t)c * n * n;
  const int nb = min(NB, n - j0);
  const int r0 = j0 + nb;
  // tile index -> (I, J) with I >= J
  const int t = blockIdx.x;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int i0 = r0 + I * 64, k0 = r0 + J * 64;
  __shared__ double LI[64][NB + 1];
  __shared__ double LJ[64][NB + 1];
  const int tid = threadIdx.x;
  const int ti = (tid >> 4) * 4, tk = (tid & 15) * 4;
  // this thread's outputs, fetched with the panels (their loads overlap)
  double old[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ti + u, k = k0 + tk + v;
      old[u][v] = (i < n && k < n && k <= i) ? A[(size_t)i * n + k] : 0.0;
    }
  if (nb == NB) {
    // a whole panel: every load issued before the first LDS store
    const int cc = tid & 63;
    double vi[16], vj[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = (tid >> 6) + 4 * q;
      vi[q] = (i0 + r < n) ? A[(size_t)(i0 + r) * n + j0 + cc] : 0.0;
      vj[q] = (k0 + r < n) ? A[(size_t)(k0 + r) * n + j0 + cc] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = (tid >> 6) + 4 * q;
      LI[r][cc] = vi[q];
      LJ[r][cc] = vj[q];
    }
  } else {
    for (int e = tid; e < 64 * nb; e += 256) {
      int r = e / nb, cc = e % nb;
      LI[r][cc] = (i0 + r < n) ? A[(size_t)(i0 + r) * n + j0 + cc] : 0.0;
      LJ[r][cc] = (k0 + r < n) ? A[(size_t)(k0 + r) * n + j0 + cc] : 0.0;
    }
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int cc = 0; cc < nb; ++cc) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = LI[ti + u][cc];
      b[u] = LJ[tk + u][cc];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int i = i0 + ti + u, k = k0 + tk + v;
      if (i < n && k < n && k <= i) A[(size_t)i * n + k] = old[u][v] - acc[u][v];
    }
}

__global__ void copy_lower_kernel(int C, int n, const double *A, double *L) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)C * n * n;
  for (; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e % ((int64_t)n * n);
    int i = (int)(r / n), k = (int)(r % n);
    L[e] = (k <= i) ? A[e] : 0.0;
  }
}

int chol_batched(int C, int n, const double *A, double *L, int32_t *info, hipStream_t s) {
  if (C <= 0 || n <= 0) return SB_OK;
  int st = launch_fill_i32(C, 0, info, s);
  if (st) return st;
  {
    int64_t total = (int64_t)C * n * n;
    unsigned blocks = (unsigned)std::min<int64_t>(8192, ceil_div(total, 256));
    hipLaunchKernelGGL(copy_lower_kernel, dim3(blocks), dim3(256), 0, s, C, n, A, L);
    SB_LAUNCH_CHECK();
  }
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int nb = std::min(NB, n - j0);
    hipLaunchKernelGGL(chol_diag_kernel, dim3(C), dim3(256), 0, s, n, j0, L, info);
    SB_LAUNCH_CHECK();
    const int rest = n - j0 - nb;
    if (rest <= 0) break;
    hipLaunchKernelGGL(chol_trsm_kernel, dim3((unsigned)ceil_div(rest, 64), C), dim3(256), 0, s, n,
                       j0, L, info);
    SB_LAUNCH_CHECK();
    const int T = (int)ceil_div(rest, 64);
    hipLaunchKernelGGL(chol_syrk_kernel, dim3((unsigned)(T * (T + 1) / 2), C), dim3(256), 0, s, n,
                       j0, L, info);
    SB_LAUNCH_CHECK();
  }
  return SB_OK;
}

// log det = 2 sum_i log L_ii from the factor (fixed-order reduction), NaN if it failed.
__global__ __launch_bounds__(256) void logdet_kernel(int n, const double *L,
                                                     const int32_t *info, double *logdet) {
  const int c = blockIdx.x;
  __shared__ double red[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += log(L[(size_t)c * n * n + (size_t)i * n + i]);
  v = block_sum<256>(v, red);
  if (threadIdx.x == 0) logdet[c] = info[c] ? NAN : 2.0 * v;
}

int launch_logdet(int C, int n, const double *L, const int32_t *info, double *logdet,
                  hipStream_t s) {
  if (C <= 0) return SB_OK;
  hipLaunchKernelGGL(logdet_kernel, dim3(C), dim3(256), 0, s, n, L, info, logdet);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Solve L L^T x = b: blocked forward (row dots over solved blocks, then the
// 64x64 diagonal block in one wave) and backward substitution.  One
// workgroup of 16 waves per matrix, x in LDS; the dots against the solved
// part are split over all waves with several independent loads per lane in
// flight (the solve is bound by the latency of reading L).
constexpr int SV_T = 1024, SV_W = SV_T / 64;
// Lane l's value to every lane (l uniform): two scalar reads, no LDS trip.
__device__ inline double lane_bcast(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__global__ __launch_bounds__(SV_T) void chol_solve_kernel(int n, const double *Lall,
                                                          const double *ball, double *xall,
                                                          const int32_t *info) {
  extern __shared__ double xs[];  // [n]
  __shared__ double part[SV_W][64];
  __shared__ double Tb[64][65];   // current diagonal block
  const int c = blockIdx.x;
  const double *L = Lall + (size_t)c * n * n;
  const double *b = ball + (size_t)c * n;
  double *x = xall + (size_t)c * n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (info && info[c] != 0) {
    for (int i = tid; i < n; i += SV_T) x[i] = NAN;
    return;
  }
  for (int i = tid; i < n; i += SV_T) xs[i] = b[i];
  __syncthreads();
  // forward: L z = b
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int nb = min(64, n - i0);
    for (int r = w; r < nb; r += SV_W)  // diagonal block into LDS, row by row
      if (lane < nb) Tb[r][lane] = L[(size_t)(i0 + r) * n + i0 + lane];
    // rows i0 + w + 16 q (q < 4) less sum_{k < i0} L[i][k] z_k; lanes split k.
    // Eight k values per lane per pass, their 32 loads issued before the
    // first product (the sums keep their order: k ascending per lane); a row
    // past the block reads row i0 and its sum is never used.
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double *Lr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = w + SV_W * q;
      Lr[q] = L + (size_t)(i0 + (r < nb ? r : 0)) * n;
    }
    int k = lane;
    for (; k + 64 * 7 < i0; k += 64 * 8) {
      double lv[8][4];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) lv[u][q] = Lr[q][k + 64 * u];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double zk = xs[k + 64 * u];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += lv[u][q] * zk;
      }
    }
    for (; k < i0; k += 64) {
      const double zk = xs[k];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += Lr[q][k] * zk;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double t = wave_sum(acc[q]);
      if (lane == 0) part[0][w + SV_W * q] = t;
    }
    __syncthreads();
    if (w == 0) {
      // lane cc holds the reciprocal of pivot cc; one division per lane
      const double rp = (lane < nb) ? 1.0 / Tb[lane][lane] : 1.0;
      double val = (lane < nb) ? xs[i0 + lane] - part[0][lane] : 0.0;
#pragma unroll 8
      for (int cc = 0; cc < nb; ++cc) {  // (unrolled: the Tb reads leave the chain)
        const double xc = lane_bcast(val * rp, cc);
        if (lane == cc) val = xc;
        if (lane > cc && lane < nb) val -= Tb[lane][cc] * xc;
      }
      if (lane < nb) xs[i0 + lane] = val;
    }
    __syncthreads();
  }
  // backward: L^T x = z
  for (int iend = n; iend > 0; iend -= 64) {
    const int i0 = max(0, iend - 64);
    const int nb = iend - i0;
    for (int r = w; r < nb; r += SV_W)
      if (lane < nb) Tb[r][lane] = L[(size_t)(i0 + r) * n + i0 + lane];
    // s_i = sum_{k >= iend} L[k][i] x_k for i in block; lanes index i, waves split k
    // (sixteen rows per pass, their loads issued before the first product;
    // k ascending per wave as before)
    double sacc = 0.0;
    if (lane < nb) {
      int k = iend + w;
      for (; k + SV_W * 15 < n; k += SV_W * 16) {
        double lv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) lv[u] = L[(size_t)(k + SV_W * u) * n + i0 + lane];
#pragma unroll
        for (int u = 0; u < 16; ++u) sacc += lv[u] * xs[k + SV_W * u];
      }
      for (; k < n; k += SV_W) sacc += L[(size_t)k * n + i0 + lane] * xs[k];
    }
    part[w][lane] = sacc;
    __syncthreads();
    if (w == 0) {
      double sv = part[0][lane];
#pragma unroll
      for (int u = 1; u < SV_W; ++u) sv += part[u][lane];
      double val = (lane < nb) ? xs[i0 + lane] - sv : 0.0;
      const double rp = (lane < nb) ? 1.0 / Tb[lane][lane] : 1.0;
#pragma unroll 8
      for (int cc = nb - 1; cc >= 0; --cc) {
        const double xc = lane_bcast(val * rp, cc);
        if (lane == cc) val = xc;
        if (lane < cc) val -= Tb[cc][lane] * xc;
      }
      if (lane < nb) xs[i0 + lane] = val;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += SV_T) x[i] = xs[i];
}

int launch_chol_solve(int C, int n, const double *L, const double *b, double *x,
                      const int32_t *info, hipStream_t s) {
  if (C <= 0) return SB_OK;
  size_t shm = sizeof(double) * (size_t)n;
  if (shm > 64 * 1024) {
    set_error("solve dimension %d too large", n);
    return SB_E_UNSUPPORTED;
  }
  hipLaunchKernelGGL(chol_solve_kernel, dim3(C), dim3(SV_T), shm, s, n, L, b, x, info);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb

// ====================================================================
// Uneven batches: matrix c has size n[c] and starts at off[c] (row-major,
// leading dimension n[c]); vectors of matrix c start at voff[c].  The panel
// loop runs to max n; a matrix whose size is reached skips the stage.
namespace sb {

__global__ __launch_bounds__(256) void chol_diag_u_kernel(int j0, const int32_t *nv,
                                                          const int64_t *off, double *L,
                                                          int32_t *info) {
  const int c = blockIdx.x;
  const int n = nv[c];
  if (j0 >= n || info[c] != 0) return;
  double *A = L + off[c];
  const int nb = min(NB, n - j0);
  const int tid = threadIdx.x;
  __shared__ double T[NB][NB + 1];
  __shared__ int fail;
  for (int e = tid; e < nb * nb; e += 256) {
    int i = e / nb, k = e % nb;
    T[i][k] = (k <= i) ? A[(size_t)(j0 + i) * n + j0 + k] : 0.0;
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int col = 0; col < nb; ++col) {
    if (tid == 0) {
      double p = T[col][col];
      if (!(p > 0.0))
        fail = col + 1;
      else
        T[col][col] = sqrt(p);
    }
    __syncthreads();
    if (fail) break;
    const double ljj = T[col][col];
    for (int i = col + 1 + tid; i < nb; i += 256) T[i][col] /= ljj;
    __syncthreads();
    const int rem = nb - col - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      int i = col + 1 + e / rem, k = col + 1 + e % rem;
      if (k <= i) T[i][k] -= T[i][col] * T[k][col];
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) info[c] = j0 + fail;
    return;
  }
  for (int e = tid; e < nb * nb; e += 256) {
    int i = e / nb, k = e % nb;
    A[(size_t)(j0 + i) * n + j0 + k] = (k <= i) ? T[i][k] : 0.0;
  }
}

__global__ __launch_bounds__(64) void chol_trsm_u_kernel(int j0, const int32_t *nv,
                                                         const int64_t *off, double *L,
                                                         const int32_t *info) {
  const int c = blockIdx.y;
  const int n = nv[c];
  if (j0 >= n || info[c] != 0) return;
  double *A = L + off[c];
  const int nb = min(NB, n - j0);
  const int r0 = j0 + nb;
  if (r0 + (int)blockIdx.x * 64 >= n) return;
  __shared__ double D[NB][NB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 64) {
    int i = e / nb, k = e % nb;
    D[i][k] = A[(size_t)(j0 + i) * n + j0 + k];
  }
  __syncthreads();
  const int i = r0 + blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  double *row = A + (size_t)i * n + j0;
  double x[NB];
#pragma unroll
  for (int cc = 0; cc < NB; ++cc) x[cc] = (cc < nb) ? row[cc] : 0.0;
#pragma unroll
  for (int cc = 0; cc < NB; ++cc) {
    if (cc < nb) {
      double s = x[cc];
#pragma unroll
      for (int t = 0; t < cc; ++t) s -= x[t] * D[cc][t];
      x[cc] = s / D[cc][cc];
    }
  }
#pragma unroll
  for (int cc = 0; cc < NB; ++cc)
    if (cc < nb) row[cc] = x[cc];
}

__global__ __launch_bounds__(256) void chol_syrk_u_kernel(int j0, const int32_t *nv,
                                                          const int64_t *off, double *L,
                                                          const int32_t *info) {
  const int c = blockIdx.y;
  const int n = nv[c];
  if (j0 >= n || info[c] != 0) return;
  double *A = L + off[c];
  const int nb = min(NB, n - j0);
  const int r0 = j0 + nb;
  const int rest = n - r0;
  if (rest <= 0) return;
  const int Tn = (rest + 63) / 64;
  const int t = blockIdx.x;
  if (t >= Tn * (Tn + 1) / 2) return;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int i0 = r0 + I * 64, k0 = r0 + J * 64;
  __shared__ double LI[64][NB + 1];
  __shared__ double LJ[64][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * nb; e += 256) {
    int r = e / nb, cc = e % nb;
    LI[r][cc] = (i0 + r < n) ? A[(size_t)(i0 + r) * n + j0 + cc] : 0.0;
    LJ[r][cc] = (k0 + r < n) ? A[(size_t)(k0 + r) * n + j0 + cc] : 0.0;
  }
  __syncthreads();
  const int ti = (tid >> 4) * 4, tk = (tid & 15) * 4;
  double acc[4][4] = {};
  for (int cc = 0; cc < nb; ++cc) {
    double a[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = LI[ti + u][cc];
      bv[u] = LJ[tk + u][cc];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * bv[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int i = i0 + ti + u, k = k0 + tk + v;
      if (i < n && k < n && k <= i) A[(size_t)i * n + k] -= acc[u][v];
    }
}

__global__ void zero_upper_u_kernel(int C, const int32_t *nv, const int64_t *off, double *L) {
  const int c = blockIdx.y;
  if (c >= C) return;
  const int n = nv[c];
  const int64_t tot = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), k = (int)(e % n);
    if (k > i) L[off[c] + e] = 0.0;
  }
}

// In-place factorisation of C matrices of sizes nv[c] at offsets off[c].
int chol_batched_u(int C, const int32_t *nv, const int64_t *off, int n_max, double *L,
                   int32_t *info, hipStream_t s) {
  if (C <= 0 || n_max <= 0) return SB_OK;
  int st = launch_fill_i32(C, 0, info, s);
  if (st) return st;
  hipLaunchKernelGGL(zero_upper_u_kernel, dim3((unsigned)std::min<int64_t>(64, ceil_div((int64_t)n_max * n_max, 256)), C),
                     dim3(256), 0, s, C, nv, off, L);
  SB_LAUNCH_CHECK();
  for (int j0 = 0; j0 < n_max; j0 += NB) {
    hipLaunchKernelGGL(chol_diag_u_kernel, dim3(C), dim3(256), 0, s, j0, nv, off, L, info);
    const int rest = n_max - j0 - std::min(NB, n_max - j0);
    if (rest <= 0) {
      SB_LAUNCH_CHECK();
      break;
    }
    hipLaunchKernelGGL(chol_trsm_u_kernel, dim3((unsigned)ceil_div(rest, 64), C), dim3(64), 0, s,
                       j0, nv, off, L, info);
    const int T = (int)ceil_div(rest, 64);
    hipLaunchKernelGGL(chol_syrk_u_kernel, dim3((unsigned)(T * (T + 1) / 2), C), dim3(256), 0, s,
                       j0, nv, off, L, info);
    SB_LAUNCH_CHECK();
  }
  return SB_OK;
}

__global__ __launch_bounds__(256) void logdet_u_kernel(const int32_t *nv, const int64_t *off,
                                                       const double *L, const int32_t *info,
                                                       double *logdet) {
  const int c = blockIdx.x;
  const int n = nv[c];
  __shared__ double red[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += log(L[off[c] + (size_t)i * n + i]);
  v = block_sum<256>(v, red);
  if (threadIdx.x == 0) logdet[c] = info[c] ? NAN : 2.0 * v;
}

int launch_logdet_u(int C, const int32_t *nv, const int64_t *off, const double *L,
                    const int32_t *info, double *logdet, hipStream_t s) {
  if (C <= 0) return SB_OK;
  hipLaunchKernelGGL(logdet_u_kernel, dim3(C), dim3(256), 0, s, nv, off, L, info, logdet);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Solve L L^T x = b for matrix c (size nv[c]); b and x rows start at c * vs.
__global__ __launch_bounds__(256) void chol_solve_u_kernel(const int32_t *nv, const int64_t *off,
                                                           const double *Lall, const double *ball,
                                                           double *xall, int64_t vs,
                                                           const int32_t *info) {
  extern __shared__ double xs[];
  __shared__ double part[4][64];
  __shared__ double Tb[64][65];
  const int c = blockIdx.x;
  const int n = nv[c];
  const double *L = Lall + off[c];
  const double *b = ball + (size_t)c * vs;
  double *x = xall + (size_t)c * vs;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (info && info[c] != 0) {
    for (int i = tid; i < n; i += 256) x[i] = NAN;
    return;
  }
  for (int i = tid; i < n; i += 256) xs[i] = b[i];
  __syncthreads();
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int nb = min(64, n - i0);
    for (int rr = 0; rr < 16; ++rr) {
      const int r = w * 16 + rr;
      double sacc = 0.0;
      if (r < nb)
#pragma unroll 8
        for (int k = lane; k < i0; k += 64) sacc += L[(size_t)(i0 + r) * n + k] * xs[k];
      sacc = wave_sum(sacc);
      if (lane == 0) part[0][r] = sacc;
    }
    for (int r = w; r < nb; r += 4)  // diagonal block into LDS, row by row
      if (lane < nb) Tb[r][lane] = L[(size_t)(i0 + r) * n + i0 + lane];
    __syncthreads();
    if (w == 0) {
      double val = (lane < nb) ? xs[i0 + lane] - part[0][lane] : 0.0;
      for (int cc = 0; cc < nb; ++cc) {
        double xc = __shfl(val / Tb[cc][cc], cc, 64);
        if (lane == cc) val = xc;
        if (lane > cc && lane < nb) val -= Tb[lane][cc] * xc;
      }
      if (lane < nb) xs[i0 + lane] = val;
    }
    __syncthreads();
  }
  for (int iend = n; iend > 0; iend -= 64) {
    const int i0 = max(0, iend - 64);
    const int nb = iend - i0;
    double sacc = 0.0;
    if (lane < nb)
#pragma unroll 8
      for (int k = iend + w; k < n; k += 4) sacc += L[(size_t)k * n + i0 + lane] * xs[k];
    part[w][lane] = sacc;
    for (int r = w; r < nb; r += 4)
      if (lane < nb) Tb[r][lane] = L[(size_t)(i0 + r) * n + i0 + lane];
    __syncthreads();
    if (w == 0) {
      double sv = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
      double val = (lane < nb) ? xs[i0 + lane] - sv : 0.0;
      for (int cc = nb - 1; cc >= 0; --cc) {
        double xc = __shfl(val / Tb[cc][cc], cc, 64);
        if (lane == cc) val = xc;
        if (lane < cc) val -= Tb[cc][lane] * xc;
      }
      if (lane < nb) xs[i0 + lane] = val;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += 256) x[i] = xs[i];
}

int launch_chol_solve_u(int C, const int32_t *nv, const int64_t *off, int n_max, const double *L,
                        const double *b, double *x, int64_t vs, const int32_t *info,
                        hipStream_t s) {
  if (C <= 0) return SB_OK;
  const size_t shm = sizeof(double) * (size_t)n_max;
  if (shm > 64 * 1024) {
    set_error("solve dimension %d too large", n_max);
    return SB_E_UNSUPPORTED;
  }
  hipLaunchKernelGGL(chol_solve_u_kernel, dim3(C), dim3(256), shm, s, nv, off, L, b, x, vs, info);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
