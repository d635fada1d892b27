// Sampler handoff of GraspBirdsTail (section "Module 4: GraspBirdsTail":
// compacted likelihood, exports): the points theta* + V_inform phi of the
// reduced coordinates, the chain rule back to phi, and the bounds of the
// reduced box.
#include "internal.h"

namespace sb {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

// C[b][n] = c0[n] + sum_k A[b][k] Bm(k, n), Bm(k, n) = Bp[k sk + n sn]
// (c0 nullable), FP64 16x16x4 MFMAs: a workgroup of four waves takes 16 rows
// and 64 columns, each wave one 16 x 16 block; operands straight from the
// L2, four k-steps' loads issued before their MFMAs.
__global__ __launch_bounds__(256) void small_gemm_f64_kernel(int64_t B, int N, int Kd,
                                                             const double *A, int64_t lda,
                                                             const double *Bp, int64_t sk,
                                                             int64_t sn, const double *c0,
                                                             double *C, int64_t ldc) {
  const int64_t b0 = (int64_t)blockIdx.x * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n0 = blockIdx.y * 64 + wave * 16;
  if (b0 >= B || n0 >= N) return;
  const int fr = lane & 15, fg = lane >> 4;
  const int64_t ra = b0 + fr;
  const int nb = n0 + fr;
  d4v acc = d4v{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < Kd; k0 += 16) {
    double a[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + fg;
      a[u] = (ra < B && k < Kd) ? A[ra * lda + k] : 0.0;
      bv[u] = (nb < N && k < Kd) ? Bp[(int64_t)k * sk + (int64_t)nb * sn] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bv[u], acc, 0, 0, 0);
  }
  // item v of lane l: row l / 16 + 4 v, column l % 16 of the block
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = b0 + fg + 4 * v;
    if (row < B && nb < N) C[row * ldc + nb] = (c0 ? c0[nb] : 0.0) + acc[v];
  }
}

// One wave per direction i: the interval of t with theta* + t V[:, i] in the
// box, the intersection over coordinates with V_ji != 0.
__global__ __launch_bounds__(256) void reduced_bounds_kernel(int d, const double *th,
                                                             const double *V, int64_t ldv, int r,
                                                             const double *lo, const double *hi,
                                                             double *plo, double *phi) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= r) return;
  double a = -INFINITY, b = INFINITY;
  for (int j = lane; j < d; j += 64) {
    const double v = V[(int64_t)j * ldv + i];
    if (v != 0.0) {
      const double t1 = (lo[j] - th[j]) / v, t2 = (hi[j] - th[j]) / v;
      a = fmax(a, fmin(t1, t2));
      b = fmin(b, fmax(t1, t2));
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    a = fmax(a, __shfl_xor(a, o, 64));
    b = fmin(b, __shfl_xor(b, o, 64));
  }
  if (lane == 0) {
    plo[i] = a;
    phi[i] = b;
  }
}

}  // namespace

int launch_small_gemm_f64(int64_t B, int N, int Kd, const double *A, int64_t lda, const double *Bp,
                          int64_t sk, int64_t sn, const double *c0, double *C, int64_t ldc,
                          hipStream_t s) {
  if (B <= 0 || N <= 0) return SB_OK;
  const int64_t gx = ceil_div(B, 16);
  if (gx > 0x7fffffffll) {
    set_error("small GEMM: %lld rows in one launch", (long long)B);
    return SB_E_UNSUPPORTED;
  }
  hipLaunchKernelGGL(small_gemm_f64_kernel, dim3((unsigned)gx, (unsigned)ceil_div(N, 64)),
                     dim3(256), 0, s, B, N, Kd, A, lda, Bp, sk, sn, c0, C, ldc);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int launch_reduced_bounds(int d, const double *th, const double *V, int64_t ldv, int r,
                          const double *lo, const double *hi, double *plo, double *phi,
                          hipStream_t s) {
  if (r <= 0) return SB_OK;
  hipLaunchKernelGGL(reduced_bounds_kernel, dim3((unsigned)ceil_div(r, 4)), dim3(256), 0, s, d,
                     th, V, ldv, r, lo, hi, plo, phi);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
