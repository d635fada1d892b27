// Mixture row scalars shared by the contraction epilogues (two-launch and
// fused paths).
#pragma once

#include "internal.h"

namespace sb {

constexpr int kMaxK = 16;

// Mixture row: q_k from its tile partials, a_k = beta_k - q_k/2, lse =
// logsumexp_k a_k and the responsibilities r_k = exp(a_k - lse) in T (FP64
// arithmetic).  Shared by the epilogue and the active-component lists, so
// both see the same zero responsibilities.
template <typename T>
__device__ inline void mixture_resp(const Model &m, const T *qp, int ntn, double &lse,
                                    T (&r)[kMaxK]) {
  const int K = m.K;
  double a[kMaxK];
  double mx = -INFINITY;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) {
    if (k < K) {
      double q = 0;
      for (int t = 0; t < ntn; ++t) q += (double)qp[k * ntn + t];
      a[k] = m.beta[k] - 0.5 * q;
      mx = fmax(mx, a[k]);
    }
  }
  if (K == 1) {
    lse = a[0];
  } else {
    double ssum = 0;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < K) ssum += exp(a[k] - mx);
    lse = mx + log(ssum);
  }
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) r[k] = (k < K) ? (K == 1 ? (T)1 : (T)exp(a[k] - lse)) : (T)0;
}

}  // namespace sb
