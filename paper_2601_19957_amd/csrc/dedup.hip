// Mode de-duplication and the Laplace combine.
//
// Dedup is L-infinity leader clustering (ChiSao / GreenDragon dedup; the
// appendix on the L-infinity metric): candidates are visited by l descending
// (ties: lower index) and each joins the first representative within tau,
// else founds one.  The same partition is produced in rounds: the
// highest-ranked unassigned candidate becomes the next representative and
// every unassigned candidate within tau of it joins it.  (A candidate that is
// not within tau of representatives 1..j-1 is still unassigned when
// representative j is chosen, and j precedes it in the visiting order, so it
// joins the first representative within tau, as in the sequential rule.)
// Each round is one argmax kernel and one distance kernel.
//
// Combine: log Z_k = l_k - log V + (d/2) log 2 pi - (1/2) log det H_k
// (Laplace with the uniform prior, appendix eq. "laplace"), modes sorted by
// log Z_k descending (ties lexicographic in theta), log Z = max + log sum
// exp(. - max) over the sorted list (appendix "Log-Sum-Exp Stability").
#include <algorithm>

#include "internal.h"

namespace sb {

// better(a, b): a precedes b in the visiting order
__device__ inline bool key_before(double la, int ia, double lb, int ib) {
  if (la != la) la = -INFINITY;
  if (lb != lb) lb = -INFINITY;
  return (la > lb) || (la == lb && ia < ib);
}

template <typename TL>
__global__ __launch_bounds__(1024) void leader_kernel(int C, const TL *l, const uint8_t *valid,
                                                      const int32_t *rep_of, int32_t *state,
                                                      int32_t *reps, int max_reps) {
  // state[0] = current leader (-1 none), state[1] = number of reps, state[2] = done flag
  if (state[2]) return;
  __shared__ double bl[1024];
  __shared__ int bi[1024];
  const int t = threadIdx.x;
  double best = -INFINITY;
  int bidx = -1;
  for (int c = t; c < C; c += 1024) {
    if ((valid && !valid[c]) || rep_of[c] >= 0) continue;
    double v = (double)l[c];
    if (bidx < 0 || key_before(v, c, best, bidx)) {
      best = v;
      bidx = c;
    }
  }
  bl[t] = best;
  bi[t] = bidx;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      int j = bi[t + o];
      if (j >= 0 && (bi[t] < 0 || key_before(bl[t + o], j, bl[t], bi[t]))) {
        bl[t] = bl[t + o];
        bi[t] = j;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const int lead = bi[0];
    state[0] = lead;
    if (lead < 0) {
      state[2] = 1;
    } else {
      if (state[1] < max_reps) reps[state[1]] = lead;
      state[1] += 1;
    }
  }
}

// One wave per candidate: join the current leader if within tau (L-infinity).
template <typename T>
__global__ __launch_bounds__(256) void assign_kernel(int C, int d, const T *X, const uint8_t *valid,
                                                     int32_t *rep_of, const int32_t *state,
                                                     double tau) {
  const int lead = state[0];
  if (lead < 0) return;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= C) return;
  if ((valid && !valid[c]) || rep_of[c] >= 0) return;
  const T *a = X + (size_t)c * d, *b = X + (size_t)lead * d;
  double m = 0.0;
  for (int i = lane; i < d; i += 64) m = fmax(m, fabs((double)a[i] - (double)b[i]));
  m = wave_max(m);
  if (lane == 0 && (c == lead || m <= tau)) rep_of[c] = lead;
}

size_t dedup_ws_bytes(int C) { return align_up(sizeof(int32_t) * 8) + 256; }

int dedup_run(int C, int d, const void *X, int x_dtype, const void *l, int l_dtype,
              const uint8_t *valid, double tau, int32_t *rep_of, int32_t *reps, int max_reps,
              int *n_reps, Arena &ar, hipStream_t s) {
  *n_reps = 0;
  if (C <= 0) return SB_OK;
  int32_t *state = ar.take<int32_t>(8);
  if (!state) return SB_E_NOMEM;
  int st = launch_fill_i32(C, -1, rep_of, s);
  if (st) return st;
  st = launch_fill_i32(8, 0, state, s);
  if (st) return st;
  int32_t host_state[3] = {0, 0, 0};
  const int chunk = 8;
  for (int round = 0; round <= C; round += chunk) {
    for (int k = 0; k < chunk; ++k) {
      if (l_dtype == DT_F64)
        hipLaunchKernelGGL(leader_kernel<double>, dim3(1), dim3(1024), 0, s, C,
                           (const double *)l, valid, rep_of, state, reps, max_reps);
      else
        hipLaunchKernelGGL(leader_kernel<float>, dim3(1), dim3(1024), 0, s, C, (const float *)l,
                           valid, rep_of, state, reps, max_reps);
      if (x_dtype == DT_F64)
        hipLaunchKernelGGL(assign_kernel<double>, dim3((unsigned)ceil_div(C, 4)), dim3(256), 0,
                           s, C, d, (const double *)X, valid, rep_of, state, tau);
      else
        hipLaunchKernelGGL(assign_kernel<float>, dim3((unsigned)ceil_div(C, 4)), dim3(256), 0, s,
                           C, d, (const float *)X, valid, rep_of, state, tau);
      SB_LAUNCH_CHECK();
    }
    SB_HIP(hipMemcpyAsync(host_state, state, sizeof(host_state), hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
    if (host_state[2]) break;
  }
  *n_reps = host_state[1];
  return (host_state[1] > max_reps) ? SB_E_CAPACITY : SB_OK;
}

// ----------------------------------------------------------------- combine

__global__ __launch_bounds__(256) void combine_kernel(int n, int d, const double *lo,
                                                      const double *hi, const double *logl,
                                                      const double *logdet, const double *modes,
                                                      int32_t *order, double *mode_log_z,
                                                      double *log_z) {
  __shared__ double red[4];
  __shared__ double lzs[1024];
  __shared__ double sorted[1024];
  double v = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) v += log(hi[i] - lo[i]);
  const double logv = block_sum<256>(v, red);
  for (int i = threadIdx.x; i < n; i += 256)
    lzs[i] = logl[i] - logv + 0.5 * (double)d * kLog2Pi - 0.5 * logdet[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      bool before = lzs[j] > lzs[i];
      if (lzs[j] == lzs[i]) {
        int cmp = 0;
        for (int t = 0; t < d && cmp == 0; ++t) {
          double a = modes[(size_t)j * d + t], b = modes[(size_t)i * d + t];
          cmp = (a < b) ? -1 : (a > b ? 1 : 0);
        }
        before = (cmp < 0) || (cmp == 0 && j < i);
      }
      rank += before;
    }
    order[rank] = i;
    sorted[rank] = lzs[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < n; ++i) mode_log_z[i] = sorted[i];
    double mx = -INFINITY;
    for (int i = 0; i < n; ++i) mx = fmax(mx, sorted[i]);
    double res;
    if (n == 0 || mx == -INFINITY || mx == INFINITY) {
      res = (n == 0) ? -INFINITY : mx;
    } else {
      double sacc = 0.0;
      for (int i = 0; i < n; ++i) sacc += exp(sorted[i] - mx);
      res = mx + log(sacc);
    }
    log_z[0] = res;
  }
}

int launch_combine(int n, int d, const double *lo, const double *hi, const double *logl,
                   const double *logdet, const double *modes, int32_t *order, double *mode_log_z,
                   double *log_z, hipStream_t s) {
  if (n > 1024) {
    set_error("combine supports at most 1024 modes");
    return SB_E_UNSUPPORTED;
  }
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(256), 0, s, n, d, lo, hi, logl, logdet, modes,
                     order, mode_log_z, log_z);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb

// ====================================================================
// Batches: the leader rounds of every problem run together (one argmax
// workgroup per problem, one distance wave per candidate); the combine runs
// one workgroup per problem.
namespace sb {

__device__ inline int find_first(const int64_t *first, int n, int64_t c) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= c)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// state: [n] leader, [n] nrep, [n] done, [1] number of problems done
__global__ __launch_bounds__(1024) void leader_group_kernel(int n, const int64_t *cfirst,
                                                            const int64_t *ccount,
                                                            const double *l,
                                                            const uint8_t *valid,
                                                            const int32_t *rep_of, int32_t *state,
                                                            const int64_t *rbase,
                                                            const int32_t *rcap, int32_t *reps) {
  const int p = blockIdx.x;
  int32_t *leader = state, *nrep = state + n, *done = state + 2 * n, *ndone = state + 3 * n;
  if (done[p]) return;
  __shared__ double bl[1024];
  __shared__ int64_t bi[1024];
  const int t = threadIdx.x;
  double best = -INFINITY;
  int64_t bidx = -1;
  for (int64_t c = cfirst[p] + t; c < cfirst[p] + ccount[p]; c += 1024) {
    if ((valid && !valid[c]) || rep_of[c] >= 0) continue;
    const double v = l[c];
    if (bidx < 0 || key_before(v, (int)(c - cfirst[p]), best, (int)(bidx - cfirst[p]))) {
      best = v;
      bidx = c;
    }
  }
  bl[t] = best;
  bi[t] = bidx;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      const int64_t j = bi[t + o];
      if (j >= 0 &&
          (bi[t] < 0 || key_before(bl[t + o], (int)(j - cfirst[p]), bl[t], (int)(bi[t] - cfirst[p])))) {
        bl[t] = bl[t + o];
        bi[t] = j;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const int64_t lead = bi[0];
    if (lead < 0 || nrep[p] >= rcap[p]) {
      // no candidate left, or one more representative than the capacity
      // (nrep = rcap + 1 flags the overflow); the problem is finished
      if (lead >= 0) nrep[p] = rcap[p] + 1;
      leader[p] = -1;
      done[p] = 1;
      atomicAdd(ndone, 1);
    } else {
      leader[p] = (int32_t)lead;
      reps[rbase[p] + nrep[p]] = (int32_t)lead;
      nrep[p] += 1;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void assign_group_kernel(int n, int64_t Ctot,
                                                           const int64_t *cfirst,
                                                           const BatchProb *probs,
                                                           const T *X, const int64_t *xoff,
                                                           const uint8_t *valid, int32_t *rep_of,
                                                           const int32_t *state,
                                                           const double *ptau) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= Ctot) return;
  const int p = find_first(cfirst, n, c);
  const int lead = state[p];
  if (lead < 0 || state[2 * n + p]) return;
  if ((valid && !valid[c]) || rep_of[c] >= 0) return;
  const int d = probs[p].d;
  const T *a = X + xoff[c], *b = X + xoff[lead];
  double m = 0.0;
  for (int i = lane; i < d; i += 64) m = fmax(m, fabs((double)a[i] - (double)b[i]));
  m = wave_max(m);
  if (lane == 0 && (c == lead || m <= ptau[p])) rep_of[c] = lead;
}

int dedup_group_run(int n, int64_t Ctot, const int64_t *cfirst, const int64_t *ccount,
                    const BatchProb *probs, const void *X, int x_dtype, const int64_t *xoff,
                    const double *l, const uint8_t *valid, const double *ptau, int32_t *rep_of,
                    const int64_t *rbase, const int32_t *rcap, int32_t *reps, int32_t *state,
                    int64_t max_rounds, hipStream_t s) {
  if (n <= 0) return SB_OK;
  int st = launch_fill_i32(3 * n + 1, 0, state, s);
  if (st) return st;
  if (Ctot <= 0) return SB_OK;
  if ((st = launch_fill_i32(Ctot, -1, rep_of, s))) return st;
  int32_t ndone = 0;
  const int chunk = 8;
  for (int64_t round = 0; round <= max_rounds; round += chunk) {
    for (int k = 0; k < chunk; ++k) {
      hipLaunchKernelGGL(leader_group_kernel, dim3(n), dim3(1024), 0, s, n, cfirst, ccount, l,
                         valid, rep_of, state, rbase, rcap, reps);
      if (x_dtype == DT_F64)
        hipLaunchKernelGGL(assign_group_kernel<double>, dim3((unsigned)ceil_div(Ctot, 4)),
                           dim3(256), 0, s, n, Ctot, cfirst, probs, (const double *)X, xoff,
                           valid, rep_of, state, ptau);
      else
        hipLaunchKernelGGL(assign_group_kernel<float>, dim3((unsigned)ceil_div(Ctot, 4)),
                           dim3(256), 0, s, n, Ctot, cfirst, probs, (const float *)X, xoff, valid,
                           rep_of, state, ptau);
      SB_LAUNCH_CHECK();
    }
    SB_HIP(hipMemcpyAsync(&ndone, state + 3 * n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
    if (ndone >= n) break;
  }
  return SB_OK;
}

// One workgroup per problem: log Z_k of its modes (reps[rbase + j], j < nrep,
// candidate data l, logdet, X + xoff), sorted descending (ties lexicographic
// in theta), log Z = logsumexp in that order.  Writes order (candidate
// indices) and mlz at rbase + rank, and log_z[p] (NaN when nrep > cap or the
// problem has no modes: -inf).
__global__ __launch_bounds__(256) void combine_group_kernel(BatchDev b, const int32_t *state,
                                                            const int64_t *rbase,
                                                            const int32_t *rcap,
                                                            const int32_t *reps, const double *l,
                                                            const double *logdet, const double *X,
                                                            const int64_t *xoff, int32_t *order,
                                                            double *mlz, double *log_z) {
  const int p = blockIdx.x;
  const BatchProb pr = b.probs[p];
  const int nm = state[b.n + p];
  __shared__ double red[4];
  __shared__ double lzs[1024];
  __shared__ double sorted[1024];
  if (nm > rcap[p] || nm > 1024) {
    if (threadIdx.x == 0) log_z[p] = NAN;
    return;
  }
  const int d = pr.d;
  const double *lo = b.lo + pr.box_off, *hi = b.hi + pr.box_off;
  double v = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) v += log(hi[i] - lo[i]);
  const double logv = block_sum<256>(v, red);
  const int32_t *rp = reps + rbase[p];
  for (int i = threadIdx.x; i < nm; i += 256)
    lzs[i] = l[rp[i]] - logv + 0.5 * (double)d * kLog2Pi - 0.5 * logdet[rp[i]];
  __syncthreads();
  for (int i = threadIdx.x; i < nm; i += 256) {
    int rank = 0;
    for (int j = 0; j < nm; ++j) {
      if (j == i) continue;
      bool before = lzs[j] > lzs[i];
      if (lzs[j] == lzs[i]) {
        int cmp = 0;
        const double *xa = X + xoff[rp[j]], *xb = X + xoff[rp[i]];
        for (int t = 0; t < d && cmp == 0; ++t) cmp = (xa[t] < xb[t]) ? -1 : (xa[t] > xb[t] ? 1 : 0);
        before = (cmp < 0) || (cmp == 0 && j < i);
      }
      rank += before;
    }
    order[rbase[p] + rank] = rp[i];
    sorted[rank] = lzs[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < nm; ++i) mlz[rbase[p] + i] = sorted[i];
    double mx = -INFINITY;
    for (int i = 0; i < nm; ++i) mx = fmax(mx, sorted[i]);
    double res;
    if (nm == 0 || mx == -INFINITY || mx == INFINITY) {
      res = (nm == 0) ? -INFINITY : mx;
    } else {
      double sacc = 0.0;
      for (int i = 0; i < nm; ++i) sacc += exp(sorted[i] - mx);
      res = mx + log(sacc);
    }
    log_z[p] = res;
  }
}

int launch_combine_group(const BatchDev &b, const int32_t *state, const int64_t *rbase,
                         const int32_t *rcap, const int32_t *reps, const double *l,
                         const double *logdet, const double *X, const int64_t *xoff,
                         int32_t *order, double *mlz, double *log_z, hipStream_t s) {
  hipLaunchKernelGGL(combine_group_kernel, dim3(b.n), dim3(256), 0, s, b, state, rbase, rcap, reps,
                     l, logdet, X, xoff, order, mlz, log_z);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
