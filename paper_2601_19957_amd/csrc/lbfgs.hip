// Batched L-BFGS on f = -l, one workgroup per start (appendix "L-BFGS
// Optimization"; batched over samples as the paper describes).
//
// Each start is a small state machine advanced once per batch step:
//   INIT      the start point has been evaluated: choose the first direction.
//   TRIAL     the trial x + alpha p has been evaluated: Armijo test
//             f(x_t) <= f(x) + 1e-4 alpha g^T p.  Accept -> store (s, y) if
//             s^T y > 1e-10 |s| |y|, compute the next direction by the
//             two-loop recursion; reject -> halve alpha (at most 40 times;
//             then clear the history and retry steepest descent once, else
//             the start is stalled).
// Starts stop when ||grad l||_inf <= tol or after max_iter accepted steps.
// The first direction, and any direction after a history reset or a
// non-descent two-loop result, is -g / max(1, ||g||_inf).
//
// Points and gradients are double-buffered per start (slots 0/1, `cur` names
// the accepted point), so accepting a trial swaps a slot index instead of
// copying.  The history S, Y [B][m][d] is a ring in memory; the kernel loads
// it into registers in logical order (oldest first) and runs both loops of
// the recursion with workgroup reductions for the dot products.
#include <algorithm>

#include "internal.h"

namespace sb {

enum { PH_INIT = 0, PH_TRIAL = 1 };
enum { ST_ACTIVE = 0, ST_CONVERGED = 1, ST_STALLED = 2, ST_MAXITER = 3, ST_DEAD = 4 };

template <typename T>
struct LbArgs {
  int64_t B;
  int d, m, max_iter;
  T tol;
  T *X, *G, *Pd, *S, *Yh, *rho, *yy, *alpha, *gtp;
  double *F;  // l at both slots, FP64 for every operand type
  int32_t *cur, *head, *cnt, *iters, *ls, *status, *phase, *rowid, *active;
  // per-start vector offset and length (nullable: s * d and d), and the
  // element offset of each start's trial row (nullable)
  const int64_t *voff;
  const int32_t *vdim;
  int64_t *rowoff;
  int64_t Ltot;
  // batches: problem of each start, per-problem tolerance and iteration cap
  // (nullable: tol / max_iter), and the first start of this launch
  const int32_t *sprob;
  const double *ptol;
  const int32_t *pmaxit;
  int64_t s_base, s_count;  // starts [s_base, s_base + s_count) of this launch
  int32_t *count_reset;     // compaction count, zeroed by this launch (nullable)
};

// A thread's chunk [i0, i0 + EPT) of a length-d vector (i0 = tid * EPT):
// one vector access when `vec` (d and the base offset multiples of EPT, so
// the chunk is aligned) and the chunk is whole, else element by element.
template <typename T, int EPT>
__device__ inline void vload(const T *p, int i0, int d, bool vec, T (&v)[EPT]) {
  if constexpr (EPT > 1) {
    typedef T vt __attribute__((ext_vector_type(EPT)));
    if (vec && i0 + EPT <= d) {
      const vt w = *(const vt *)(p + i0);
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = w[e];
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) v[e] = (i0 + e < d) ? p[i0 + e] : (T)0;
}
template <typename T, int EPT>
__device__ inline void vstore(T *p, int i0, int d, bool vec, const T (&v)[EPT]) {
  if constexpr (EPT > 1) {
    typedef T vt __attribute__((ext_vector_type(EPT)));
    if (vec && i0 + EPT <= d) {
      vt w;
#pragma unroll
      for (int e = 0; e < EPT; ++e) w[e] = v[e];
      *(vt *)(p + i0) = w;
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (i0 + e < d) p[i0 + e] = v[e];
}

// Streaming variants for the history ring, read and written once per step and
// not again before the whole batch has moved several times the size of the
// last-level cache: non-temporal accesses keep it from displacing the points
// and gradients the contraction reads next.
template <typename T, int EPT>
__device__ inline void vload_nt(const T *p, int i0, int d, bool vec, T (&v)[EPT]) {
  if constexpr (EPT > 1) {
    typedef T vt __attribute__((ext_vector_type(EPT)));
    if (vec && i0 + EPT <= d) {
      const vt w = __builtin_nontemporal_load((const vt *)(p + i0));
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = w[e];
      return;
    }
  }
  vload<T, EPT>(p, i0, d, vec, v);
}
template <typename T, int EPT>
__device__ inline void vstore_nt(T *p, int i0, int d, bool vec, const T (&v)[EPT]) {
  if constexpr (EPT > 1) {
    typedef T vt __attribute__((ext_vector_type(EPT)));
    if (vec && i0 + EPT <= d) {
      vt w;
#pragma unroll
      for (int e = 0; e < EPT; ++e) w[e] = v[e];
      __builtin_nontemporal_store(w, (vt *)(p + i0));
      return;
    }
  }
  vstore<T, EPT>(p, i0, d, vec, v);
}

// The history ring in BF16 (FP32 starts): a thread's EPT values as EPT
// 16-bit words, widened on load (exact) and rounded to nearest on store; the
// pair is rounded before any use, so the stored values are the ones used.
__device__ inline float bf16_round(float v) {
  const __bf16 h = (__bf16)v;
  return (float)h;
}
template <int EPT>
__device__ inline void hload_nt(const uint16_t *p, int i0, int d, bool vec, float (&v)[EPT]) {
  if constexpr (EPT == 4) {
    if (vec && i0 + 4 <= d) {
      typedef uint32_t u2v __attribute__((ext_vector_type(2)));
      const u2v w = __builtin_nontemporal_load((const u2v *)(p + i0));
      v[0] = __builtin_bit_cast(float, w[0] << 16);
      v[1] = __builtin_bit_cast(float, w[0] & 0xffff0000u);
      v[2] = __builtin_bit_cast(float, w[1] << 16);
      v[3] = __builtin_bit_cast(float, w[1] & 0xffff0000u);
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    v[e] = (i0 + e < d) ? __builtin_bit_cast(float, (uint32_t)p[i0 + e] << 16) : 0.f;
}
template <int EPT>
__device__ inline void hstore_nt(uint16_t *p, int i0, int d, bool vec, const float (&v)[EPT]) {
  // (v already holds BF16 values: the top 16 bits are exact)
  auto pk = [&](int e) {
    return (__builtin_bit_cast(uint32_t, v[e]) >> 16) |
           (__builtin_bit_cast(uint32_t, v[e + 1]) & 0xffff0000u);
  };
  if constexpr (EPT % 8 == 0) {
    if (vec && i0 + EPT <= d) {
      typedef uint32_t u4v __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int q = 0; q < EPT; q += 8) {
        u4v w;
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = pk(q + 2 * e);
        __builtin_nontemporal_store(w, (u4v *)(p + i0 + q));
      }
      return;
    }
  }
  if constexpr (EPT == 4) {
    if (vec && i0 + 4 <= d) {
      typedef uint32_t u2v __attribute__((ext_vector_type(2)));
      u2v w;
      w[0] = pk(0);
      w[1] = pk(2);
      __builtin_nontemporal_store(w, (u2v *)(p + i0));
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (i0 + e < d) p[i0 + e] = (uint16_t)(__builtin_bit_cast(uint32_t, v[e]) >> 16);
}
// The raw words of a thread's EPT BF16 values (EPT even, whole aligned
// chunk), kept packed in registers: no conversion between the loads, so the
// loads of a whole history issue back to back.
template <int EPT>
__device__ inline void hload_raw_nt(const uint16_t *p, int i0, uint32_t (&w)[EPT / 2]) {
  static_assert(EPT % 2 == 0, "whole 32-bit words");
  typedef uint32_t u2v __attribute__((ext_vector_type(2)));
  typedef uint32_t u4v __attribute__((ext_vector_type(4)));
  if constexpr (EPT % 8 == 0) {
#pragma unroll
    for (int q = 0; q < EPT / 2; q += 4) {
      const u4v t = __builtin_nontemporal_load((const u4v *)(p + i0 + 2 * q));
#pragma unroll
      for (int e = 0; e < 4; ++e) w[q + e] = t[e];
    }
  } else if constexpr (EPT % 4 == 0) {
#pragma unroll
    for (int q = 0; q < EPT / 2; q += 2) {
      const u2v t = __builtin_nontemporal_load((const u2v *)(p + i0 + 2 * q));
      w[q] = t[0];
      w[q + 1] = t[1];
    }
  } else {
#pragma unroll
    for (int q = 0; q < EPT / 2; ++q)
      w[q] = __builtin_nontemporal_load((const uint32_t *)(p + i0 + 2 * q));
  }
}
// Ring access for history type HB (BF16 when true, else T).
template <typename T, int EPT, bool HB>
__device__ inline void ring_load(const T *base, size_t off, int i0, int d, bool vec, T (&v)[EPT]) {
  if constexpr (HB)
    hload_nt<EPT>((const uint16_t *)base + off, i0, d, vec, v);
  else
    vload_nt<T, EPT>(base + off, i0, d, vec, v);
}
template <typename T, int EPT, bool HB>
__device__ inline void ring_store(T *base, size_t off, int i0, int d, bool vec, const T (&v)[EPT]) {
  if constexpr (HB)
    hstore_nt<EPT>((uint16_t *)base + off, i0, d, vec, v);
  else
    vstore_nt<T, EPT>(base + off, i0, d, vec, v);
}

// A thread's slices of the kMaxHist register-resident history vectors:
// EPT values of type T each, or (PK: FP32 starts with the history in BF16,
// EPT even) the same values packed two per 32-bit word and widened on each
// read, which halves the registers the history holds.  Values given to set
// must be BF16-exact in the packed form (the low 16 bits are dropped).
template <typename T, int EPT, bool PK>
struct HistReg {
  T v[kMaxHist][EPT];
  __device__ T get(int j, int e) const { return v[j][e]; }
  __device__ void set(int j, const T (&x)[EPT]) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) v[j][e] = x[e];
  }
  __device__ void zero(int j) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) v[j][e] = 0;
  }
  __device__ void move(int j, int k) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) v[j][e] = v[k][e];
  }
};
template <int EPT>
struct HistReg<float, EPT, true> {
  static_assert(EPT % 2 == 0, "two BF16 values per word");
  uint32_t w[kMaxHist][EPT / 2];
  __device__ float get(int j, int e) const {
    const uint32_t x = w[j][e >> 1];
    return __builtin_bit_cast(float, (e & 1) ? (x & 0xffff0000u) : (x << 16));
  }
  __device__ void set(int j, const float (&x)[EPT]) {
#pragma unroll
    for (int q = 0; q < EPT / 2; ++q)
      w[j][q] = (__builtin_bit_cast(uint32_t, x[2 * q]) >> 16) |
                (__builtin_bit_cast(uint32_t, x[2 * q + 1]) & 0xffff0000u);
  }
  __device__ void zero(int j) {
#pragma unroll
    for (int q = 0; q < EPT / 2; ++q) w[j][q] = 0;
  }
  __device__ void move(int j, int k) {
#pragma unroll
    for (int q = 0; q < EPT / 2; ++q) w[j][q] = w[k][q];
  }
};

// Workgroup reductions over a two-slot LDS ring, one barrier each (the
// summation order of block_sum: butterfly within each wave, then the wave
// totals in order, so results are the same).  Reduction k writes slot
// k & 1; a thread reaches the write of reduction k + 2 only after every
// thread has passed the barrier of reduction k + 1, that is, after every
// read of reduction k.  All threads make the same sequence of calls.
template <int TPB, typename T>
struct BlockRed {
  static constexpr int NW = TPB / 64, NMAX = 4;
  T *buf;  // LDS, 2 * NMAX * NW elements
  int slot;
  template <int N, bool MAX>
  __device__ __forceinline__ void reduce(T (&v)[N]) {
    static_assert(N <= NMAX, "values per reduction");
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = MAX ? wave_max(v[j]) : wave_sum(v[j]);
    if constexpr (NW > 1) {
      T *r = buf + slot * (NMAX * NW);
      slot ^= 1;
      const int w = threadIdx.x / 64, l = threadIdx.x % 64;
      if (l == 0)
#pragma unroll
        for (int j = 0; j < N; ++j) r[j * NW + w] = v[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < N; ++j) {
        T t = r[j * NW];
#pragma unroll
        for (int i = 1; i < NW; ++i) t = MAX ? fmax(t, r[j * NW + i]) : t + r[j * NW + i];
        v[j] = t;
      }
    }
  }
  __device__ __forceinline__ T sum(T x) {
    T v[1] = {x};
    reduce<1, false>(v);
    return v[0];
  }
};

// Two-loop recursion on register-resident history (logical order, oldest
// first).  q <- g; backward: alpha_j = rho_j s_j^T q, q -= alpha_j y_j;
// r = gamma q, gamma = s^T y / y^T y of the newest pair; forward:
// beta = rho_j y_j^T r, r += (alpha_j - beta) s_j; returns p = -r.
template <typename T, int TPB, int EPT, class H>
__device__ inline void two_loop(const H &Sr, const H &Yr, const T (&rh)[kMaxHist], T gamma,
                                int cnt, const T (&g)[EPT], T (&p)[EPT], BlockRed<TPB, T> &red) {
  T q[EPT], al[kMaxHist];
#pragma unroll
  for (int e = 0; e < EPT; ++e) q[e] = g[e];
#pragma unroll
  for (int j = kMaxHist - 1; j >= 0; --j) {
    if (j < cnt) {
      T dd = 0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) dd += Sr.get(j, e) * q[e];
      dd = red.sum(dd);
      al[j] = rh[j] * dd;
#pragma unroll
      for (int e = 0; e < EPT; ++e) q[e] -= al[j] * Yr.get(j, e);
    } else {
      al[j] = 0;
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) q[e] *= gamma;
#pragma unroll
  for (int j = 0; j < kMaxHist; ++j) {
    if (j < cnt) {
      T bb = 0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) bb += Yr.get(j, e) * q[e];
      bb = rh[j] * red.sum(bb);
#pragma unroll
      for (int e = 0; e < EPT; ++e) q[e] += (al[j] - bb) * Sr.get(j, e);
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) p[e] = -q[e];
}

// The same recursion with the history left in memory, for memories beyond
// what registers hold (m up to kMaxMem).  Pair j (logical order, oldest
// first) sits at Sb + slot(j) * d and Yb + slot(j) * d with its rho at
// rho[slot(j)], slot(j) = (head - cnt + j) mod m.  The backward loop reads
// the pairs newest first, the forward loop oldest first, so each pair is
// read twice; the oldest pairs are the last read by the first loop and the
// first by the second, and the second read of a pair is its last use
// (non-temporal).  The next pair's chunks are loaded before the current
// pair's reduction so that the load latency overlaps it.  When `reg_new`,
// the newest pair (logical cnt - 1) is taken from sn, yn, rn instead.  The
// arithmetic and its order are those of two_loop.
template <typename T, int TPB, int EPT>
__device__ __forceinline__ void two_loop_stream(const T *Sb, const T *Yb, const T *rho, int d, int m,
                                       int head, int cnt, bool vec, bool reg_new,
                                       const T (&sn)[EPT], const T (&yn)[EPT], T rn, T gamma,
                                       const T (&g)[EPT], T (&p)[EPT], BlockRed<TPB, T> &red) {
  const int i0 = threadIdx.x * EPT;
  T q[EPT], al[kMaxMem];
#pragma unroll
  for (int e = 0; e < EPT; ++e) q[e] = g[e];
  auto slot = [&](int j) { return (head - cnt + j + 2 * m) % m; };
  auto fetch = [&](int j, T (&sv)[EPT], T (&yv)[EPT], T &rv, bool last) {
    if (reg_new && j == cnt - 1) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        sv[e] = sn[e];
        yv[e] = yn[e];
      }
      rv = rn;
      return;
    }
    const int ph = slot(j);
    if (last) {
      vload_nt<T, EPT>(Sb + (size_t)ph * d, i0, d, vec, sv);
      vload_nt<T, EPT>(Yb + (size_t)ph * d, i0, d, vec, yv);
    } else {
      vload<T, EPT>(Sb + (size_t)ph * d, i0, d, vec, sv);
      vload<T, EPT>(Yb + (size_t)ph * d, i0, d, vec, yv);
    }
    rv = rho[ph];
  };
  T cs[EPT], cy[EPT], cr = 0;
  if (cnt > 0) fetch(cnt - 1, cs, cy, cr, false);
#pragma unroll
  for (int j = kMaxMem - 1; j >= 0; --j) {
    if (j < cnt) {
      T ns[EPT], ny[EPT], nr = 0;
      if (j > 0) fetch(j - 1, ns, ny, nr, false);
      T dd = 0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) dd += cs[e] * q[e];
      dd = red.sum(dd);
      al[j] = cr * dd;
#pragma unroll
      for (int e = 0; e < EPT; ++e) q[e] -= al[j] * cy[e];
      if (j > 0) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          cs[e] = ns[e];
          cy[e] = ny[e];
        }
        cr = nr;
      }
    } else {
      al[j] = 0;
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) q[e] *= gamma;
  if (cnt > 0) fetch(0, cs, cy, cr, true);
#pragma unroll
  for (int j = 0; j < kMaxMem; ++j) {
    if (j < cnt) {
      T ns[EPT], ny[EPT], nr = 0;
      if (j + 1 < cnt) fetch(j + 1, ns, ny, nr, true);
      T bb = 0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) bb += cy[e] * q[e];
      bb = cr * red.sum(bb);
#pragma unroll
      for (int e = 0; e < EPT; ++e) q[e] += (al[j] - bb) * cs[e];
      if (j + 1 < cnt) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          cs[e] = ns[e];
          cy[e] = ny[e];
        }
        cr = nr;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) p[e] = -q[e];
}

// One step of start s (the whole workgroup; every branch is uniform in s).
// HREG: the history is held in registers (m <= kMaxHist); otherwise it stays
// in memory and two_loop_stream reads it (m <= kMaxMem).  HB (FP32, HREG):
// the ring holds BF16 pairs (s and y rounded to BF16 when formed).
template <typename T, int TPB, int EPT, bool HREG, bool HB = false>
__device__ __forceinline__ void lbfgs_step_one(const LbArgs<T> &a, const int64_t s,
                                               BlockRed<TPB, T> &red) {
  static_assert(!HB || (HREG && sizeof(T) == 4), "BF16 history: FP32, register-resident");
  const int tid = threadIdx.x;
  const int64_t B = a.B;
  // every per-start scalar is read before the first decision, so the reads
  // share one memory round trip (all are in bounds for any start)
  const int status = a.status[s];
  int cur = a.cur[s];
  const int phase = a.phase[s];
  int cnt = a.cnt[s], head = a.head[s], it = a.iters[s];
  const double f0 = a.F[s], f1 = a.F[(size_t)B + s];
  const T alpha_s = a.alpha[s], gtp_s = a.gtp[s];
  const int ls_s = a.ls[s];
  const int dv = a.vdim ? a.vdim[s] : a.d;
  const int64_t vov = a.voff ? a.voff[s] : (int64_t)s * a.d;
  if (status != ST_ACTIVE) {
    if (tid == 0) a.active[s] = 0;
    return;
  }
  const int m = a.m;
  const int d = dv;
  const int64_t vo = vov;
  const int64_t Lt = a.Ltot;
  const int i0 = tid * EPT;  // this thread's chunk of every vector
  const bool vec = (d % EPT == 0) && (vo % EPT == 0) && (Lt % EPT == 0);
  T tol = a.tol;
  int max_iter = a.max_iter;
  if (a.sprob) {
    const int p = a.sprob[s];
    tol = (T)a.ptol[p];
    max_iter = a.pmaxit[p];
  }
  const double lcur = cur ? f1 : f0;

  // ---- decide what this step does from the scalars alone
  enum { M_INIT, M_ACCEPT, M_BACKTRACK, M_RESET, M_STALL };
  int mode = M_INIT;
  T alpha = 1;
  int lsn = 0;
  if (phase == PH_TRIAL) {
    const double lt = cur ? f0 : f1;
    alpha = alpha_s;
    const double gtp_old = (double)gtp_s;
    const double fc = -lcur, ft = -lt;
    if (isfinite(ft) && ft <= fc + 1e-4 * (double)alpha * gtp_old) {
      mode = M_ACCEPT;
    } else {
      lsn = ls_s + 1;
      alpha *= (T)0.5;
      if (lsn <= 40)
        mode = M_BACKTRACK;
      else
        mode = (cnt > 0) ? M_RESET : M_STALL;
    }
  }
  if (mode == M_STALL) {
    if (tid == 0) {
      a.status[s] = ST_STALLED;
      a.active[s] = 0;
    }
    return;
  }
  if (mode == M_BACKTRACK) {
    const int tr = 1 - cur;
    const T *xc = a.X + (size_t)cur * Lt + vo;
    T *xt = a.X + (size_t)tr * Lt + vo;
    const T *pd = a.Pd + vo;
    T c[EPT], q[EPT];
    vload<T, EPT>(xc, i0, d, vec, c);
    vload<T, EPT>(pd, i0, d, vec, q);
#pragma unroll
    for (int e = 0; e < EPT; ++e) c[e] = c[e] + alpha * q[e];
    vstore<T, EPT>(xt, i0, d, vec, c);
    if (tid == 0) {
      a.alpha[s] = alpha;
      a.ls[s] = lsn;
      a.active[s] = 1;
      a.rowid[s] = (int32_t)((size_t)tr * B + s);
      if (a.rowoff) a.rowoff[s] = (int64_t)tr * Lt + vo;
    }
    return;
  }

  // ---- load the point whose direction we now compute (and, on accept, the old one)
  T x[EPT], gl[EPT], sv[EPT], yv[EPT];
  const int newcur = (mode == M_ACCEPT) ? 1 - cur : cur;
  {
    const T *xn = a.X + (size_t)newcur * Lt + vo;
    const T *gn = a.G + (size_t)newcur * Lt + vo;
    const T *xo = a.X + (size_t)cur * Lt + vo;
    const T *go = a.G + (size_t)cur * Lt + vo;
    vload<T, EPT>(xn, i0, d, vec, x);
    vload<T, EPT>(gn, i0, d, vec, gl);
    if (mode == M_ACCEPT) {
      T xov[EPT], gov[EPT];
      vload<T, EPT>(xo, i0, d, vec, xov);
      vload<T, EPT>(go, i0, d, vec, gov);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        sv[e] = x[e] - xov[e];
        yv[e] = gov[e] - gl[e];  // grad f(x_t) - grad f(x), grad f = -grad l
        if constexpr (HB) {
          sv[e] = bf16_round(sv[e]);
          yv[e] = bf16_round(yv[e]);
        }
      }
    }
  }
  if (mode == M_RESET) {
    cnt = 0;
    head = 0;
  }
  // history in logical order (loads issued before the reductions below).
  // With the ring full, the oldest pair is evicted when the curvature test
  // passes, so its load waits for that test and happens only when it fails.
  constexpr int MH = HREG ? kMaxHist : 1;
  constexpr bool PK = HB && EPT % 2 == 0;
  HistReg<T, EPT, PK> Sr, Yr;
  T rh[MH], yyr[MH];
  const bool defer_oldest = (mode == M_ACCEPT && cnt == m);
  if constexpr (HREG) {
    // packed BF16 history in whole aligned chunks: the raw words go straight
    // to registers, every load issued before the first use
    const bool raw = PK && vec && i0 + EPT <= d;
#pragma unroll
    for (int j = 0; j < kMaxHist; ++j) {
      rh[j] = 0;
      yyr[j] = 0;
      Sr.zero(j);
      Yr.zero(j);
      if (mode == M_ACCEPT && j < cnt && !(j == 0 && defer_oldest)) {
        const int ph = (head - cnt + j + 2 * m) % m;
        const size_t off = (size_t)m * vo + (size_t)ph * d;
        if constexpr (PK) {
          if (raw) {
            hload_raw_nt<EPT>((const uint16_t *)a.S + off, i0, Sr.w[j]);
            hload_raw_nt<EPT>((const uint16_t *)a.Yh + off, i0, Yr.w[j]);
          } else {
            T t[EPT];
            ring_load<T, EPT, HB>(a.S, off, i0, d, vec, t);
            Sr.set(j, t);
            ring_load<T, EPT, HB>(a.Yh, off, i0, d, vec, t);
            Yr.set(j, t);
          }
        } else {
          ring_load<T, EPT, HB>(a.S, off, i0, d, vec, Sr.v[j]);
          ring_load<T, EPT, HB>(a.Yh, off, i0, d, vec, Yr.v[j]);
        }
        rh[j] = a.rho[(size_t)s * m + ph];
        yyr[j] = a.yy[(size_t)s * m + ph];
      }
    }
  }
  // streamed history: the pair pushed in this step stays in registers
  bool reg_new = false;
  T r_new = 0, yy_new = 1;
  if (mode == M_ACCEPT) {
    T v3[3] = {0, 0, 0};
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      v3[0] += sv[e] * yv[e];
      v3[1] += sv[e] * sv[e];
      v3[2] += yv[e] * yv[e];
    }
    red.template reduce<3, false>(v3);
    const T sy = v3[0], ss = v3[1], yy = v3[2];
    cur = newcur;
    ++it;
    if (sy > (T)1e-10 * sqrt(ss) * sqrt(yy)) {
      // store the pair in the ring and append it to the logical history
      ring_store<T, EPT, HB>(a.S, (size_t)m * vo + (size_t)head * d, i0, d, vec, sv);
      ring_store<T, EPT, HB>(a.Yh, (size_t)m * vo + (size_t)head * d, i0, d, vec, yv);
      if (tid == 0) {
        a.rho[(size_t)s * m + head] = (T)1 / sy;
        a.yy[(size_t)s * m + head] = yy;
      }
      const bool full = (cnt == m);
      if constexpr (HREG) {
        if (full) {
#pragma unroll
          for (int j = 0; j < kMaxHist - 1; ++j) {
            Sr.move(j, j + 1);
            Yr.move(j, j + 1);
            rh[j] = rh[j + 1];
            yyr[j] = yyr[j + 1];
          }
        }
        const int pos = full ? m - 1 : cnt;
#pragma unroll
        for (int j = 0; j < kMaxHist; ++j) {
          if (j == pos) {
            Sr.set(j, sv);
            Yr.set(j, yv);
            rh[j] = (T)1 / sy;
            yyr[j] = yy;
          }
        }
      } else {
        reg_new = true;
        r_new = (T)1 / sy;
        yy_new = yy;
      }
      head = (head + 1) % m;
      cnt = full ? m : cnt + 1;
    } else if (defer_oldest) {
      if constexpr (HREG) {
        // pair kept out: the oldest pair (ring slot head) stays in the history
        T t[EPT];
        ring_load<T, EPT, HB>(a.S, (size_t)m * vo + (size_t)head * d, i0, d, vec, t);
        Sr.set(0, t);
        ring_load<T, EPT, HB>(a.Yh, (size_t)m * vo + (size_t)head * d, i0, d, vec, t);
        Yr.set(0, t);
        rh[0] = a.rho[(size_t)s * m + head];
        yyr[0] = a.yy[(size_t)s * m + head];
      }
    }
  }

  // ---- convergence tests at the current point
  // ||grad l||_inf; a non-finite entry makes it NaN (no convergence on NaN)
  T gn = 0, bad = 0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    gn = fmax(gn, fabs(gl[e]));
    if (!isfinite(gl[e])) bad = 1;
  }
  {
    T v2[2] = {gn, bad};
    red.template reduce<2, true>(v2);
    gn = v2[0];
    if (v2[1] != (T)0) gn = (T)NAN;
  }
  int newst = ST_ACTIVE;
  if (mode == M_INIT && !(isfinite(lcur) && isfinite(gn)))
    newst = ST_DEAD;
  else if (gn <= tol)
    newst = ST_CONVERGED;
  else if (it >= max_iter)
    newst = ST_MAXITER;
  if (newst != ST_ACTIVE) {
    if (tid == 0) {
      a.status[s] = newst;
      a.active[s] = 0;
      a.cur[s] = cur;
      a.cnt[s] = cnt;
      a.head[s] = head;
      a.iters[s] = it;
    }
    return;
  }

  // ---- next direction
  T g[EPT], p[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) g[e] = -gl[e];
  T gtp = 0;
  bool sd = (cnt == 0);
  if (!sd) {
    // gamma = s^T y / y^T y of the newest pair (logical index cnt - 1)
    T rnew = 0, yynew = 1;
    if constexpr (HREG) {
#pragma unroll
      for (int j = 0; j < kMaxHist; ++j)
        if (j == cnt - 1) {
          rnew = rh[j];
          yynew = yyr[j];
        }
    } else {
      if (reg_new) {
        rnew = r_new;
        yynew = yy_new;
      } else {
        const int ph = (head - 1 + m) % m;
        rnew = a.rho[(size_t)s * m + ph];
        yynew = a.yy[(size_t)s * m + ph];
      }
    }
    const T gamma = ((T)1 / rnew) / yynew;
    if constexpr (HREG)
      two_loop<T, TPB, EPT>(Sr, Yr, rh, gamma, cnt, g, p, red);
    else
      two_loop_stream<T, TPB, EPT>(a.S + (size_t)m * vo, a.Yh + (size_t)m * vo,
                                   a.rho + (size_t)s * m, d, m, head, cnt, vec, reg_new, sv, yv,
                                   r_new, gamma, g, p, red);
    T t = 0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) t += g[e] * p[e];
    gtp = red.sum(t);
    if (!(gtp < (T)0)) {
      sd = true;
      cnt = 0;
      head = 0;
    }
  }
  if (sd) {
    const T sc = (T)1 / (gn > (T)1 ? gn : (T)1);
    T t = 0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      p[e] = -g[e] * sc;
      t += g[e] * p[e];
    }
    gtp = red.sum(t);
  }
  const int tr = 1 - cur;
  T *xt = a.X + (size_t)tr * Lt + vo;
  T *pd = a.Pd + vo;
  T xtv[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) xtv[e] = x[e] + p[e];
  vstore_nt<T, EPT>(pd, i0, d, vec, p);
  vstore<T, EPT>(xt, i0, d, vec, xtv);
  if (tid == 0) {
    a.alpha[s] = (T)1;
    a.gtp[s] = gtp;
    a.ls[s] = 0;
    a.cur[s] = cur;
    a.cnt[s] = cnt;
    a.head[s] = head;
    a.iters[s] = it;
    a.phase[s] = PH_TRIAL;
    a.active[s] = 1;
    a.rowid[s] = (int32_t)((size_t)tr * B + s);
    if (a.rowoff) a.rowoff[s] = (int64_t)tr * Lt + vo;
  }
}

// Start s_base + blockIdx.x (one workgroup per start of the launch's range).
template <typename T, int TPB, int EPT, bool HREG, bool HB = false>
__global__ __launch_bounds__(TPB) void lbfgs_step_kernel(LbArgs<T> a) {
  __shared__ T rbuf[2 * BlockRed<TPB, T>::NMAX * (TPB / 64)];
  BlockRed<TPB, T> red{rbuf, 0};
  // the compaction that follows counts from zero; every reader of the
  // previous count ran before this launch
  if (a.count_reset && blockIdx.x == 0 && threadIdx.x == 0) *a.count_reset = 0;
  if ((int64_t)blockIdx.x < a.s_count)
    lbfgs_step_one<T, TPB, EPT, HREG, HB>(a, a.s_base + blockIdx.x, red);
}

// Two-loop direction only, for B independent histories given in logical
// order (used to check the recursion in isolation).
template <typename T, int TPB, int EPT, bool HREG>
__global__ __launch_bounds__(TPB) void two_loop_kernel(int d, int m, const int32_t *cntv,
                                                       const T *S, const T *Y, const T *G, T *P) {
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ T rbuf[2 * BlockRed<TPB, T>::NMAX * (TPB / 64)];
  BlockRed<TPB, T> red{rbuf, 0};
  const int cnt = min(max(cntv[b], 0), m);  // never read past this start's m slots
  if constexpr (!HREG) {
    // rho_j and gamma from one pass over the pairs, then the streamed
    // recursion (logical order is the slot order: head = cnt mod m)
    __shared__ T rho_s[kMaxMem];
    const int i0 = tid * EPT;
    const bool vec = (d % EPT == 0);
    T g[EPT], p[EPT], z[EPT], gamma = 1;
#pragma unroll
    for (int e = 0; e < EPT; ++e) z[e] = 0;
    vload<T, EPT>(G + (size_t)b * d, i0, d, vec, g);
    for (int j = 0; j < cnt; ++j) {
      T sv[EPT], yv[EPT];
      vload<T, EPT>(S + ((size_t)b * m + j) * d, i0, d, vec, sv);
      vload<T, EPT>(Y + ((size_t)b * m + j) * d, i0, d, vec, yv);
      T v2[2] = {0, 0};
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        v2[0] += sv[e] * yv[e];
        v2[1] += yv[e] * yv[e];
      }
      red.template reduce<2, false>(v2);
      if (tid == 0) rho_s[j] = (T)1 / v2[0];
      if (j == cnt - 1) gamma = v2[0] / v2[1];
    }
    __syncthreads();
    two_loop_stream<T, TPB, EPT>(S + (size_t)b * m * d, Y + (size_t)b * m * d, rho_s, d, m,
                                 cnt % m, cnt, vec, false, z, z, (T)0, gamma, g, p, red);
    vstore<T, EPT>(P + (size_t)b * d, i0, d, vec, p);
    return;
  }
  HistReg<T, EPT, false> Sr, Yr;
  T rh[kMaxHist], g[EPT], p[EPT];
  T gamma = 1;
  const int i0 = tid * EPT;
  const bool vec = (d % EPT == 0);
  vload<T, EPT>(G + (size_t)b * d, i0, d, vec, g);
#pragma unroll
  for (int j = 0; j < kMaxHist; ++j) {
    rh[j] = 0;
    if (j < cnt) {
      vload<T, EPT>(S + ((size_t)b * m + j) * d, i0, d, vec, Sr.v[j]);
      vload<T, EPT>(Y + ((size_t)b * m + j) * d, i0, d, vec, Yr.v[j]);
    } else {
      Sr.zero(j);
      Yr.zero(j);
    }
    if (j < cnt) {
      T v2[2] = {0, 0};
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        v2[0] += Sr.v[j][e] * Yr.v[j][e];
        v2[1] += Yr.v[j][e] * Yr.v[j][e];
      }
      red.template reduce<2, false>(v2);
      rh[j] = (T)1 / v2[0];
      if (j == cnt - 1) gamma = v2[0] / v2[1];
    }
  }
  two_loop<T, TPB, EPT>(Sr, Yr, rh, gamma, cnt, g, p, red);
  vstore<T, EPT>(P + (size_t)b * d, i0, d, vec, p);
}

// ------------------------------------------------------------- dispatch

// Workgroup size and elements per thread by d; HR: history in registers.
#define SB_LB_CASES_H(KERNEL, T, HR, ...)                                                     \
  if (d <= 64) {                                                                              \
    hipLaunchKernelGGL((KERNEL<T, 64, 1, HR>), dim3((unsigned)B), dim3(64), 0, s, __VA_ARGS__);   \
  } else if (d <= 128) {                                                                      \
    hipLaunchKernelGGL((KERNEL<T, 64, 2, HR>), dim3((unsigned)B), dim3(64), 0, s, __VA_ARGS__);   \
  } else if (d <= 256) {                                                                      \
    hipLaunchKernelGGL((KERNEL<T, 64, 4, HR>), dim3((unsigned)B), dim3(64), 0, s, __VA_ARGS__);   \
  } else if (d <= 512) {                                                                      \
    hipLaunchKernelGGL((KERNEL<T, 128, 4, HR>), dim3((unsigned)B), dim3(128), 0, s, __VA_ARGS__); \
  } else if (d <= 1024) {                                                                     \
    hipLaunchKernelGGL((KERNEL<T, 256, 4, HR>), dim3((unsigned)B), dim3(256), 0, s, __VA_ARGS__); \
  } else if (d <= 2048) {                                                                     \
    hipLaunchKernelGGL((KERNEL<T, 512, 4, HR>), dim3((unsigned)B), dim3(512), 0, s, __VA_ARGS__); \
  } else {                                                                                    \
    hipLaunchKernelGGL((KERNEL<T, 1024, 4, HR>), dim3((unsigned)B), dim3(1024), 0, s,          \
                       __VA_ARGS__);                                                          \
  }
// Register-resident history for m <= kMaxHist, streamed beyond.
#define SB_LB_CASES(KERNEL, T, M, ...)              \
  if ((M) <= kMaxHist) {                            \
    SB_LB_CASES_H(KERNEL, T, true, __VA_ARGS__)     \
  } else {                                          \
    SB_LB_CASES_H(KERNEL, T, false, __VA_ARGS__)    \
  }
// FP32 starts with the BF16 history ring (register-resident, m <= kMaxHist).
#define SB_LB_CASES_HB(KERNEL, ...)                                                            \
  if (d <= 64) {                                                                               \
    hipLaunchKernelGGL((KERNEL<float, 64, 1, true, true>), dim3((unsigned)B), dim3(64), 0, s,   \
                       __VA_ARGS__);                                                           \
  } else if (d <= 128) {                                                                       \
    hipLaunchKernelGGL((KERNEL<float, 64, 2, true, true>), dim3((unsigned)B), dim3(64), 0, s,   \
                       __VA_ARGS__);                                                           \
  } else if (d <= 256) {                                                                       \
    hipLaunchKernelGGL((KERNEL<float, 64, 4, true, true>), dim3((unsigned)B), dim3(64), 0, s,   \
                       __VA_ARGS__);                                                           \
  } else if (d <= 512) {                                                                       \
    hipLaunchKernelGGL((KERNEL<float, 64, 8, true, true>), dim3((unsigned)B), dim3(64), 0, s,   \
                       __VA_ARGS__);                                                           \
  } else if (d <= 1024) {                                                                      \
    hipLaunchKernelGGL((KERNEL<float, 128, 8, true, true>), dim3((unsigned)B), dim3(128), 0, s, \
                       __VA_ARGS__);                                                           \
  } else if (d <= 2048) {                                                                      \
    hipLaunchKernelGGL((KERNEL<float, 256, 8, true, true>), dim3((unsigned)B), dim3(256), 0, s, \
                       __VA_ARGS__);                                                           \
  } else {                                                                                     \
    hipLaunchKernelGGL((KERNEL<float, 512, 8, true, true>), dim3((unsigned)B), dim3(512), 0,    \
                       s, __VA_ARGS__);                                                        \
  }

static int check_d(int d, int m) {
  if (d < 1 || d > 4096) {
    set_error("L-BFGS supports 1 <= d <= 4096 (got %d)", d);
    return SB_E_UNSUPPORTED;
  }
  if (m < 1 || m > kMaxMem) {
    set_error("L-BFGS memory m must be in [1, %d] (got %d)", kMaxMem, m);
    return SB_E_INVAL;
  }
  return SB_OK;
}
static int check_hist(const LbfgsBuffers &b) {
  if (b.hist_bf16 && (b.dtype != DT_F32 || b.m > kMaxHist)) {
    set_error("BF16 history needs FP32 starts and m <= %d (got m = %d)", kMaxHist, b.m);
    return SB_E_UNSUPPORTED;
  }
  return SB_OK;
}

template <typename T>
static LbArgs<T> make_args(const LbfgsBuffers &b, int max_iter, double tol) {
  LbArgs<T> a;
  a.B = b.B;
  a.d = b.d;
  a.m = b.m;
  a.max_iter = max_iter;
  a.tol = (T)tol;
  a.X = (T *)b.X;
  a.G = (T *)b.G;
  a.F = (double *)b.F;
  a.Pd = (T *)b.Pd;
  a.S = (T *)b.S;
  a.Yh = (T *)b.Yh;
  a.rho = (T *)b.rho;
  a.yy = (T *)b.yy;
  a.alpha = (T *)b.alpha;
  a.gtp = (T *)b.gtp;
  a.cur = b.cur;
  a.head = b.head;
  a.cnt = b.cnt;
  a.iters = b.iters;
  a.ls = b.ls;
  a.status = b.status;
  a.phase = b.phase;
  a.rowid = b.rowid;
  a.active = b.active;
  a.voff = b.voff;
  a.vdim = b.vdim;
  a.rowoff = b.rowoff;
  a.Ltot = b.voff ? b.Ltot : b.B * (int64_t)b.d;
  a.sprob = b.sprob;
  a.ptol = b.ptol;
  a.pmaxit = b.pmaxit;
  a.s_base = 0;
  a.s_count = b.B;
  a.count_reset = nullptr;
  return a;
}

// One workgroup per start of the launch: the dispatcher hands freed slots
// to the next start, which balances starts of uneven cost (a fixed grid
// striding over starts measured slower: its last round runs part-empty).
static int64_t step_grid(int64_t count) { return count; }

int launch_lbfgs_step(const LbfgsBuffers &b, int max_iter, double grad_tol, hipStream_t s) {
  int st = check_d(b.d, b.m);
  if (!st) st = check_hist(b);
  if (st) return st;
  const int d = b.d;
  const int64_t B = step_grid(b.B);
  if (B <= 0) return SB_OK;
  if (b.dtype == DT_F64) {
    LbArgs<double> a = make_args<double>(b, max_iter, grad_tol);
    a.count_reset = b.count;
    SB_LB_CASES(lbfgs_step_kernel, double, b.m, a);
  } else if (b.hist_bf16) {
    LbArgs<float> a = make_args<float>(b, max_iter, grad_tol);
    a.count_reset = b.count;
    SB_LB_CASES_HB(lbfgs_step_kernel, a);
  } else {
    LbArgs<float> a = make_args<float>(b, max_iter, grad_tol);
    a.count_reset = b.count;
    SB_LB_CASES(lbfgs_step_kernel, float, b.m, a);
  }
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int launch_lbfgs_step_range(const LbfgsBuffers &b, int64_t s_begin, int64_t count, int d_class,
                            double grad_tol, int max_iter, hipStream_t s) {
  int st = check_d(d_class, b.m);
  if (!st) st = check_hist(b);
  if (st) return st;
  if (count <= 0) return SB_OK;
  if (s_begin < 0 || s_begin + count > b.B) {
    set_error("start range [%lld, %lld) outside [0, %lld)", (long long)s_begin,
              (long long)(s_begin + count), (long long)b.B);
    return SB_E_INVAL;
  }
  const int d = d_class;
  const int64_t B = step_grid(count);
  if (b.dtype == DT_F64) {
    LbArgs<double> a = make_args<double>(b, max_iter, grad_tol);
    a.s_base = s_begin;
    a.s_count = count;
    SB_LB_CASES(lbfgs_step_kernel, double, b.m, a);
  } else if (b.hist_bf16) {
    LbArgs<float> a = make_args<float>(b, max_iter, grad_tol);
    a.s_base = s_begin;
    a.s_count = count;
    SB_LB_CASES_HB(lbfgs_step_kernel, a);
  } else {
    LbArgs<float> a = make_args<float>(b, max_iter, grad_tol);
    a.s_base = s_begin;
    a.s_count = count;
    SB_LB_CASES(lbfgs_step_kernel, float, b.m, a);
  }
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int launch_two_loop(int64_t B, int d, int m, const int32_t *cnt, const void *S, const void *Y,
                    const void *G, void *P, int dtype, hipStream_t s) {
  int st = check_d(d, m);
  if (st) return st;
  if (B <= 0) return SB_OK;
  if (dtype == DT_F64) {
    SB_LB_CASES(two_loop_kernel, double, m, d, m, cnt, (const double *)S, (const double *)Y,
                (const double *)G, (double *)P);
  } else {
    SB_LB_CASES(two_loop_kernel, float, m, d, m, cnt, (const float *)S, (const float *)Y,
                (const float *)G, (float *)P);
  }
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// ------------------------------------------------------------- state

size_t lbfgs_state_bytes(int dtype, int64_t B, int d, int m) {
  LbfgsBuffers b;
  b.dtype = dtype;
  b.B = B;
  b.d = d;
  b.m = m;
  Arena ar(nullptr, 0);
  lbfgs_carve(ar, b);
  return ar.off;
}

int lbfgs_carve(Arena &ar, LbfgsBuffers &b) {
  const size_t es = (b.dtype == DT_F64) ? 8 : 4;
  const int64_t B = b.B, d = b.d, m = b.m;
  auto take = [&](size_t n) -> void * { return (void *)ar.take<char>(n * es); };
  b.X = take(2 * B * d);
  b.G = take(2 * B * d);
  b.F = (void *)ar.take<double>(2 * B);
  b.Pd = take(B * d);
  b.S = take(B * m * d);
  b.Yh = take(B * m * d);
  b.rho = take(B * m);
  b.yy = take(B * m);
  b.alpha = take(B);
  b.gtp = take(B);
  b.cur = ar.take<int32_t>(B);
  b.head = ar.take<int32_t>(B);
  b.cnt = ar.take<int32_t>(B);
  b.iters = ar.take<int32_t>(B);
  b.ls = ar.take<int32_t>(B);
  b.status = ar.take<int32_t>(B);
  b.phase = ar.take<int32_t>(B);
  b.rowid = ar.take<int32_t>(B);
  b.active = ar.take<int32_t>(B);
  b.idx = ar.take<int32_t>(B);
  b.count = ar.take<int32_t>(4);
  b.evals = ar.take<int64_t>(2);
  return ar.ok() ? SB_OK : SB_E_NOMEM;
}

template <typename T>
__global__ void lbfgs_init_kernel(int64_t B, int d, const T *X0, T *X, int32_t *cur,
                                  int32_t *head, int32_t *cnt, int32_t *iters, int32_t *ls,
                                  int32_t *status, int32_t *phase, int32_t *count,
                                  int64_t *evals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = B * d;
  for (int64_t e = i; e < n; e += (int64_t)gridDim.x * blockDim.x) X[e] = X0[e];
  for (int64_t e = i; e < B; e += (int64_t)gridDim.x * blockDim.x) {
    cur[e] = 0;
    head[e] = 0;
    cnt[e] = 0;
    iters[e] = 0;
    ls[e] = 0;
    status[e] = ST_ACTIVE;
    phase[e] = PH_INIT;
  }
  if (i == 0) {
    count[0] = (int32_t)B;
    evals[0] = B;
  }
}

int launch_lbfgs_init(const LbfgsBuffers &b, const void *X0, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<int64_t>(8192, ceil_div(b.B * b.d, 256));
  if (b.dtype == DT_F64)
    hipLaunchKernelGGL(lbfgs_init_kernel<double>, dim3(blocks), dim3(256), 0, s, b.B, b.d,
                       (const double *)X0, (double *)b.X, b.cur, b.head, b.cnt, b.iters, b.ls,
                       b.status, b.phase, b.count, b.evals);
  else
    hipLaunchKernelGGL(lbfgs_init_kernel<float>, dim3(blocks), dim3(256), 0, s, b.B, b.d,
                       (const float *)X0, (float *)b.X, b.cur, b.head, b.cnt, b.iters, b.ls,
                       b.status, b.phase, b.count, b.evals);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// Compaction of the active starts into idx (their trial row ids), in start
// order; count[0] = number active, evals[0] += count.  One workgroup: each
// thread owns a contiguous chunk, exclusive scan of the chunk counts in LDS.
// Active starts' trial rows into idx[0, count).  Each wave ballots its
// starts and reserves its slice with one atomic: the order of the list
// depends on wave timing, the rows' results do not (every row of the
// contraction and of the epilogue is computed on its own).
__global__ __launch_bounds__(256) void compact_kernel(int64_t B, const int32_t *active,
                                                      const int32_t *rowid, int32_t *idx,
                                                      int32_t *count, int64_t *evals) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool on = s < B && active[s] != 0;
  const unsigned long long mask = __ballot(on);
  const int lane = threadIdx.x & 63;
  const int n = __popcll(mask);
  int base = 0;
  if (lane == 0 && n > 0) {
    base = atomicAdd(count, n);
    atomicAdd((unsigned long long *)evals, (unsigned long long)n);
  }
  base = __shfl(base, 0, 64);
  if (on) idx[base + __popcll(mask & ((1ull << lane) - 1ull))] = rowid[s];
}

// The step launch that precedes each compaction zeroes count.
int launch_compact(const LbfgsBuffers &b, hipStream_t s) {
  if (b.B > 0)
    hipLaunchKernelGGL(compact_kernel, dim3((unsigned)ceil_div(b.B, 256)), dim3(256), 0, s, b.B,
                       b.active, b.rowid, b.idx, b.count, b.evals);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

template <typename T>
__global__ void lbfgs_gather_kernel(int64_t B, int d, const T *X, const T *G, const double *F,
                                    const int32_t *cur, const int32_t *st, const int32_t *its,
                                    T *Xo, void *lo, bool lo_f64, T *go, int32_t *sto,
                                    int32_t *ito) {
  const int64_t s = blockIdx.x;
  const int c = cur[s];
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    if (Xo) Xo[(size_t)s * d + i] = X[((size_t)c * B + s) * d + i];
    if (go) go[(size_t)s * d + i] = G[((size_t)c * B + s) * d + i];
  }
  if (threadIdx.x == 0) {
    if (lo) {
      if (lo_f64)
        ((double *)lo)[s] = F[(size_t)c * B + s];
      else
        ((T *)lo)[s] = (T)F[(size_t)c * B + s];
    }
    if (sto) sto[s] = st[s];
    if (ito) ito[s] = its[s];
  }
}

int launch_lbfgs_gather(const LbfgsBuffers &b, void *X, void *logl, bool logl_f64, void *grad,
                        int32_t *status, int32_t *iters, hipStream_t s) {
  if (b.B <= 0) return SB_OK;
  if (b.dtype == DT_F64)
    hipLaunchKernelGGL(lbfgs_gather_kernel<double>, dim3((unsigned)b.B), dim3(256), 0, s, b.B,
                       b.d, (const double *)b.X, (const double *)b.G, (const double *)b.F, b.cur,
                       b.status, b.iters, (double *)X, logl, logl_f64, (double *)grad, status,
                       iters);
  else
    hipLaunchKernelGGL(lbfgs_gather_kernel<float>, dim3((unsigned)b.B), dim3(256), 0, s, b.B, b.d,
                       (const float *)b.X, (const float *)b.G, (const double *)b.F, b.cur,
                       b.status, b.iters, (float *)X, logl, logl_f64, (float *)grad, status,
                       iters);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb

// ====================================================================
// Batches: per-problem compaction, layout-preserving init and gather.
namespace sb {

// One workgroup per problem: active starts of [s0, s0 + B) in start order.
__global__ __launch_bounds__(1024) void compact_group_kernel(const BatchProb *probs,
                                                             const int32_t *active,
                                                             const int32_t *rowid,
                                                             const int64_t *rowoff, int32_t *idx,
                                                             int64_t *croff, int32_t *counts,
                                                             int64_t *evals) {
  __shared__ int32_t sc[1024];
  const BatchProb pr = probs[blockIdx.x];
  const int t = threadIdx.x;
  const int64_t B = pr.B, s0 = pr.s0;
  const int64_t per = (B + 1023) / 1024;
  const int64_t b0 = s0 + (int64_t)t * per, b1 = std::min<int64_t>(s0 + B, b0 + per);
  int32_t c = 0;
  for (int64_t i = b0; i < b1; ++i) c += active[i] ? 1 : 0;
  sc[t] = c;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int32_t v = (t >= o) ? sc[t - o] : 0;
    __syncthreads();
    sc[t] += v;
    __syncthreads();
  }
  int64_t pos = s0 + sc[t] - c;
  for (int64_t i = b0; i < b1; ++i)
    if (active[i]) {
      idx[pos] = rowid[i];
      croff[pos] = rowoff[i];
      ++pos;
    }
  if (t == 1023) {
    counts[blockIdx.x] = sc[1023];
    evals[blockIdx.x] += sc[1023];  // one workgroup per problem: no race
  }
}

int launch_compact_group(const BatchDev &b, const LbfgsBuffers &lb, int32_t *counts,
                         hipStream_t s) {
  hipLaunchKernelGGL(compact_group_kernel, dim3(b.n), dim3(1024), 0, s, b.probs, lb.active,
                     lb.rowid, lb.rowoff, lb.idx, lb.croff, counts, lb.pevals);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

template <typename T>
__global__ void lbfgs_init_group_kernel(int64_t B, int64_t L, const T *X0, T *X, int32_t *cur,
                                        int32_t *head, int32_t *cnt, int32_t *iters, int32_t *ls,
                                        int32_t *status, int32_t *phase, int64_t *evals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = i; e < L; e += stride) X[e] = X0[e];
  for (int64_t e = i; e < B; e += stride) {
    cur[e] = 0;
    head[e] = 0;
    cnt[e] = 0;
    iters[e] = 0;
    ls[e] = 0;
    status[e] = ST_ACTIVE;
    phase[e] = PH_INIT;
  }
  if (i == 0 && evals) evals[0] = B;
}

int launch_lbfgs_init_group(const LbfgsBuffers &b, const void *X0, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<int64_t>(8192, ceil_div(std::max(b.Ltot, b.B), 256));
  if (b.dtype == DT_F64)
    hipLaunchKernelGGL(lbfgs_init_group_kernel<double>, dim3(blocks), dim3(256), 0, s, b.B,
                       b.Ltot, (const double *)X0, (double *)b.X, b.cur, b.head, b.cnt, b.iters,
                       b.ls, b.status, b.phase, b.evals);
  else
    hipLaunchKernelGGL(lbfgs_init_group_kernel<float>, dim3(blocks), dim3(256), 0, s, b.B,
                       b.Ltot, (const float *)X0, (float *)b.X, b.cur, b.head, b.cnt, b.iters,
                       b.ls, b.status, b.phase, b.evals);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

template <typename T>
__global__ void lbfgs_gather_group_kernel(int64_t B, int64_t L, const int64_t *voff,
                                          const int32_t *vdim, const T *X, const double *F,
                                          const int32_t *cur, const int32_t *st, T *Xo,
                                          double *lo, int32_t *sto) {
  const int64_t s = blockIdx.x;
  const int c = cur[s];
  const int64_t vo = voff[s];
  for (int i = threadIdx.x; i < vdim[s]; i += blockDim.x) Xo[vo + i] = X[(size_t)c * L + vo + i];
  if (threadIdx.x == 0) {
    lo[s] = F[(size_t)c * B + s];
    sto[s] = st[s];
  }
}

int launch_lbfgs_gather_group(const LbfgsBuffers &b, void *X, double *logl, int32_t *status,
                              hipStream_t s) {
  if (b.B <= 0) return SB_OK;
  if (b.dtype == DT_F64)
    hipLaunchKernelGGL(lbfgs_gather_group_kernel<double>, dim3((unsigned)b.B), dim3(256), 0, s,
                       b.B, b.Ltot, b.voff, b.vdim, (const double *)b.X, (const double *)b.F,
                       b.cur, b.status, (double *)X, logl, status);
  else
    hipLaunchKernelGGL(lbfgs_gather_group_kernel<float>, dim3((unsigned)b.B), dim3(256), 0, s,
                       b.B, b.Ltot, b.voff, b.vdim, (const float *)b.X, (const double *)b.F,
                       b.cur, b.status, (float *)X, logl, status);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

}  // namespace sb
