// Evidence of many independent problems of uneven dimension on one stream.
// Every phase of the single-problem path (section 4 modules in order) runs
// as one batched launch sequence over all problems:
//   prep        symmetry / Cholesky / log det P_k of every component at once
//   discovery   all problems' rays in one launch, one grouped GEMM over all
//               ray points, per-problem argmax and top starts
//   bulk        one L-BFGS state machine over every start of every problem;
//               per step: step kernels (one per dimension class), per-problem
//               compaction, one grouped GEMM + epilogue; blocks of steps are
//               captured once and replayed as a HIP graph
//   dedup       leader rounds of all problems together
//   polish      FP64 Newton on all problems' representatives in chunks
//               (grouped GEMM, Hessian, uneven batched Cholesky)
//   combine     one workgroup per problem
// Problems are laid out in order of padded dimension dp = ceil(d / 8) * 8;
// every vector, mean and precision row is zero beyond d.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace sb {

namespace {

// ------------------------------------------------------------ glue kernels

__device__ inline int prob_of_start(const BatchProb *probs, int n, int64_t s) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].s0 <= s)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Per start: vector offset and length, problem.
__global__ void start_tables_kernel(BatchDev b, int64_t *voff, int32_t *vdim, int32_t *sprob) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.Btot) return;
  const int p = prob_of_start(b.probs, b.n, s);
  const BatchProb pr = b.probs[p];
  voff[s] = pr.voff0 + (s - pr.s0) * pr.dp;
  vdim[s] = pr.dp;
  sprob[s] = p;
}

__global__ void init_pevals_kernel(BatchDev b, int64_t *pevals) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < b.n) pevals[p] = b.probs[p].B;
}

// Component c's d x d precision block into compact storage at off[c].
__global__ __launch_bounds__(256) void compact_prec_kernel(BatchDev b, const int32_t *comp_prob,
                                                           const int32_t *comp_k,
                                                           const int64_t *off, double *L) {
  const int c = blockIdx.y;
  const BatchProb pr = b.probs[comp_prob[c]];
  const int d = pr.d, dp = pr.dp;
  const double *P = b.P64 + pr.P_off + (size_t)comp_k[c] * dp * dp;
  const int64_t n = (int64_t)d * d;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    L[off[c] + e] = P[(e / d) * dp + (e % d)];
}

__global__ void cast_bf16_kernel(int64_t n, const double *a, bf16_t *b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = f32_to_bf16((float)a[i]);
}

// valid[s]: end point usable as a candidate; per problem: dead starts and
// candidates (pc[2p], pc[2p+1]).
__global__ void candidate_flags_group_kernel(int64_t B, const int32_t *sprob, const int32_t *status,
                                             const double *l, uint8_t *valid, int32_t *pc) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const int st = status[s];
  const bool ok = (st == 1 || st == 2 || st == 3) && isfinite(l[s]);
  valid[s] = ok ? 1 : 0;
  const int p = sprob[s];
  if (st == 4) atomicAdd(&pc[2 * p], 1);
  if (ok) atomicAdd(&pc[2 * p + 1], 1);
}

// Xp row c (stride dpm) = candidate cand[c]'s end point (dp_p entries).
template <typename T>
__global__ void gather_polish_kernel(BatchDev b, int dpm, const int32_t *cand,
                                     const int32_t *rprob, const int64_t *voff, const T *X,
                                     double *Xp) {
  const int c = blockIdx.x;
  const int dp = b.probs[rprob[c]].dp;
  const T *x = X + voff[cand[c]];
  for (int i = threadIdx.x; i < dpm; i += blockDim.x)
    Xp[(size_t)c * dpm + i] = (i < dp) ? (double)x[i] : 0.0;
}

// Newton update of row c (true dimension d_p), as in the single path.
__global__ __launch_bounds__(256) void newton_update_u_kernel(BatchDev b, int dpm,
                                                              const int32_t *rprob, double *X,
                                                              const double *dx,
                                                              const int32_t *info, int32_t *done,
                                                              int32_t *rejected,
                                                              int32_t *n_active) {
  const int c = blockIdx.x;
  __shared__ double red[4];
  if (done[c]) return;
  if (info[c] != 0) {
    if (threadIdx.x == 0) {
      rejected[c] = 1;
      done[c] = 1;
    }
    return;
  }
  const int d = b.probs[rprob[c]].d;
  double *x = X + (size_t)c * dpm;
  const double *u = dx + (size_t)c * dpm;
  double mx = 0.0, mdx = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double v = x[i] + u[i];
    x[i] = v;
    mx = fmax(mx, fabs(v));
    mdx = fmax(mdx, fabs(u[i]));
  }
  mx = block_max<256>(mx, red);
  mdx = block_max<256>(mdx, red);
  if (threadIdx.x == 0) {
    if (mdx <= 1e-14 * (mx > 1.0 ? mx : 1.0))
      done[c] = 1;
    else
      atomicAdd(n_active, 1);
  }
}

// Filters at the polished point (per-problem box); non-PD count per problem.
__global__ __launch_bounds__(256) void filter_u_kernel(BatchDev b, int dpm, const int32_t *rprob,
                                                       const double *X, const double *l,
                                                       const double *G, const int32_t *rejected,
                                                       const int32_t *info, uint8_t *ok,
                                                       int32_t *pnonpd) {
  const int c = blockIdx.x;
  __shared__ double red[4];
  const int p = rprob[c];
  const BatchProb pr = b.probs[p];
  const double *lo = b.lo + pr.box_off, *hi = b.hi + pr.box_off;
  double gmax = 0.0, outside = 0.0;
  for (int i = threadIdx.x; i < pr.d; i += 256) {
    const double g = G[(size_t)c * dpm + i];
    gmax = fmax(gmax, fabs(g));
    if (g != g) outside = 1.0;
    const double x = X[(size_t)c * dpm + i];
    if (!(x >= lo[i] && x <= hi[i])) outside = 1.0;
  }
  gmax = block_max<256>(gmax, red);
  outside = block_max<256>(outside, red);
  if (threadIdx.x == 0) {
    const bool rej = rejected[c] != 0;
    const bool pd = info[c] == 0;
    if (!rej && !pd) atomicAdd(&pnonpd[p], 1);
    ok[c] = (!rej && pd && outside == 0.0 && isfinite(l[c]) && gmax <= 1e-8) ? 1 : 0;
  }
}

// ------------------------------------------------------------ host helpers

struct DevMem {
  void *p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

struct Timer {
  hipEvent_t ev[8];
  int n = 0;
  bool ok = false;
  void init() {
    ok = true;
    for (int i = 0; i < 8; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) ok = false;
  }
  void mark(hipStream_t s) {
    if (ok && n < 8) (void)hipEventRecord(ev[n++], s);
  }
  double between(int a, int b) {
    if (!ok || a >= n || b >= n) return 0.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    return ms * 1e-3;
  }
  ~Timer() {
    if (ok)
      for (int i = 0; i < 8; ++i) (void)hipEventDestroy(ev[i]);
  }
};

// Row segments and M-tile table of a grouped GEMM (host side).
struct SegTable {
  std::vector<GSeg> segs;
  std::vector<int32_t> tile_seg, tile_idx;
  int64_t rows = 0, ylen = 0, qlen = 0;
  void add(const BatchProb &pr, int32_t prob, int64_t nrows, int bm, int bn) {
    GSeg g;
    g.prob = prob;
    g.rows = (int32_t)nrows;
    g.row0 = rows;
    g.yoff = ylen;
    g.qoff = qlen;
    const int32_t sid = (int32_t)segs.size();
    segs.push_back(g);
    for (int64_t t = 0; t < ceil_div(nrows, (int64_t)bm); ++t) {
      tile_seg.push_back(sid);
      tile_idx.push_back((int32_t)t);
    }
    rows += nrows;
    ylen += nrows * pr.K * pr.dp;
    qlen += nrows * pr.K * group_ntn(pr.dp, bn);
  }
};

// Device copy of a SegTable (carved from an arena).
struct SegDev {
  GSeg *segs = nullptr;
  int32_t *tile_seg = nullptr, *tile_idx = nullptr;
  int nseg = 0;
  int64_t ntiles = 0;
  void carve(Arena &ar, size_t nseg_cap, size_t ntile_cap) {
    segs = ar.take<GSeg>(nseg_cap);
    tile_seg = ar.take<int32_t>(ntile_cap);
    tile_idx = ar.take<int32_t>(ntile_cap);
  }
  int upload(const SegTable &t, hipStream_t s) {
    nseg = (int)t.segs.size();
    ntiles = (int64_t)t.tile_seg.size();
    if (nseg)
      SB_HIP(hipMemcpyAsync(segs, t.segs.data(), sizeof(GSeg) * nseg, hipMemcpyHostToDevice, s));
    if (ntiles) {
      SB_HIP(hipMemcpyAsync(tile_seg, t.tile_seg.data(), 4 * ntiles, hipMemcpyHostToDevice, s));
      SB_HIP(hipMemcpyAsync(tile_idx, t.tile_idx.data(), 4 * ntiles, hipMemcpyHostToDevice, s));
    }
    return SB_OK;
  }
  GroupView view(const BatchDev &b, int kind, const int64_t *rowoff, const int32_t *counts) const {
    GroupView g;
    g.probs = b.probs;
    g.segs = segs;
    g.nseg = nseg;
    g.tile_seg = tile_seg;
    g.tile_idx = tile_idx;
    g.counts = counts;
    g.kind = kind;
    g.rowoff = rowoff;
    return g;
  }
};

template <typename T>
int upload(T *dst, const std::vector<T> &src, hipStream_t s) {
  if (src.empty()) return SB_OK;
  SB_HIP(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
  return SB_OK;
}
template <typename T>
int download(std::vector<T> &dst, const T *src, size_t n, hipStream_t s) {
  dst.resize(n);
  if (n == 0) return SB_OK;
  SB_HIP(hipMemcpyAsync(dst.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost, s));
  return SB_OK;
}

// Tile shape of a grouped GEMM phase: the autotuner's choice for the batch's
// largest padded dimension and the phase's row count (timed on private
// buffers: this is a host-level entry point, which allocates anyway), among
// the 16-wide k-tiles the grouped kernels run (most of a batch's problems are
// far narrower than its widest, where a 32-wide k-tile is mostly padding:
// 64 x 128 x 32 ran the 512-problem batch in 856 ms, 64 x 64 x 16 in 693).
TileCfg batch_tiles(int dtype, int dp_max, int K_max, int64_t rows, hipStream_t s) {
  Model m;
  m.d = dp_max;
  m.K = K_max;
  TileCfg t = autotune_tiles(dtype, m, rows, s, nullptr, true, 16);
  if (t.bm != 64 && t.bm != 128) t.bm = 64;  // (the grouped kernels: 64 or 128 rows)
  return t;
}

}  // namespace

// ------------------------------------------------------------ the path

int run_evidence_batch(int n, const sb_loglik *ll, const sb_box *box, const sb_config *cfg,
                       sb_result *res, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const bool mixed = cfg[0].precision == SB_PREC_MIXED;
  const int m_hist = cfg[0].m;
  for (int j = 1; j < n; ++j) {
    if (cfg[j].precision != cfg[0].precision || cfg[j].m != m_hist) {
      set_error("problem %d: every problem of a batch needs the same precision and m", j);
      return SB_E_INVAL;
    }
  }
  const int ddt = mixed ? DT_BF16 : DT_F64;  // discovery GEMM
  const int bdt = mixed ? DT_F32 : DT_F64;   // bulk
  const size_t bes = mixed ? 4 : 8;

  // ---------------- layout: problems in order of padded dimension
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  auto dp_of = [&](int j) { return (int)align_up((size_t)ll[j].d, 8); };
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return dp_of(a) < dp_of(b); });
  std::vector<BatchProb> probs(n);
  std::vector<int32_t> rcap(n), pmaxit(n);
  std::vector<double> ptau_pre(n), ptau(n);
  int64_t Ptot = 0, Mtot = 0, Ktot = 0, Dtot = 0, Btot = 0, Ltot = 0, Rtot = 0, RLtot = 0,
          NPtot = 0, NRcap = 0, CDtot = 0;
  int dp_max = 0, d_max = 0, K_max = 0;
  for (int q = 0; q < n; ++q) {
    const int j = perm[q];
    const sb_loglik &L = ll[j];
    const sb_config &C = cfg[j];
    BatchProb &pr = probs[q];
    pr.d = L.d;
    pr.dp = dp_of(j);
    pr.K = L.K;
    pr.family = L.family;
    pr.norm = L.norm;
    pr.n_pts = C.n_points;
    pr.nu = L.nu;
    pr.c = L.logl_offset;
    pr.P_off = Ptot;
    pr.mu_off = Mtot;
    pr.beta_off = Ktot;
    pr.box_off = Dtot;
    pr.s0 = Btot;
    pr.B = C.n_starts;
    pr.voff0 = Ltot;
    pr.r0 = Rtot;
    pr.R = C.n_rays;
    pr.roff0 = RLtot;
    pr.pt0 = NPtot;
    pr.seed = C.seed;
    pr.index = j;
    Ptot += (int64_t)L.K * pr.dp * pr.dp;
    Mtot += (int64_t)L.K * pr.dp;
    Ktot += L.K;
    Dtot += pr.dp;
    Btot += pr.B;
    Ltot += pr.B * pr.dp;
    Rtot += pr.R;
    RLtot += pr.R * pr.dp;
    NPtot += pr.R * pr.n_pts;
    CDtot += (int64_t)L.K * L.d * L.d;
    dp_max = std::max(dp_max, pr.dp);
    d_max = std::max(d_max, pr.d);
    K_max = std::max(K_max, pr.K);
    rcap[q] = (int32_t)std::min<int64_t>(pr.B, 4 * (int64_t)C.max_modes + 64);
    NRcap += rcap[q];
    pmaxit[q] = C.max_iter > 0 ? C.max_iter : 10 * L.d + 200;
    ptau_pre[q] = C.dedup_tol_pre > 0 ? C.dedup_tol_pre : 0.25;
    double w = 0.0;
    for (int i = 0; i < L.d; ++i) w = std::max(w, box[j].hi[i] - box[j].lo[i]);
    ptau[q] = C.dedup_tol > 0 ? C.dedup_tol : 1e-6 * w;
    if (C.max_modes > 1024) {
      set_error("problem %d: max_modes above 1024 is not supported in a batch", j);
      return SB_E_UNSUPPORTED;
    }
  }
  if (Btot >= ((int64_t)1 << 30) || NPtot >= ((int64_t)1 << 31)) {
    set_error("batch too large: %lld starts, %lld ray points", (long long)Btot, (long long)NPtot);
    return SB_E_INVAL;
  }

  // ---------------- packed inputs on the host
  std::vector<double> hP(Ptot, 0.0), hmu(Mtot, 0.0), hlw(Ktot, 0.0), hlo(Dtot, 0.0),
      hhi(Dtot, 0.0);
  std::vector<int32_t> comp_prob, comp_k, comp_d;
  std::vector<int64_t> comp_off;
  {
    int64_t co = 0;
    for (int q = 0; q < n; ++q) {
      const int j = perm[q];
      const BatchProb &pr = probs[q];
      const int d = pr.d, dp = pr.dp;
      for (int k = 0; k < pr.K; ++k) {
        const double *Pk = ll[j].prec + (size_t)k * d * d;
        double *dst = hP.data() + pr.P_off + (size_t)k * dp * dp;
        for (int r = 0; r < d; ++r) std::memcpy(dst + (size_t)r * dp, Pk + (size_t)r * d, 8 * d);
        std::memcpy(hmu.data() + pr.mu_off + (size_t)k * dp, ll[j].mu + (size_t)k * d, 8 * d);
        hlw[pr.beta_off + k] = ll[j].log_w ? ll[j].log_w[k] : 0.0;
        comp_prob.push_back(q);
        comp_k.push_back(k);
        comp_d.push_back(d);
        comp_off.push_back(co);
        co += (int64_t)d * d;
      }
      std::memcpy(hlo.data() + pr.box_off, box[j].lo, 8 * d);
      std::memcpy(hhi.data() + pr.box_off, box[j].hi, 8 * d);
    }
  }
  const int ncomp = (int)Ktot;
  if (Ktot > 65535) {
    set_error("batch has %lld components; at most 65535 are supported", (long long)Ktot);
    return SB_E_UNSUPPORTED;
  }
  const int chunks = 16;

  // per-problem tables of the bulk and the dedup
  std::vector<int64_t> cfirst(n), ccount(n), rbase(n);
  {
    int64_t rb = 0;
    for (int q = 0; q < n; ++q) {
      cfirst[q] = probs[q].s0;
      ccount[q] = probs[q].B;
      rbase[q] = rb;
      rb += rcap[q];
    }
  }

  // grouped GEMM tables of discovery and bulk
  const TileCfg tdisc = batch_tiles(ddt, dp_max, K_max, NPtot, s);
  const TileCfg tbulk = batch_tiles(bdt, dp_max, K_max, Btot, s);
  SegTable sdisc, sbulk;
  for (int q = 0; q < n; ++q) {
    sdisc.add(probs[q], q, probs[q].R * probs[q].n_pts, tdisc.bm, tdisc.bn);
    sbulk.add(probs[q], q, probs[q].B, tbulk.bm, tbulk.bn);
  }

  // dimension classes of the L-BFGS step (starts are in order of dp)
  struct Cls {
    int64_t s_begin, count;
    int dcls;
  };
  std::vector<Cls> classes;
  {
    const int bounds[] = {64, 128, 256, 512, 1024, 2048, 4096};
    int q = 0;
    for (int bnd : bounds) {
      const int64_t sb0 = (q < n) ? probs[q].s0 : Btot;
      int64_t cnt = 0;
      while (q < n && probs[q].dp <= bnd) cnt += probs[q++].B;
      if (cnt > 0) classes.push_back({sb0, cnt, bnd});
    }
  }

  // ---------------- device memory, stage 1 (through the pre-polish dedup)
  const int m = m_hist;
  struct Stage1 {
    BatchProb *probs;
    double *P64, *mu64, *lw, *lo, *hi, *beta, *logdetP, *Lprep, *mx;
    float *P32, *mu32;
    bf16_t *Pbf;
    int32_t *comp_prob, *comp_k, *comp_d, *info, *flags;
    int64_t *comp_off;
    double *P0, *P1, *best_l, *X0;
    float *P0f, *P1f, *X0f;
    void *lpts, *qdisc;
    int32_t *best_j, *start_ray;
    SegDev sdisc, sbulk;
    void *Ybulk, *qbulk;
    int64_t *voff;
    int32_t *vdim, *sprob, *pmaxit, *pcounts, *pcand;
    double *ptol;
    int64_t *pevals;
    void *Xend;
    double *lend;
    int32_t *status_end, *rep_of, *reps, *state, *rcap;
    uint8_t *valid;
    int64_t *cfirst, *ccount, *rbase;
    double *ptau_pre;
  } D{};
  LbfgsBuffers lb;
  lb.dtype = bdt;
  lb.B = Btot;
  lb.d = dp_max;
  lb.m = m;
  lb.Ltot = Ltot;
  auto carve = [&](Arena &ar) {
    D.probs = ar.take<BatchProb>(n);
    D.P64 = ar.take<double>(Ptot);
    D.mu64 = ar.take<double>(Mtot);
    D.lw = ar.take<double>(Ktot);
    D.lo = ar.take<double>(Dtot);
    D.hi = ar.take<double>(Dtot);
    D.beta = ar.take<double>(Ktot);
    D.logdetP = ar.take<double>(Ktot);
    D.Lprep = ar.take<double>(CDtot);
    D.mx = ar.take<double>((size_t)ncomp * chunks);
    if (mixed) {
      D.P32 = ar.take<float>(Ptot);
      D.Pbf = ar.take<bf16_t>(Ptot);
      D.mu32 = ar.take<float>(Mtot);
    }
    D.comp_prob = ar.take<int32_t>(ncomp);
    D.comp_k = ar.take<int32_t>(ncomp);
    D.comp_d = ar.take<int32_t>(ncomp);
    D.comp_off = ar.take<int64_t>(ncomp);
    D.info = ar.take<int32_t>(ncomp);
    D.flags = ar.take<int32_t>(16);
    D.P0 = ar.take<double>(RLtot);
    D.P1 = ar.take<double>(RLtot);
    if (mixed) {
      D.P0f = ar.take<float>(RLtot);
      D.P1f = ar.take<float>(RLtot);
      D.X0f = ar.take<float>(Ltot);
    }
    D.lpts = ar.take<char>((size_t)NPtot * (ddt == DT_F64 ? 8 : 4));
    D.qdisc = ar.take<char>((size_t)sdisc.qlen * (ddt == DT_F64 ? 8 : 4));
    D.best_l = ar.take<double>(Rtot);
    D.best_j = ar.take<int32_t>(Rtot);
    D.start_ray = ar.take<int32_t>(Btot);
    D.X0 = ar.take<double>(Ltot);
    D.sdisc.carve(ar, sdisc.segs.size(), sdisc.tile_seg.size());
    D.sbulk.carve(ar, sbulk.segs.size(), sbulk.tile_seg.size());
    D.Ybulk = ar.take<char>(bes * (size_t)sbulk.ylen);
    D.qbulk = ar.take<char>(bes * (size_t)sbulk.qlen);
    D.voff = ar.take<int64_t>(Btot);
    D.vdim = ar.take<int32_t>(Btot);
    D.sprob = ar.take<int32_t>(Btot);
    D.pmaxit = ar.take<int32_t>(n);
    D.ptol = ar.take<double>(n);
    D.pevals = ar.take<int64_t>(n);
    D.pcounts = ar.take<int32_t>(n);
    D.pcand = ar.take<int32_t>(2 * (size_t)n);
    // L-BFGS state
    lb.X = ar.take<char>(bes * 2 * (size_t)Ltot);
    lb.G = ar.take<char>(bes * 2 * (size_t)Ltot);
    lb.F = ar.take<double>(2 * (size_t)Btot);
    lb.Pd = ar.take<char>(bes * (size_t)Ltot);
    lb.S = ar.take<char>(bes * (size_t)m * Ltot);
    lb.Yh = ar.take<char>(bes * (size_t)m * Ltot);
    lb.rho = ar.take<char>(bes * (size_t)m * Btot);
    lb.yy = ar.take<char>(bes * (size_t)m * Btot);
    lb.alpha = ar.take<char>(bes * (size_t)Btot);
    lb.gtp = ar.take<char>(bes * (size_t)Btot);
    lb.cur = ar.take<int32_t>(Btot);
    lb.head = ar.take<int32_t>(Btot);
    lb.cnt = ar.take<int32_t>(Btot);
    lb.iters = ar.take<int32_t>(Btot);
    lb.ls = ar.take<int32_t>(Btot);
    lb.status = ar.take<int32_t>(Btot);
    lb.phase = ar.take<int32_t>(Btot);
    lb.rowid = ar.take<int32_t>(Btot);
    lb.active = ar.take<int32_t>(Btot);
    lb.idx = ar.take<int32_t>(Btot);
    lb.rowoff = ar.take<int64_t>(Btot);
    lb.croff = ar.take<int64_t>(Btot);
    D.Xend = ar.take<char>(bes * (size_t)Ltot);
    D.lend = ar.take<double>(Btot);
    D.status_end = ar.take<int32_t>(Btot);
    D.valid = ar.take<uint8_t>(Btot);
    D.rep_of = ar.take<int32_t>(Btot);
    D.reps = ar.take<int32_t>(NRcap);
    D.state = ar.take<int32_t>(3 * (size_t)n + 1);
    D.rcap = ar.take<int32_t>(n);
    D.cfirst = ar.take<int64_t>(n);
    D.ccount = ar.take<int64_t>(n);
    D.rbase = ar.take<int64_t>(n);
    D.ptau_pre = ar.take<double>(n);
  };
  DevMem mem1;
  {
    Arena meas(nullptr, 0);
    carve(meas);
    const size_t bytes = meas.off + 4096;
    if (hipMalloc(&mem1.p, bytes) != hipSuccess) {
      set_error("hipMalloc of %zu bytes failed", bytes);
      return SB_E_NOMEM;
    }
    Arena ar(mem1.p, bytes);
    carve(ar);
    if (!ar.ok()) return SB_E_NOMEM;
  }
  BatchDev bd;
  bd.n = n;
  bd.probs = D.probs;
  bd.Btot = Btot;
  bd.Ltot = Ltot;
  bd.Rtot = Rtot;
  bd.RLtot = RLtot;
  bd.NPtot = NPtot;
  bd.dp_max = dp_max;
  bd.K_max = K_max;
  bd.P64 = D.P64;
  bd.mu64 = D.mu64;
  bd.beta = D.beta;
  bd.lo = D.lo;
  bd.hi = D.hi;
  bd.P32 = D.P32;
  bd.mu32 = D.mu32;
  bd.Pbf = D.Pbf;
  lb.voff = D.voff;
  lb.vdim = D.vdim;
  lb.sprob = D.sprob;
  lb.ptol = D.ptol;
  lb.pmaxit = D.pmaxit;
  lb.pevals = D.pevals;

  Timer tm;
  tm.init();
  tm.mark(s);  // 0
  int st;
  // ---------------- uploads
  if ((st = upload(D.probs, probs, s)) || (st = upload(D.P64, hP, s)) ||
      (st = upload(D.mu64, hmu, s)) || (st = upload(D.lw, hlw, s)) ||
      (st = upload(D.lo, hlo, s)) || (st = upload(D.hi, hhi, s)) ||
      (st = upload(D.comp_prob, comp_prob, s)) || (st = upload(D.comp_k, comp_k, s)) ||
      (st = upload(D.comp_d, comp_d, s)) || (st = upload(D.comp_off, comp_off, s)) ||
      (st = upload(D.pmaxit, pmaxit, s)) || (st = upload(D.rcap, rcap, s)) ||
      (st = upload(D.cfirst, cfirst, s)) || (st = upload(D.ccount, ccount, s)) ||
      (st = upload(D.rbase, rbase, s)) || (st = upload(D.ptau_pre, ptau_pre, s)))
    return st;
  if ((st = D.sdisc.upload(sdisc, s)) || (st = D.sbulk.upload(sbulk, s))) return st;
  SB_HIP(hipStreamSynchronize(s));  // host vectors may go out of scope below
  hipLaunchKernelGGL(start_tables_kernel, dim3((unsigned)ceil_div(Btot, 256)), dim3(256), 0, s,
                     bd, D.voff, D.vdim, D.sprob);
  SB_LAUNCH_CHECK();

  // ---------------- A1 prep
  if ((st = launch_fill_i32(16, 0, D.flags, s))) return st;
  if ((st = launch_check_group(bd, ncomp, D.comp_prob, D.comp_k, D.mx, chunks, D.flags, s)))
    return st;
  hipLaunchKernelGGL(compact_prec_kernel, dim3(32, ncomp), dim3(256), 0, s, bd, D.comp_prob,
                     D.comp_k, D.comp_off, D.Lprep);
  SB_LAUNCH_CHECK();
  if ((st = chol_batched_u(ncomp, D.comp_d, D.comp_off, d_max, D.Lprep, D.info, s))) return st;
  if ((st = launch_logdet_u(ncomp, D.comp_d, D.comp_off, D.Lprep, D.info, D.logdetP, s)))
    return st;
  if ((st = launch_beta_group(bd, D.lw, D.logdetP, D.beta, s))) return st;
  if (mixed) {
    if ((st = launch_cast_f64_f32(Ptot, D.P64, D.P32, s))) return st;
    if ((st = launch_cast_f64_f32(Mtot, D.mu64, D.mu32, s))) return st;
    hipLaunchKernelGGL(cast_bf16_kernel, dim3((unsigned)std::min<int64_t>(8192, ceil_div(Ptot, 256))),
                       dim3(256), 0, s, Ptot, D.P64, D.Pbf);
    SB_LAUNCH_CHECK();
  }
  std::vector<double> ptol(n);
  {
    std::vector<int32_t> hflag, hinfo;
    std::vector<double> hmx;
    if ((st = download(hflag, D.flags, 1, s)) || (st = download(hinfo, D.info, ncomp, s)) ||
        (st = download(hmx, D.mx, (size_t)ncomp * chunks, s)))
      return st;
    SB_HIP(hipStreamSynchronize(s));
    if (hflag[0]) {
      set_error("a precision matrix of the batch is not symmetric to 1e-12 relative");
      return SB_E_NOTPD;
    }
    std::vector<double> pmax(n, 0.0);
    for (int c = 0; c < ncomp; ++c) {
      const int j = perm[comp_prob[c]];
      if (hinfo[c] != 0) {
        set_error("problem %d: precision matrix %d is not positive definite (pivot %d)", j,
                  comp_k[c], hinfo[c]);
        return SB_E_NOTPD;
      }
      for (int t = 0; t < chunks; ++t) {
        const double v = hmx[(size_t)c * chunks + t];
        if (!std::isfinite(v)) {
          set_error("problem %d: precision matrix %d has non-finite entries", j, comp_k[c]);
          return SB_E_INVAL;
        }
        pmax[comp_prob[c]] = std::max(pmax[comp_prob[c]], v);
      }
    }
    for (int q = 0; q < n; ++q) {
      const int j = perm[q];
      const double gt = cfg[j].grad_tol;
      if (mixed) {
        double th = 0.0;
        for (int i = 0; i < ll[j].d; ++i)
          th = std::max(th, std::max(std::fabs(box[j].lo[i]), std::fabs(box[j].hi[i])));
        // FP32 bulk tolerance: its rounding floor 32 u32 max|P| (1 + max|theta|)
        ptol[q] = 32.0 * 5.9604644775390625e-08 * pmax[q] * (1.0 + th);
        if (gt > 0) ptol[q] = std::max(ptol[q], gt);
      } else {
        ptol[q] = gt > 0 ? gt : 1e-10;
      }
    }
  }
  if ((st = upload(D.ptol, ptol, s))) return st;
  SB_HIP(hipStreamSynchronize(s));
  tm.mark(s);  // 1

  // ---------------- A2 discovery
  if ((st = launch_rays_group(bd, D.P0, D.P1, D.P0f, D.P1f, s))) return st;
  {
    GroupView gv = D.sdisc.view(bd, 1, nullptr, nullptr);
    if ((st = launch_quad_gemm_group(ddt, bd, gv, mixed ? (const void *)D.P0f : D.P0,
                                     mixed ? (const void *)D.P1f : D.P1, D.sdisc.ntiles, nullptr,
                                     D.qdisc, tdisc, s)))
      return st;
    FinishGroupArgs f;
    f.segs = D.sdisc.segs;
    f.nseg = D.sdisc.nseg;
    f.nrows = NPtot;
    f.qpart = D.qdisc;
    f.bn = tdisc.bn;
    f.lout = D.lpts;
    if ((st = launch_finish_group(ddt == DT_F64 ? DT_F64 : DT_F32, bd, f, s))) return st;
  }
  if ((st = launch_ray_argmax_group(bd, ddt == DT_F64 ? DT_F64 : DT_F32, D.lpts, D.best_l,
                                    D.best_j, s)))
    return st;
  if ((st = launch_topn_group(bd, D.best_l, D.start_ray, s))) return st;
  if ((st = launch_gather_starts_group(bd, D.start_ray, D.best_j, D.P0, D.P1,
                                       mixed ? (void *)D.X0f : (void *)D.X0, bdt, s)))
    return st;
  tm.mark(s);  // 2

  // ---------------- A3-A5 bulk L-BFGS over every start of every problem
  int steps = 0;
  {
    if ((st = launch_lbfgs_init_group(lb, mixed ? (const void *)D.X0f : D.X0, s))) return st;
    hipLaunchKernelGGL(init_pevals_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, bd,
                       D.pevals);
    SB_LAUNCH_CHECK();
    auto eval = [&](const int64_t *rowoff, const int32_t *counts, const int32_t *fidx) -> int {
      GroupView gv = D.sbulk.view(bd, 0, rowoff, counts);
      int r = launch_quad_gemm_group(bdt, bd, gv, lb.X, nullptr, D.sbulk.ntiles, D.Ybulk,
                                     D.qbulk, tbulk, s);
      if (r) return r;
      FinishGroupArgs f;
      f.segs = D.sbulk.segs;
      f.nseg = D.sbulk.nseg;
      f.nrows = Btot;
      f.rowseg = D.sprob;  // bulk segments are the problems, rows the starts
      f.counts = counts;
      f.qpart = D.qbulk;
      f.bn = tbulk.bn;
      f.Y = D.Ybulk;
      f.F = (double *)lb.F;
      f.fidx = fidx;
      f.grad = lb.G;
      f.goff = rowoff;
      return launch_finish_group(bdt, bd, f, s);
    };
    if ((st = eval(D.voff, nullptr, nullptr))) return st;
    auto one_step = [&]() -> int {
      for (const Cls &c : classes) {
        int r = launch_lbfgs_step_range(lb, c.s_begin, c.count, c.dcls, 0.0, 0, s);
        if (r) return r;
      }
      int r = launch_compact_group(bd, lb, D.pcounts, s);
      if (r) return r;
      return eval(lb.croff, D.pcounts, lb.idx);
    };
    const char *e = getenv("SB_NO_GRAPH");
    const bool use_graph = !(e && e[0] == '1');
    const int blk = 8;
    int max_it = 0;
    for (int q = 0; q < n; ++q) max_it = std::max(max_it, pmaxit[q]);
    const int max_steps = 42 * max_it + 64;
    // (pageable host copy of the counts, read after a stream synchronisation:
    // no pinned allocation per call)
    std::vector<int32_t> hcounts((size_t)n);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int rc_st = SB_OK;
    while (steps < max_steps) {
      if (use_graph) {
        if (!exec) {
          if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            set_error("graph capture failed to begin");
            rc_st = SB_E_DEVICE;
            break;
          }
          int r = SB_OK;
          for (int k = 0; k < blk && r == SB_OK; ++k) r = one_step();
          const hipError_t e1 = hipStreamEndCapture(s, &graph);
          if (r || e1 != hipSuccess) {
            set_error("graph capture failed (%d, %s)", r, hipGetErrorString(e1));
            rc_st = r ? r : SB_E_DEVICE;
            break;
          }
          if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            set_error("graph instantiate failed");
            rc_st = SB_E_DEVICE;
            break;
          }
        }
        if (hipGraphLaunch(exec, s) != hipSuccess) {
          set_error("graph launch failed");
          rc_st = SB_E_DEVICE;
          break;
        }
      } else {
        int r = SB_OK;
        for (int k = 0; k < blk && r == SB_OK; ++k) r = one_step();
        if (r) {
          rc_st = r;
          break;
        }
      }
      steps += blk;
      if (hipMemcpyAsync(hcounts.data(), D.pcounts, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost,
                         s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        set_error("count readback failed");
        rc_st = SB_E_DEVICE;
        break;
      }
      int64_t active = 0;
      for (int q = 0; q < n; ++q) active += hcounts[q];
      if (active == 0) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc_st) return rc_st;
    if ((st = launch_lbfgs_gather_group(lb, D.Xend, D.lend, D.status_end, s))) return st;
  }
  tm.mark(s);  // 3

  // ---------------- A7 pre-polish dedup, all problems' leader rounds together
  SB_HIP(hipMemsetAsync(D.pcand, 0, sizeof(int32_t) * 2 * (size_t)n, s));
  hipLaunchKernelGGL(candidate_flags_group_kernel, dim3((unsigned)ceil_div(Btot, 256)), dim3(256),
                     0, s, Btot, D.sprob, D.status_end, D.lend, D.valid, D.pcand);
  SB_LAUNCH_CHECK();
  {
    int max_rcap = 0;
    for (int q = 0; q < n; ++q) max_rcap = std::max(max_rcap, rcap[q]);
    if ((st = dedup_group_run(n, Btot, D.cfirst, D.ccount, D.probs, D.Xend, bdt, D.voff, D.lend,
                              D.valid, D.ptau_pre, D.rep_of, D.rbase, D.rcap, D.reps, D.state,
                              max_rcap + 1, s)))
      return st;
  }
  std::vector<int32_t> hstate, hreps, hpcand;
  std::vector<int64_t> hpevals;
  if ((st = download(hstate, D.state, 3 * (size_t)n + 1, s)) ||
      (st = download(hreps, D.reps, NRcap, s)) || (st = download(hpcand, D.pcand, 2 * (size_t)n, s)) ||
      (st = download(hpevals, D.pevals, n, s)))
    return st;
  SB_HIP(hipStreamSynchronize(s));
  tm.mark(s);  // 4
  std::vector<int32_t> nrep(n);
  std::vector<uint8_t> overflow(n, 0);
  for (int q = 0; q < n; ++q) {
    nrep[q] = hstate[n + q];
    if (nrep[q] > rcap[q]) {
      overflow[q] = 1;
      nrep[q] = 0;
    }
  }

  // ---------------- A6 polish + A8/A9 Hessian, Cholesky, log det (chunks)
  // all representatives, problem by problem: global index g
  std::vector<int64_t> pfirst(n);
  int64_t NR = 0;
  for (int q = 0; q < n; ++q) {
    pfirst[q] = NR;
    NR += nrep[q];
  }
  const int dpm = dp_max;
  const int64_t H_budget = (int64_t)(512ll << 20) / 8;  // doubles of H per chunk
  const int64_t row_cap = 32768;  // rows per chunk (grid.y / grid.z limits)
  // chunk boundaries over g
  std::vector<int64_t> chunk_g0;
  std::vector<int32_t> grow_prob(NR);
  std::vector<int32_t> gcand(NR);
  {
    int64_t g = 0;
    for (int q = 0; q < n; ++q)
      for (int jr = 0; jr < nrep[q]; ++jr, ++g) {
        grow_prob[g] = q;
        gcand[g] = hreps[rbase[q] + jr];
      }
    int64_t used = 0, rows = 0;
    for (int64_t gg = 0; gg < NR; ++gg) {
      const int64_t dd = (int64_t)probs[grow_prob[gg]].d * probs[grow_prob[gg]].d;
      if (rows == 0 || used + dd > H_budget || rows >= row_cap) {
        chunk_g0.push_back(gg);
        used = 0;
        rows = 0;
      }
      used += dd;
      ++rows;
    }
    chunk_g0.push_back(NR);
  }
  int64_t PC = 0, HC = 0, YC = 0, QC = 0, SC = 0, TC = 0;
  const TileCfg tpol = batch_tiles(DT_F64, dp_max, K_max, std::min<int64_t>(NR, row_cap), s);
  std::vector<SegTable> ctabs(chunk_g0.size() > 0 ? chunk_g0.size() - 1 : 0);
  for (size_t c = 0; c + 1 < chunk_g0.size(); ++c) {
    const int64_t g0 = chunk_g0[c], g1 = chunk_g0[c + 1];
    int64_t hc = 0;
    SegTable &t = ctabs[c];
    int64_t gg = g0;
    while (gg < g1) {
      const int q = grow_prob[gg];
      int64_t e = gg;
      while (e < g1 && grow_prob[e] == q) ++e;
      t.add(probs[q], q, e - gg, tpol.bm, tpol.bn);
      hc += (e - gg) * (int64_t)probs[q].d * probs[q].d;
      gg = e;
    }
    PC = std::max(PC, g1 - g0);
    HC = std::max(HC, hc);
    YC = std::max(YC, t.ylen);
    QC = std::max(QC, t.qlen);
    SC = std::max<int64_t>(SC, (int64_t)t.segs.size());
    TC = std::max<int64_t>(TC, (int64_t)t.tile_seg.size());
  }
  struct Stage2 {
    double *Xp, *Gp, *dx, *lp, *auxp, *H, *ldh, *Y, *qp;
    int32_t *pinfo, *done, *rejected, *nact, *rprob, *cand, *nv, *pnonpd;
    int64_t *hoff, *rowoffp;
    uint8_t *okp;
    SegDev sd;
    double *XA, *lA, *ldhA, *mlz, *logz, *ptau;
    uint8_t *okA;
    int64_t *xoffA, *cf2, *cc2, *rb2;
    int32_t *rep2_of, *reps2, *state2, *rc2, *order;
  } E{};
  auto carve2 = [&](Arena &ar) {
    const int64_t pc = std::max<int64_t>(PC, 1);
    E.Xp = ar.take<double>((size_t)pc * dpm);
    E.Gp = ar.take<double>((size_t)pc * dpm);
    E.dx = ar.take<double>((size_t)pc * dpm);
    E.lp = ar.take<double>(pc);
    E.auxp = ar.take<double>((size_t)pc * K_max);
    E.H = ar.take<double>(std::max<int64_t>(HC, 1));
    E.ldh = ar.take<double>(pc);
    E.Y = ar.take<double>(std::max<int64_t>(YC, 1));
    E.qp = ar.take<double>(std::max<int64_t>(QC, 1));
    E.pinfo = ar.take<int32_t>(pc);
    E.done = ar.take<int32_t>(pc);
    E.rejected = ar.take<int32_t>(pc);
    E.nact = ar.take<int32_t>(4);
    E.rprob = ar.take<int32_t>(pc);
    E.cand = ar.take<int32_t>(pc);
    E.nv = ar.take<int32_t>(pc);
    E.pnonpd = ar.take<int32_t>(n);
    E.hoff = ar.take<int64_t>(pc);
    E.rowoffp = ar.take<int64_t>(pc);
    E.okp = ar.take<uint8_t>(pc);
    E.sd.carve(ar, std::max<int64_t>(SC, 1), std::max<int64_t>(TC, 1));
    const int64_t nr = std::max<int64_t>(NR, 1);
    E.XA = ar.take<double>((size_t)nr * dpm);
    E.lA = ar.take<double>(nr);
    E.ldhA = ar.take<double>(nr);
    E.okA = ar.take<uint8_t>(nr);
    E.xoffA = ar.take<int64_t>(nr);
    E.rep2_of = ar.take<int32_t>(nr);
    E.reps2 = ar.take<int32_t>(nr);
    E.order = ar.take<int32_t>(nr);
    E.mlz = ar.take<double>(nr);
    E.cf2 = ar.take<int64_t>(n);
    E.cc2 = ar.take<int64_t>(n);
    E.rb2 = ar.take<int64_t>(n);
    E.rc2 = ar.take<int32_t>(n);
    E.state2 = ar.take<int32_t>(3 * (size_t)n + 1);
    E.logz = ar.take<double>(n);
    E.ptau = ar.take<double>(n);
  };
  DevMem mem2;
  {
    Arena meas(nullptr, 0);
    carve2(meas);
    const size_t bytes = meas.off + 4096;
    if (hipMalloc(&mem2.p, bytes) != hipSuccess) {
      set_error("hipMalloc of %zu bytes failed", bytes);
      return SB_E_NOMEM;
    }
    Arena ar(mem2.p, bytes);
    carve2(ar);
    if (!ar.ok()) return SB_E_NOMEM;
  }
  SB_HIP(hipMemsetAsync(E.pnonpd, 0, sizeof(int32_t) * (size_t)n, s));
  int64_t pol_grad = 0, pol_hess = 0;
  std::vector<int64_t> pgrad(n, 0), phess(n, 0);
  for (size_t c = 0; c + 1 < chunk_g0.size(); ++c) {
    const int64_t g0 = chunk_g0[c], g1 = chunk_g0[c + 1];
    const int C = (int)(g1 - g0);
    const SegTable &t = ctabs[c];
    std::vector<int32_t> rprob(C), cand(C), nv(C);
    std::vector<int64_t> hoff(C), rowoffp(C);
    int64_t ho = 0;
    int dmc = 0;
    for (int r = 0; r < C; ++r) {
      const int q = grow_prob[g0 + r];
      rprob[r] = q;
      cand[r] = gcand[g0 + r];
      nv[r] = probs[q].d;
      hoff[r] = ho;
      ho += (int64_t)probs[q].d * probs[q].d;
      rowoffp[r] = (int64_t)r * dpm;
      dmc = std::max(dmc, probs[q].d);
    }
    SB_HIP(hipStreamSynchronize(s));  // previous chunk done with the tables
    if ((st = upload(E.rprob, rprob, s)) || (st = upload(E.cand, cand, s)) ||
        (st = upload(E.nv, nv, s)) || (st = upload(E.hoff, hoff, s)) ||
        (st = upload(E.rowoffp, rowoffp, s)) || (st = E.sd.upload(t, s)))
      return st;
    SB_HIP(hipStreamSynchronize(s));
    if (mixed)
      hipLaunchKernelGGL(gather_polish_kernel<float>, dim3(C), dim3(256), 0, s, bd, dpm, E.cand,
                         E.rprob, D.voff, (const float *)D.Xend, E.Xp);
    else
      hipLaunchKernelGGL(gather_polish_kernel<double>, dim3(C), dim3(256), 0, s, bd, dpm, E.cand,
                         E.rprob, D.voff, (const double *)D.Xend, E.Xp);
    SB_LAUNCH_CHECK();
    auto eval = [&]() -> int {
      GroupView gv = E.sd.view(bd, 0, E.rowoffp, nullptr);
      int r = launch_quad_gemm_group(DT_F64, bd, gv, E.Xp, nullptr, E.sd.ntiles, E.Y, E.qp, tpol,
                                     s);
      if (r) return r;
      FinishGroupArgs f;
      f.segs = E.sd.segs;
      f.nseg = E.sd.nseg;
      f.nrows = C;
      f.qpart = E.qp;
      f.bn = tpol.bn;
      f.Y = E.Y;
      f.F = E.lp;
      f.grad = E.Gp;
      f.goff = E.rowoffp;
      f.aux = E.auxp;
      f.auxs = K_max;
      if ((r = launch_finish_group(DT_F64, bd, f, s))) return r;
      return launch_hessian_group(bd, E.sd.segs, E.sd.nseg, C, E.Y, E.auxp, K_max, E.Gp, dpm,
                                  E.hoff, E.H, dmc, s);
    };
    if ((st = launch_fill_i32(C, 0, E.done, s))) return st;
    if ((st = launch_fill_i32(C, 0, E.rejected, s))) return st;
    int32_t nact_h = 0;
    int iters = 0;
    for (int it = 0; it < 20; ++it) {
      if ((st = eval())) return st;
      ++iters;
      if ((st = chol_batched_u(C, E.nv, E.hoff, dmc, E.H, E.pinfo, s))) return st;
      if ((st = launch_chol_solve_u(C, E.nv, E.hoff, dmc, E.H, E.Gp, E.dx, dpm, E.pinfo, s)))
        return st;
      if ((st = launch_fill_i32(1, 0, E.nact, s))) return st;
      hipLaunchKernelGGL(newton_update_u_kernel, dim3(C), dim3(256), 0, s, bd, dpm, E.rprob, E.Xp,
                         E.dx, E.pinfo, E.done, E.rejected, E.nact);
      SB_LAUNCH_CHECK();
      SB_HIP(hipMemcpyAsync(&nact_h, E.nact, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      SB_HIP(hipStreamSynchronize(s));
      if (nact_h == 0) break;
    }
    // final point
    if ((st = eval())) return st;
    ++iters;
    if ((st = chol_batched_u(C, E.nv, E.hoff, dmc, E.H, E.pinfo, s))) return st;
    if ((st = launch_logdet_u(C, E.nv, E.hoff, E.H, E.pinfo, E.ldh, s))) return st;
    hipLaunchKernelGGL(filter_u_kernel, dim3(C), dim3(256), 0, s, bd, dpm, E.rprob, E.Xp, E.lp,
                       E.Gp, E.rejected, E.pinfo, E.okp, E.pnonpd);
    SB_LAUNCH_CHECK();
    SB_HIP(hipMemcpyAsync(E.XA + (size_t)g0 * dpm, E.Xp, sizeof(double) * (size_t)C * dpm,
                          hipMemcpyDeviceToDevice, s));
    SB_HIP(hipMemcpyAsync(E.lA + g0, E.lp, sizeof(double) * C, hipMemcpyDeviceToDevice, s));
    SB_HIP(hipMemcpyAsync(E.ldhA + g0, E.ldh, sizeof(double) * C, hipMemcpyDeviceToDevice, s));
    SB_HIP(hipMemcpyAsync(E.okA + g0, E.okp, C, hipMemcpyDeviceToDevice, s));
    for (int r = 0; r < C; ++r) {
      pgrad[rprob[r]] += iters;
      phess[rprob[r]] += iters;
    }
    pol_grad += (int64_t)iters * C;
    pol_hess += (int64_t)iters * C;
  }
  tm.mark(s);  // 5

  // ---------------- A7 final dedup and A10 combine
  {
    std::vector<int64_t> xoffA(NR), cf2(n), cc2(n);
    std::vector<int32_t> rc2(n);
    for (int64_t g = 0; g < NR; ++g) xoffA[g] = g * dpm;
    for (int q = 0; q < n; ++q) {
      cf2[q] = pfirst[q];
      cc2[q] = nrep[q];
      rc2[q] = nrep[q];
    }
    SB_HIP(hipStreamSynchronize(s));
    if ((st = upload(E.xoffA, xoffA, s)) || (st = upload(E.cf2, cf2, s)) ||
        (st = upload(E.cc2, cc2, s)) || (st = upload(E.rb2, cf2, s)) ||
        (st = upload(E.rc2, rc2, s)) || (st = upload(E.ptau, ptau, s)))
      return st;
    SB_HIP(hipStreamSynchronize(s));
    int max_nrep = 0;
    for (int q = 0; q < n; ++q) max_nrep = std::max(max_nrep, nrep[q]);
    if ((st = dedup_group_run(n, NR, E.cf2, E.cc2, D.probs, E.XA, DT_F64, E.xoffA, E.lA, E.okA,
                              E.ptau, E.rep2_of, E.rb2, E.rc2, E.reps2, E.state2, max_nrep + 1,
                              s)))
      return st;
    if ((st = launch_combine_group(bd, E.state2, E.rb2, E.rc2, E.reps2, E.lA, E.ldhA, E.XA,
                                   E.xoffA, E.order, E.mlz, E.logz, s)))
      return st;
  }
  std::vector<int32_t> hstate2, horder, hnonpd;
  std::vector<double> hmlz, hlogz, hXA, hlA, hldhA;
  if ((st = download(hstate2, E.state2, 3 * (size_t)n + 1, s)) ||
      (st = download(horder, E.order, NR, s)) || (st = download(hmlz, E.mlz, NR, s)) ||
      (st = download(hlogz, E.logz, n, s)) || (st = download(hXA, E.XA, (size_t)NR * dpm, s)) ||
      (st = download(hlA, E.lA, NR, s)) || (st = download(hldhA, E.ldhA, NR, s)) ||
      (st = download(hnonpd, E.pnonpd, n, s)))
    return st;
  SB_HIP(hipStreamSynchronize(s));
  tm.mark(s);  // 6

  // ---------------- results, in the caller's problem order
  const double total =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  int ret = SB_OK;
  for (int q = 0; q < n; ++q) {
    const int j = perm[q];
    sb_result &r = res[j];
    const int d = probs[q].d;
    r.n_logl_evals = probs[q].R * probs[q].n_pts;
    r.n_grad_evals = hpevals[q] + pgrad[q];
    r.n_hess_evals = phess[q];
    r.iterations = steps;
    r.n_dead_starts = hpcand[2 * q];
    r.n_candidates = hpcand[2 * q + 1];
    r.n_rejected_nonpd = hnonpd[q];
    r.n_reps_pre = overflow[q] ? hstate[n + q] : nrep[q];
    for (int i = 0; i < 8; ++i) r.seconds[i] = 0.0;
    r.seconds[0] = tm.between(0, 1);
    r.seconds[1] = tm.between(1, 2);
    r.seconds[2] = tm.between(2, 3);
    r.seconds[3] = tm.between(3, 4);
    r.seconds[4] = tm.between(4, 5);
    r.seconds[6] = tm.between(5, 6);
    r.seconds[7] = total;
    int pst = SB_OK;
    const int nm = hstate2[n + q];
    r.n_modes = nm;
    if (overflow[q]) {
      r.log_z = NAN;
      r.n_modes = 0;
      pst = SB_E_CAPACITY;
      if (ret == SB_OK)
        set_error("problem %d: more than %d representatives after the pre-polish dedup", j,
                  rcap[q]);
    } else if (nm == 0) {
      r.log_z = -INFINITY;
      pst = SB_E_NOMODE;
    } else if (nm > cfg[j].max_modes) {
      r.log_z = NAN;
      pst = SB_E_CAPACITY;
      if (ret == SB_OK) set_error("problem %d: %d modes found, max_modes = %d", j, nm,
                                  cfg[j].max_modes);
    } else {
      r.log_z = hlogz[q];
      for (int k = 0; k < nm; ++k) {
        const int64_t g = horder[pfirst[q] + k];
        if (r.modes) std::memcpy(r.modes + (size_t)k * d, hXA.data() + (size_t)g * dpm, 8 * d);
        if (r.mode_log_z) r.mode_log_z[k] = hmlz[pfirst[q] + k];
        if (r.mode_logl) r.mode_logl[k] = hlA[g];
        if (r.log_det_h) r.log_det_h[k] = hldhA[g];
      }
    }
    if (pst != SB_OK && pst != SB_E_NOMODE && ret == SB_OK) ret = pst;
  }
  (void)pol_grad;
  (void)pol_hess;
  return ret;
}

}  // namespace sb
