// Host orchestration of the evidence path on one GPU and one stream:
//   A1 prep        Cholesky of each P_k -> log det P_k, beta_k; low-precision copies
//   A2 discovery   rays -> l at ray points (GEMM) -> per-ray argmax -> top starts
//   A3-A5 bulk     batched L-BFGS: [step, compact, GEMM, finish] per batch
//                  step, blocks of steps captured and replayed as HIP graphs;
//                  the host reads one active-start count per block
//   A7 pre-dedup   L-infinity leader clustering of the optimiser's end points
//   A6 polish      FP64 Newton with the exact Hessian on the representatives
//   A8/A9          Hessian assembly, Cholesky, log det, filters
//   A7 final dedup and A10 combine -> log Z
// Small glue kernels (flags, gathers, the Newton update) live here too.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <vector>

#include "internal.h"

namespace sb {

static thread_local char g_err[512] = {0};
void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char *last_error() { return g_err; }

// ------------------------------------------------------------ glue kernels

// valid[s] = optimiser end point usable as a candidate (not dead, finite l)
template <typename T>
__global__ void candidate_flags_kernel(int64_t B, const int32_t *status, const T *l,
                                       uint8_t *valid, int32_t *counts) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const int st = status[s];
  const bool ok = (st == 1 || st == 2 || st == 3) && isfinite((double)l[s]);
  valid[s] = ok ? 1 : 0;
  if (st == 4) atomicAdd(&counts[0], 1);  // integer count: order-independent
  if (ok) atomicAdd(&counts[1], 1);
}

// Xp[c] = (double) X[reps[c]]
template <typename T>
__global__ void gather_reps_kernel(int d, const int32_t *reps, const T *X, double *Xp) {
  const int c = blockIdx.x;
  const int r = reps[c];
  for (int i = threadIdx.x; i < d; i += blockDim.x)
    Xp[(size_t)c * d + i] = (double)X[(size_t)r * d + i];
}

// Newton update x += dx for reps not yet done; done when the factorisation
// failed (rejected) or ||dx||_inf <= 1e-14 max(1, ||x||_inf) after the update.
__global__ __launch_bounds__(256) void newton_update_kernel(int d, double *X, const double *dx,
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
  double mx = 0.0, mdx = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    double v = X[(size_t)c * d + i] + dx[(size_t)c * d + i];
    X[(size_t)c * d + i] = v;
    mx = fmax(mx, fabs(v));
    mdx = fmax(mdx, fabs(dx[(size_t)c * d + i]));
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

// Filters at the polished point: not rejected, factorisation ok, inside the
// box, finite l, ||grad l||_inf <= 1e-8.
__global__ __launch_bounds__(256) void filter_kernel(int d, const double *X, const double *l,
                                                     const double *G, const double *lo,
                                                     const double *hi, const int32_t *rejected,
                                                     const int32_t *info, uint8_t *ok,
                                                     int32_t *n_nonpd) {
  const int c = blockIdx.x;
  __shared__ double red[4];
  double gmax = 0.0, outside = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    double g = G[(size_t)c * d + i];
    gmax = fmax(gmax, fabs(g));
    if (g != g) outside = 1.0;
    double x = X[(size_t)c * d + i];
    if (!(x >= lo[i] && x <= hi[i])) outside = 1.0;
  }
  gmax = block_max<256>(gmax, red);
  outside = block_max<256>(outside, red);
  if (threadIdx.x == 0) {
    const bool rej = rejected[c] != 0;
    const bool pd = info[c] == 0;
    if (!rej && !pd) atomicAdd(n_nonpd, 1);
    ok[c] = (!rej && pd && outside == 0.0 && isfinite(l[c]) && gmax <= 1e-8) ? 1 : 0;
  }
}

// out[i] = in[idx[i]] for rows of length d (FP64)
__global__ void gather_rows_kernel(int d, const int32_t *idx, const double *in, double *out) {
  const int i = blockIdx.x;
  const int r = idx[i];
  for (int j = threadIdx.x; j < d; j += blockDim.x)
    out[(size_t)i * d + j] = in[(size_t)r * d + j];
}
__global__ void gather_scalars_kernel(int n, const int32_t *idx, const double *a, const double *b,
                                      double *ao, double *bo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ao[i] = a[idx[i]];
  bo[i] = b[idx[i]];
}

// ------------------------------------------------------------ helpers

// Phase marks on the events of an execution context (none without one).
struct Timer {
  hipEvent_t *ev = nullptr;
  int n = 0;
  bool ok = false;
  void init(ExecCtx *ex) {
    if (ex && ex->ev_ok) {
      ev = ex->ev;
      ok = true;
    }
  }
  void mark(hipStream_t s) {
    if (ok && n < 10) hipEventRecord(ev[n++], s);
  }
  double between(int a, int b) {
    if (!ok || a >= n || b >= n) return 0.0;
    float ms = 0.f;
    hipEventElapsedTime(&ms, ev[a], ev[b]);
    return ms * 1e-3;
  }
};

// The prior box on the device: info[0] = 1 where some bound is not finite or
// lo_i >= hi_i (else 0), info[1] = max_i max(|lo_i|, |hi_i|), info[2] =
// max_i (hi_i - lo_i).  One workgroup; maxima need no fixed order.
__global__ __launch_bounds__(256) void box_info_kernel(int d, const double *lo, const double *hi,
                                                       double *info) {
  __shared__ double part[3][4];
  double bad = 0.0, mabs = 0.0, mw = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double a = lo[i], b = hi[i];
    if (!(isfinite(a) && isfinite(b) && a < b)) bad = 1.0;
    mabs = fmax(mabs, fmax(fabs(a), fabs(b)));
    mw = fmax(mw, b - a);
  }
  bad = wave_max(bad);
  mabs = wave_max(mabs);
  mw = wave_max(mw);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    part[0][w] = bad;
    part[1][w] = mabs;
    part[2][w] = mw;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int j = threadIdx.x;
    info[j] = fmax(fmax(part[j][0], part[j][1]), fmax(part[j][2], part[j][3]));
  }
}

// One evaluation of l (+grad, +aux) at B rows of X through GEMM + finish.
struct Evaluator {
  Model m;
  int dtype = DT_F64;      // data / epilogue type
  int gemm_dtype = -1;     // contraction type (-1: dtype)
  int64_t cap = 0;  // rows
  void *Y = nullptr, *qpart = nullptr;
  int64_t ldy = 0;
  TileCfg tile;
  int ntn = 0;
  // Two-stage mixture contraction (split BF16, K > 1): q_k = |Z_k|^2 with
  // Z_k = (X - mu_k) U_k^T, U_k = L_k^T from P_k = L_k L_k^T (the triangle
  // halves the contraction), then Y_k = (X - mu_k) P_k^T only for the rows
  // whose responsibility r_k is not zero.  A separated mixture's start sees
  // one component, so the K contractions of a row shrink to K/2 + 1.
  bool two_stage = false;
  // Screened instead: a rows pass bounds every q_k from the row's last
  // evaluated point (bounds there, widened by the distance moved) and lists
  // only the components the bounds cannot rule out; the split contraction
  // forms Y_k and q_k for those, and a post pass forms l and r from its q and
  // renews the listed components' bounds.
  bool screen = false;
  const double *rho = nullptr;  // [K] largest absolute row sum of P_k
  int64_t nstate = 0;           // operand rows with state (both L-BFGS slots)
  float *xref = nullptr, *nrm = nullptr;
  double *bnd = nullptr;
  int32_t *hasref = nullptr;
  uint32_t *mask = nullptr;  // [cap]
  const bf16_t *Uhi = nullptr, *Ulo = nullptr;  // [K][d][d]
  TileCfg tile1, tile2;                         // tiles of the two stages
  int32_t *lcnt = nullptr, *lrows = nullptr, *lxrows = nullptr, *lgdst = nullptr;
  float *resp = nullptr;  // [cap][K]
  // Single Gaussian on the split kernel: grad l = -Y, so the contraction
  // writes -Y straight into the gradient rows and the epilogue forms l only.
  bool grad_direct = false;
  int carve(Arena &ar) {
    const size_t es = (dtype == DT_F64) ? 8 : 4;
    ldy = (int64_t)m.K * m.d;
    Y = ar.take<char>(es * (size_t)cap * ldy);
    qpart = ar.take<char>(es * (size_t)cap * m.K * ceil_div(m.d, 64));
    if (two_stage) {
      lcnt = ar.take<int32_t>(m.K);
      lrows = ar.take<int32_t>((size_t)m.K * cap);
      lxrows = ar.take<int32_t>((size_t)m.K * cap);
      resp = ar.take<float>((size_t)m.K * cap);
      if (screen) {
        nstate = 2 * cap;
        xref = ar.take<float>((size_t)nstate * m.d);
        nrm = ar.take<float>((size_t)cap * m.K);
        bnd = ar.take<double>((size_t)nstate * 2 * m.K);
        hasref = ar.take<int32_t>(nstate);
        mask = ar.take<uint32_t>(cap);
        lgdst = ar.take<int32_t>((size_t)m.K * cap);
      }
    }
    return ar.ok() ? SB_OK : SB_E_NOMEM;
  }
  // Screened: the screen and list passes, the split contraction of the
  // listed (row, component) pairs (Y and q), the post pass (l, r, refreshed
  // bounds).  Unscreened: stage 1 (q partials), l and the
  // responsibilities with the row lists, stage 2 (Y of the active
  // components); the epilogue takes r from the rows pass.  Either way it reads
  // exactly the Y rows the contraction wrote.
  // (screened, with grad: the rows with a single listed component take their
  // gradient from the contraction, the epilogue skips them)
  int contract_two_stage(const ASrc &a, int64_t M, const int32_t *count, void *logl,
                         const int32_t *outmap, bool logl_f64, void *grad, int64_t ldg,
                         hipStream_t s) {
    int st;
    if (screen) {
      ScreenArgs sa;
      sa.M = M;
      sa.count = count;
      sa.X = (const float *)a.X;
      sa.ldx = a.ldx;
      sa.rowmap = a.rowmap;
      sa.nstate = nstate;
      sa.rho = rho;
      sa.xref = xref;
      sa.bnd = bnd;
      sa.hasref = hasref;
      sa.nrm = nrm;
      sa.qpart = (float *)qpart;
      sa.ntn = (int)ceil_div(m.d, tile2.bn == 256 ? 256 : 128);
      sa.mask = mask;
      sa.cnt = lcnt;
      sa.rows = lrows;
      sa.xrows = lxrows;
      sa.cap = cap;
      sa.logl = logl;
      sa.outmap = outmap;
      sa.logl_f64 = logl_f64;
      sa.resp = resp;
      const bool gdir = grad && dtype == DT_F32;  // (the contraction writes FP32 rows)
      sa.gdst = gdir ? lgdst : nullptr;
      if ((a.rows > 0 ? a.rows : M) > nstate) {
        set_error("screened mixture: %lld operand rows, state for %lld",
                  (long long)(a.rows > 0 ? a.rows : M), (long long)nstate);
        return SB_E_INVAL;
      }
      if ((st = launch_mixture_screen(m, sa, s))) return st;
      ASrc a2 = a;
      a2.rowmap = lxrows;
      a2.rows = a.rows > 0 ? a.rows : M;
      QuadOut o2;
      o2.Y = Y;
      o2.ldy = ldy;
      o2.ymap = lrows;
      o2.gcnt = lcnt;
      o2.gcap = cap;
      o2.qpart = qpart;
      if (gdir) {
        o2.gdst = lgdst;
        o2.gdir = grad;
        o2.ldg = ldg;
      }
      if ((st = launch_quad_gemm(DT_F32S, m, a2, cap, nullptr, o2, tile2, s))) return st;
      if (o2.ntn != sa.ntn) {
        set_error("screened mixture: %d column tiles, expected %d", o2.ntn, sa.ntn);
        return SB_E_UNSUPPORTED;
      }
      ntn = o2.ntn;
      return launch_mixture_post(m, sa, s);
    }
    Model m1 = m;
    m1.Phi = Uhi;
    m1.Plo = Ulo;
    QuadOut o1;
    o1.ldy = ldy;
    o1.qpart = qpart;
    o1.sumsq = true;
    st = launch_quad_gemm(DT_F32S, m1, a, M, count, o1, tile1, s);
    if (st) return st;
    ntn = o1.ntn;
    if ((st = launch_fill_i32(m.K, 0, lcnt, s))) return st;
    MixRowsArgs mr;
    mr.M = M;
    mr.count = count;
    mr.qpart = (const float *)qpart;
    mr.ntn = ntn;
    mr.rowmap = a.rowmap;
    mr.outmap = outmap;
    mr.logl = logl;
    mr.logl_f64 = logl_f64;
    mr.resp = resp;
    mr.cnt = lcnt;
    mr.rows = lrows;
    mr.xrows = lxrows;
    mr.cap = cap;
    if ((st = launch_mixture_rows(m, mr, s))) return st;
    ASrc a2 = a;
    a2.rowmap = lxrows;
    a2.rows = a.rows > 0 ? a.rows : M;
    QuadOut o2;
    o2.Y = Y;
    o2.ldy = ldy;
    o2.ymap = lrows;
    o2.gcnt = lcnt;
    o2.gcap = cap;
    return launch_quad_gemm(DT_F32S, m, a2, cap, nullptr, o2, tile2, s);
  }
  // rows: X rows (via rowmap if given), count: device count or null (M rows)
  int run(const ASrc &a, int64_t M, const int32_t *count, void *logl, void *grad, int64_t ldg,
          const int32_t *outmap, void *aux, bool logl_f64, hipStream_t s, bool want_y = true) {
    int st;
    const bool ts = two_stage && want_y && !aux;
    const bool gd = grad_direct && want_y && grad && !aux;
    // small FP64 problems without a Y consumer (the Hessian assembly reads Y
    // and passes aux): contraction and epilogue fused in one launch
    if (!aux && !ts && !gd && dtype == DT_F64 && (gemm_dtype < 0 || gemm_dtype == DT_F64) &&
        fused_logl_grad_ok(m, a))
      return launch_fused_logl_grad(m, a, M, count, outmap, (double *)logl, (double *)grad, ldg,
                                    nullptr, s);
    if (ts) {
      if ((st = contract_two_stage(a, M, count, logl, outmap, logl_f64, grad, ldg, s))) return st;
    } else if (gd) {
      QuadOut o;
      o.Y = grad;
      o.ldy = ldg;
      o.ymap = outmap;
      o.yneg = true;
      o.qpart = qpart;
      if ((st = launch_quad_gemm(DT_F32S, m, a, M, count, o, tile, s))) return st;
      ntn = o.ntn;
    } else {
      QuadOut o;
      o.Y = want_y ? Y : nullptr;
      o.ldy = ldy;
      o.qpart = qpart;
      st = launch_quad_gemm(gemm_dtype >= 0 ? gemm_dtype : dtype, m, a, M, count, o, tile, s);
      if (st) return st;
      ntn = o.ntn;
    }
    FinishArgs f;
    f.M = M;
    f.count = count;
    f.outmap = outmap;
    f.qpart = qpart;
    f.ntn = ntn;
    f.Y = Y;
    f.ldy = ldy;
    f.logl = logl;
    f.grad = grad;
    f.ldg = ldg;
    f.aux = aux;
    f.logl_f64 = logl_f64;
    f.resp = ts ? resp : nullptr;
    if (ts && screen && grad && dtype == DT_F32)
      f.skip1 = mask;  // (single-component rows: by the contraction)
    if (gd) f.grad = nullptr;  // (written by the contraction)
    return launch_finish(dtype, m, f, s);
  }
};

// ------------------------------------------------------------ config

struct RunCfg {
  int R, n_pts, n_starts, m, max_iter, max_modes, precision;
  double grad_tol, dedup_tol, dedup_tol_pre;
  uint64_t seed;
  int cap_pre;       // representatives polished at most
  int polish_chunk;  // reps per Newton batch
  int blk;           // batch steps per captured graph
  bool use_graph;
  bool cyc = false;     // the ChiSao cycle replaces the single convergence phase
  sb_chisao_config cc;  // its parameters, defaults filled in
};

static RunCfg resolve(const sb_loglik *ll, const sb_config *c,
                      const sb_chisao_config *cc = nullptr) {
  RunCfg r;
  r.R = c->n_rays;
  r.n_pts = c->n_points;
  r.n_starts = c->n_starts;
  r.m = c->m;
  r.max_iter = c->max_iter > 0 ? c->max_iter : 10 * ll->d + 200;
  r.max_modes = c->max_modes;
  r.precision = c->precision;
  r.grad_tol = c->grad_tol;
  r.dedup_tol = c->dedup_tol;
  r.dedup_tol_pre = c->dedup_tol_pre > 0 ? c->dedup_tol_pre : 0.25;
  r.seed = c->seed;
  r.cap_pre = std::min(r.n_starts, 4 * r.max_modes + 64);
  r.polish_chunk = std::max(1, std::min(r.cap_pre, (int)std::max<int64_t>(
                                                       1, (int64_t)(512ll << 20) /
                                                              (8ll * ll->d * ll->d))));
  r.blk = 8;
  const char *e = getenv("SB_NO_GRAPH");
  r.use_graph = !(e && e[0] == '1');
  if (cc) {
    r.cyc = true;
    r.cc = *cc;
    if (r.cc.n_conv <= 0) r.cc.n_conv = r.max_iter;
    if (!(r.cc.stick_tol > 0)) r.cc.stick_tol = 1e-6;
    if (r.cc.n_reseed_pts <= 0) r.cc.n_reseed_pts = 32;
    if (r.cc.n_smooth <= 0) r.cc.n_smooth = 4;
    if (!(r.cc.alpha_cloud > 0)) r.cc.alpha_cloud = 0.01;
    if (!(r.cc.alpha_anti > 0)) r.cc.alpha_anti = 0.01;
    if (!(r.cc.ref_delta > 0)) r.cc.ref_delta = 10.0;
    if (r.cc.n_ref < 0) r.cc.n_ref = 0;
  }
  return r;
}

// Workspace layout (measured with a null arena, carved with the real one).
struct Layout {
  // prep
  double *Lprep = nullptr, *logdetP = nullptr, *beta = nullptr, *mx = nullptr;
  double *boxinfo = nullptr;  // [4] from box_info_kernel
  int32_t *info = nullptr, *flags = nullptr;
  float *P32 = nullptr, *mu32 = nullptr;
  bf16_t *Pbf = nullptr, *Plo = nullptr;
  bf16_t *Uhi = nullptr, *Ulo = nullptr;  // split U_k = L_k^T (two-stage mixture bulk)
  double *rho = nullptr;     // [K] bound of P_k's largest eigenvalue (screen)
  double *pw = nullptr;      // [2 K d + K] power steps
  int32_t *cinfo = nullptr;  // [K] certifying factorisations
  // discovery
  double *P0 = nullptr, *P1 = nullptr, *best_l = nullptr, *X0 = nullptr;
  float *P0f = nullptr, *P1f = nullptr;
  void *lpts = nullptr;
  int32_t *best_j = nullptr, *start_ray = nullptr;
  Evaluator disc;
  // bulk
  LbfgsBuffers lb;
  Evaluator bulk;
  void *X0b = nullptr, *Xend = nullptr, *lend = nullptr;
  int32_t *status = nullptr, *counts = nullptr;
  uint8_t *valid = nullptr;
  int32_t *rep_of = nullptr, *reps = nullptr;
  // polish (chunk)
  Evaluator pol;
  double *Xp = nullptr, *lp = nullptr, *Gp = nullptr, *auxp = nullptr, *H = nullptr, *dx = nullptr, *ldh = nullptr;
  int32_t *pinfo = nullptr, *done = nullptr, *rejected = nullptr, *nact = nullptr;
  uint8_t *okp = nullptr;
  // all polished reps (cap_pre)
  double *XA = nullptr, *lA = nullptr, *ldhA = nullptr;
  uint8_t *okA = nullptr;
  int32_t *rep2 = nullptr, *rep2_of = nullptr;
  // modes
  double *Xm = nullptr, *lm = nullptr, *ldm = nullptr, *mlz = nullptr, *logz = nullptr,
         *Xs = nullptr, *ls_ = nullptr, *lds = nullptr;
  int32_t *order = nullptr;
  Arena dedup_ar;
  // ChiSao cycle: slot flags, l of the active slots, end gradients, dedup
  // outputs, host-built index lists, directions and ray origins, the spread
  // per coordinate, the perturbations, and the moves' own workspaces
  uint8_t *cactive = nullptr, *cstuck = nullptr, *cconv = nullptr, *cfrozen = nullptr;
  double *clmask = nullptr, *Gend = nullptr, *U = nullptr, *Xo = nullptr, *sd = nullptr,
         *Z = nullptr;
  int32_t *crep_of = nullptr, *creps = nullptr, *clist = nullptr;  // clist [4][B]
  void *reseed_ws = nullptr, *explore_ws = nullptr;
  size_t reseed_bytes = 0, explore_bytes = 0;
  // refinement pass: refined parameters, points and scores, best t per ray
  double *tref = nullptr, *Xref = nullptr, *lref = nullptr, *best_t = nullptr;
  Evaluator refe;
};

// The mixed bulk runs its contraction as split BF16 when d allows
// (SB_BULK_GEMM=f32 keeps the FP32 matrix-core kernel), for mixtures behind
// the screen (SB_MIX_SCREEN=0: the unscreened two stages; SB_MIX_TWO_STAGE=0:
// one stage over every component).
static bool bulk_split(const sb_loglik *ll, const RunCfg &rc) {
  const char *bg = getenv("SB_BULK_GEMM");
  return rc.precision == SB_PREC_MIXED && quad_gemm_bf16_ok(ll->d) && !(bg && bg[0] == 'f');
}
// SB_TILE2=BMxBN[xBK[xSTAGES]] forces the screened contraction's tile.
static TileCfg env_tile(const char *name, TileCfg t) {
  (void)parse_tile(getenv(name), &t);
  return t;
}
// The mixed bulk keeps its L-BFGS history ring in BF16 (SB_BULK_HIST=f32 keeps
// it in FP32): the ring is most of the step's traffic, and the pairs only
// shape the search direction, whose descent is checked and whose stop is the
// FP32 gradient test; the FP64 polish sets the final accuracy.
static bool bulk_hist_bf16(const RunCfg &rc) {
  const char *e = getenv("SB_BULK_HIST");
  return rc.precision == SB_PREC_MIXED && rc.m <= kMaxHist && !(e && e[0] == 'f');
}
static bool bulk_screen() {
  const char *e = getenv("SB_MIX_SCREEN");
  return !(e && e[0] == '0');
}
static bool bulk_two_stage(const sb_loglik *ll, const RunCfg &rc) {
  const char *ts = getenv("SB_MIX_TWO_STAGE");
  return bulk_split(ll, rc) && ll->family == SB_FAMILY_GAUSS_MIX && ll->K > 1 &&
         !(ts && ts[0] == '0');
}

static int carve_layout(Arena &ar, Layout &L, const sb_loglik *ll, const RunCfg &rc) {
  const int d = ll->d, K = ll->K;
  const int64_t B = rc.n_starts, R = rc.R, NP = (int64_t)rc.R * rc.n_pts;
  const bool mixed = rc.precision == SB_PREC_MIXED;
  const int ddt = mixed ? DT_BF16 : DT_F64;  // discovery dtype
  const int bdt = mixed ? DT_F32 : DT_F64;   // bulk dtype
  const size_t bes = (bdt == DT_F64) ? 8 : 4;
  L.Lprep = ar.take<double>((size_t)K * d * d);
  L.logdetP = ar.take<double>(K);
  L.beta = ar.take<double>(K);
  L.mx = ar.take<double>(K);
  L.info = ar.take<int32_t>(K);
  L.flags = ar.take<int32_t>(16);
  L.boxinfo = ar.take<double>(4);
  if (mixed) {
    L.P32 = ar.take<float>((size_t)K * d * d);
    L.Pbf = ar.take<bf16_t>((size_t)K * d * d);
    L.Plo = ar.take<bf16_t>((size_t)K * d * d);
    L.mu32 = ar.take<float>((size_t)K * d);
  }
  if (bulk_two_stage(ll, rc) && bulk_screen()) {
    L.rho = ar.take<double>(K);
    L.pw = ar.take<double>((size_t)2 * K * d + K);
    L.cinfo = ar.take<int32_t>(K);
  } else if (bulk_two_stage(ll, rc)) {
    L.Uhi = ar.take<bf16_t>((size_t)K * d * d);
    L.Ulo = ar.take<bf16_t>((size_t)K * d * d);
  }
  L.P0 = ar.take<double>((size_t)R * d);
  L.P1 = ar.take<double>((size_t)R * d);
  if (mixed) {
    L.P0f = ar.take<float>((size_t)R * d);
    L.P1f = ar.take<float>((size_t)R * d);
  }
  L.lpts = ar.take<char>((size_t)NP * (ddt == DT_F64 ? 8 : 4));
  L.best_l = ar.take<double>(R);
  L.best_j = ar.take<int32_t>(R);
  L.start_ray = ar.take<int32_t>(B);
  L.X0 = ar.take<double>((size_t)B * d);
  // discovery evaluator: no Y, qpart only
  L.disc.dtype = ddt;
  L.disc.cap = NP;
  {
    const size_t es = (ddt == DT_F64) ? 8 : 4;
    L.disc.qpart = ar.take<char>(es * (size_t)NP * K * ceil_div(d, 64));
    L.disc.Y = nullptr;
    L.disc.ldy = (int64_t)K * d;
  }
  // bulk
  L.lb.dtype = bdt;
  L.lb.hist_bf16 = bulk_hist_bf16(rc);
  L.lb.B = B;
  L.lb.d = d;
  L.lb.m = rc.m;
  if (lbfgs_carve(ar, L.lb)) return SB_E_NOMEM;
  L.bulk.dtype = bdt;
  L.bulk.cap = B;
  L.bulk.m.d = d;
  L.bulk.m.K = K;
  L.bulk.two_stage = bulk_two_stage(ll, rc);
  L.bulk.screen = L.bulk.two_stage && bulk_screen();
  if (L.bulk.carve(ar)) return SB_E_NOMEM;
  L.X0b = mixed ? (void *)ar.take<float>((size_t)B * d) : (void *)L.X0;
  L.Xend = ar.take<char>(bes * (size_t)B * d);
  L.lend = ar.take<double>((size_t)B);
  L.status = ar.take<int32_t>(B);
  L.counts = ar.take<int32_t>(8);
  L.valid = ar.take<uint8_t>(B);
  L.rep_of = ar.take<int32_t>(B);
  L.reps = ar.take<int32_t>(rc.cap_pre);
  // polish chunk
  const int PC = rc.polish_chunk;
  L.pol.dtype = DT_F64;
  L.pol.cap = PC;
  L.pol.m.d = d;
  L.pol.m.K = K;
  if (L.pol.carve(ar)) return SB_E_NOMEM;
  L.Xp = ar.take<double>((size_t)PC * d);
  L.lp = ar.take<double>(PC);
  L.Gp = ar.take<double>((size_t)PC * d);
  L.auxp = ar.take<double>((size_t)PC * K);
  L.H = ar.take<double>((size_t)PC * d * d);
  L.dx = ar.take<double>((size_t)PC * d);
  L.ldh = ar.take<double>(PC);
  L.pinfo = ar.take<int32_t>(PC);
  L.done = ar.take<int32_t>(PC);
  L.rejected = ar.take<int32_t>(PC);
  L.nact = ar.take<int32_t>(4);
  L.okp = ar.take<uint8_t>(PC);
  const int CA = rc.cap_pre;
  L.XA = ar.take<double>((size_t)CA * d);
  L.lA = ar.take<double>(CA);
  L.ldhA = ar.take<double>(CA);
  L.okA = ar.take<uint8_t>(CA);
  L.rep2 = ar.take<int32_t>(CA);
  L.rep2_of = ar.take<int32_t>(CA);
  L.Xm = ar.take<double>((size_t)CA * d);
  L.lm = ar.take<double>(CA);
  L.ldm = ar.take<double>(CA);
  L.mlz = ar.take<double>(CA);
  L.logz = ar.take<double>(4);
  L.order = ar.take<int32_t>(CA);
  L.Xs = ar.take<double>((size_t)CA * d);
  L.ls_ = ar.take<double>(CA);
  L.lds = ar.take<double>(CA);
  void *dd = ar.take<char>(dedup_ws_bytes(0) * 2);
  L.dedup_ar = Arena(dd, dedup_ws_bytes(0) * 2);
  if (ar.measure) L.dedup_ar.measure = true;
  if (rc.cyc) {
    const sb_chisao_config &cc = rc.cc;
    L.cactive = ar.take<uint8_t>(B);
    L.cstuck = ar.take<uint8_t>(B);
    L.cconv = ar.take<uint8_t>(B);
    L.cfrozen = ar.take<uint8_t>(B);
    L.clmask = ar.take<double>(B);
    L.Gend = ar.take<double>((size_t)B * d);
    L.U = ar.take<double>((size_t)B * d);
    L.Xo = ar.take<double>((size_t)B * d);
    L.sd = ar.take<double>(d);
    L.crep_of = ar.take<int32_t>(B);
    L.creps = ar.take<int32_t>(B);
    L.clist = ar.take<int32_t>((size_t)4 * B);
    L.Z = ar.take<double>((size_t)std::max(cc.n_cloud, 1) * cc.n_smooth * B * d);
    L.reseed_bytes = sb_chisao_reseed_workspace_bytes(d, K, B, cc.n_reseed_pts);
    L.reseed_ws = ar.take<char>(L.reseed_bytes);
    L.explore_bytes = sb_chisao_explore_workspace_bytes(d, K, B, cc.n_smooth);
    L.explore_ws = ar.take<char>(L.explore_bytes);
    if (cc.n_ref > 0) {
      const int64_t NR = R * cc.n_ref;
      L.tref = ar.take<double>(NR);
      L.Xref = ar.take<double>((size_t)NR * d);
      L.lref = ar.take<double>(NR);
      L.best_t = ar.take<double>(R);
      L.refe.dtype = DT_F64;
      L.refe.cap = NR;
      L.refe.m.d = d;
      L.refe.m.K = K;
      L.refe.qpart = ar.take<char>(8 * (size_t)NR * K * ceil_div(d, 64));
      L.refe.Y = nullptr;
      L.refe.ldy = (int64_t)K * d;
    }
  }
  return ar.ok() ? SB_OK : SB_E_NOMEM;
}

size_t evidence_ws_bytes(const sb_loglik *ll, const sb_config *cfg, const sb_chisao_config *cc) {
  RunCfg rc = resolve(ll, cfg, cc);
  Arena ar(nullptr, 0);
  Layout L;
  carve_layout(ar, L, ll, rc);
  return ar.off + 4096;
}

// ------------------------------------------------------------ the path

// The executable graph of an iteration block for `key`: a cached one, or
// the block captured from `record` and written into the least recently used
// slot (updated in place when the slot's executable accepts it, else
// instantiated anew).  nullptr on failure (error set).
template <typename F>
static hipGraphExec_t block_graph(ExecCtx *ex, const BlockKey &key, hipStream_t s, F record,
                                  int *st) {
  ExecCtx::Slot *hit = nullptr, *victim = &ex->slot[0];
  for (int i = 0; i < ExecCtx::kSlots; ++i) {
    ExecCtx::Slot &sl = ex->slot[i];
    if (sl.used && memcmp(&sl.key, &key, sizeof(BlockKey)) == 0) hit = &sl;
    if (!sl.used || (victim->used && sl.last < victim->last)) victim = &sl;
  }
  if (hit) {
    hit->last = ++ex->tick;
    return hit->exec;
  }
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("graph capture could not begin");
    *st = SB_E_DEVICE;
    return nullptr;
  }
  const int r = record();
  hipGraph_t graph = nullptr;
  const hipError_t e1 = hipStreamEndCapture(s, &graph);
  if (r || e1 != hipSuccess) {
    set_error("graph capture failed (%d, %s)", r, hipGetErrorString(e1));
    if (graph) (void)hipGraphDestroy(graph);
    *st = r ? r : SB_E_DEVICE;
    return nullptr;
  }
  ++ex->n_capture;
  bool ok = false;
  if (victim->exec) {
    hipGraphNode_t bad_node = nullptr;
    hipGraphExecUpdateResult ur;
    ok = hipGraphExecUpdate(victim->exec, graph, &bad_node, &ur) == hipSuccess &&
         ur == hipGraphExecUpdateSuccess;
    (void)hipGetLastError();
    if (ok) {
      ++ex->n_update;
    } else {
      (void)hipGraphExecDestroy(victim->exec);
      victim->exec = nullptr;
    }
  }
  if (!ok) {
    if (hipGraphInstantiate(&victim->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      victim->exec = nullptr;
      victim->used = false;
      (void)hipGraphDestroy(graph);
      set_error("graph instantiate failed");
      *st = SB_E_DEVICE;
      return nullptr;
    }
    ++ex->n_instantiate;
  }
  (void)hipGraphDestroy(graph);
  victim->used = true;
  victim->key = key;
  victim->last = ++ex->tick;
  return victim->exec;
}

// Bulk L-BFGS over all starts in dtype of lb; X0 in that dtype.  With an
// execution context (and a stream that can be captured) the iteration blocks
// run as its graph for `key`; without one they are launched directly.
static int run_bulk(Layout &L, const RunCfg &rc, double tol, hipStream_t s,
                    int64_t *evals_out, int *steps_out, ExecCtx *ex, const BlockKey &key,
                    const uint8_t *active = nullptr, void *grad_out = nullptr) {
  LbfgsBuffers &lb = L.lb;
  Evaluator &ev = L.bulk;
  int st = launch_lbfgs_init(lb, L.X0b, s);
  if (st) return st;
  // empty slots of the ChiSao cycle: dead from the start
  if (active && (st = launch_mask_dead(lb.B, active, lb.status, s))) return st;
  if (ev.screen) {  // no reference points yet: the first evaluation of every row takes all K
    if ((st = launch_fill_i32(ev.nstate, 0, ev.hasref, s))) return st;
  }
  const int d = lb.d;
  // initial evaluation of every start (slot 0, rows 0..B-1)
  ASrc a0;
  a0.kind = 0;
  a0.X = lb.X;
  a0.ldx = d;
  st = ev.run(a0, lb.B, nullptr, lb.F, lb.G, d, nullptr, nullptr, true, s);
  if (st) return st;
  ASrc at;
  at.kind = 0;
  at.X = lb.X;
  at.ldx = d;
  at.rowmap = lb.idx;
  at.rows = 2 * lb.B;  // both slots
  auto one_step = [&]() -> int {
    int r = launch_lbfgs_step(lb, rc.max_iter, tol, s);
    if (r) return r;
    r = launch_compact(lb, s);
    if (r) return r;
    return ev.run(at, lb.B, lb.count, lb.F, lb.G, d, lb.idx, nullptr, true, s);
  };
  // the per-block active count lands in pinned memory of the context, else
  // in a host stack word (the copy then completes before the synchronise)
  int32_t hstack[4] = {0, 0, 0, 0};
  int32_t *hcount = ex ? ex->pinned : hstack;
  const bool graphs = ex && rc.use_graph && s != nullptr;
  hipGraphExec_t exec = nullptr;
  int steps = 0;
  const int max_steps = 42 * rc.max_iter + 64;
  int rc_st = SB_OK;
  while (steps < max_steps) {
    if (graphs) {
      if (!exec) {
        int r = SB_OK;
        exec = block_graph(ex, key, s, [&]() -> int {
          int q = SB_OK;
          for (int k = 0; k < rc.blk && q == SB_OK; ++k) q = one_step();
          return q;
        }, &r);
        if (!exec) {
          rc_st = r ? r : SB_E_DEVICE;
          break;
        }
      }
      if (hipGraphLaunch(exec, s) != hipSuccess) {
        set_error("graph launch failed");
        rc_st = SB_E_DEVICE;
        break;
      }
      ++ex->n_launch;
    } else {
      int r = SB_OK;
      for (int k = 0; k < rc.blk && r == SB_OK; ++k) r = one_step();
      if (r) {
        rc_st = r;
        break;
      }
    }
    steps += rc.blk;
    if (hipMemcpyAsync(hcount, lb.count, sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("count readback failed: %s", hipGetErrorString(hipGetLastError()));
      rc_st = SB_E_DEVICE;
      break;
    }
    if (hcount[0] == 0) break;
  }
  int64_t ev_h = 0;
  if (rc_st == SB_OK) {
    if (hipMemcpyAsync(&ev_h, lb.evals, sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc_st = SB_E_DEVICE;
  }
  *evals_out = ev_h;
  *steps_out = steps;
  if (rc_st) return rc_st;
  return launch_lbfgs_gather(lb, L.Xend, L.lend, true, grad_out, L.status, nullptr, s);
}

// FP64 Newton polish + final Hessian/Cholesky/filters for reps [c0, c0+n).
static int polish_chunk(Layout &L, const Model &m64, const DevProblem &P, int n, hipStream_t s,
                        int64_t *grad_evals, int64_t *hess_evals) {
  const int d = m64.d, K = m64.K;
  Evaluator &ev = L.pol;
  ev.m = m64;
  ev.dtype = DT_F64;
  ASrc a;
  a.kind = 0;
  a.X = L.Xp;
  a.ldx = d;
  {
    TuneProbe pr;
    pr.a = a;
    pr.o.Y = ev.Y;
    pr.o.ldy = (int64_t)K * d;
    pr.o.qpart = ev.qpart;
    ev.tile = autotune_tiles(DT_F64, m64, n, s, &pr);
  }
  int st;
  if ((st = launch_fill_i32(n, 0, L.done, s))) return st;
  if ((st = launch_fill_i32(n, 0, L.rejected, s))) return st;
  int32_t nact_h = 0;
  for (int it = 0; it < 20; ++it) {
    if ((st = ev.run(a, n, nullptr, L.lp, L.Gp, d, nullptr, L.auxp, true, s))) return st;
    *grad_evals += n;
    if ((st = launch_hessian_assemble(m64, n, (const double *)ev.Y, ev.ldy, L.auxp, L.Gp, L.H, s)))
      return st;
    *hess_evals += n;
    if ((st = chol_batched(n, d, L.H, L.H, L.pinfo, s))) return st;
    if ((st = launch_chol_solve(n, d, L.H, L.Gp, L.dx, L.pinfo, s))) return st;
    if ((st = launch_fill_i32(1, 0, L.nact, s))) return st;
    hipLaunchKernelGGL(newton_update_kernel, dim3(n), dim3(256), 0, s, d, L.Xp, L.dx, L.pinfo,
                       L.done, L.rejected, L.nact);
    SB_LAUNCH_CHECK();
    SB_HIP(hipMemcpyAsync(&nact_h, L.nact, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
    if (nact_h == 0) break;
  }
  // final point: l, grad, Hessian, Cholesky, log det, filters
  if ((st = ev.run(a, n, nullptr, L.lp, L.Gp, d, nullptr, L.auxp, true, s))) return st;
  *grad_evals += n;
  if ((st = launch_hessian_assemble(m64, n, (const double *)ev.Y, ev.ldy, L.auxp, L.Gp, L.H, s)))
    return st;
  *hess_evals += n;
  if ((st = chol_batched(n, d, L.H, L.H, L.pinfo, s))) return st;
  if ((st = launch_logdet(n, d, L.H, L.pinfo, L.ldh, s))) return st;
  hipLaunchKernelGGL(filter_kernel, dim3(n), dim3(256), 0, s, d, L.Xp, L.lp, L.Gp, P.lo, P.hi,
                     L.rejected, L.pinfo, L.okp, L.counts + 4);
  SB_LAUNCH_CHECK();
  (void)K;
  return SB_OK;
}

// The ChiSao oscillation cycle over the n_starts slots, FP64, from the start
// points in L.X0 (section "ChiSao Exploration"; the steps and readings are
// those of sb_evidence_chisao_dev).  Leaves the last convergence phase's end
// points, l and statuses in L.Xend, L.lend, L.status (empty slots dead) for
// the tail of the path.  Host bookkeeping per oscillation: the slots' stuck,
// converged and representative flags are read back, the lost / unconverged /
// peak lists formed in slot order and uploaded as index lists.
static int run_cycle(Layout &L, const RunCfg &rc, const Model &m64, const DevProblem &P,
                     double tol, hipStream_t s, int64_t *bulk_evals, int *steps,
                     int64_t *grad_evals, int64_t *logl_evals, const BlockKey &key) {
  const sb_chisao_config &cc = rc.cc;
  const int64_t B = rc.n_starts;
  const int d = m64.d;
  int st;
  RunCfg rconv = rc;
  rconv.max_iter = cc.n_conv;
  sb_model_dev md;
  md.family = m64.family;
  md.norm = m64.norm;
  md.d = d;
  md.K = m64.K;
  md.log_w = P.log_w;
  md.mu = P.mu;
  md.prec = P.prec;
  md.nu = P.nu;
  md.logl_offset = P.c;
  md.beta = m64.beta;
  md.prec_lp = nullptr;
  md.mu_lp = nullptr;
  std::vector<uint8_t> act(B, 1), stk(B), cnv(B);
  std::vector<int32_t> rep_of(B), reps(B), lst;
  SB_HIP(hipMemcpyAsync(L.cactive, act.data(), B, hipMemcpyHostToDevice, s));
  bool gr_enabled = true, gr_used = false;
  int prev_found = -1;
  for (int k = 0; k < cc.n_osc; ++k) {
    const bool last = k == cc.n_osc - 1;
    // 1. convergence phase from the slots' points (fresh history)
    int64_t ev = 0;
    int stp = 0;
    if ((st = run_bulk(L, rconv, tol, s, &ev, &stp, nullptr, key, L.cactive, L.Gend))) return st;
    *bulk_evals += ev;
    *steps += stp;
    // 2. stick detection over the active slots
    if ((st = launch_cycle_flags(B, L.cactive, L.status, (const double *)L.lend, L.cconv,
                                 L.clmask, s)))
      return st;
    if ((st = sb_chisao_stick_dev(B, d, L.clmask, L.Gend, cc.stick_tol, L.cstuck, L.sd,
                                  sizeof(double) * d, s)))
      return st;
    // 3. dedup of the stuck slots; the converged slots' distinct peaks
    int npk = 0, nfound = 0;
    Arena ar3(L.dedup_ar.base, L.dedup_ar.cap);
    if ((st = dedup_run((int)B, d, L.Xend, DT_F64, L.lend, DT_F64, L.cstuck, rc.dedup_tol_pre,
                        L.crep_of, L.creps, (int)B, &npk, ar3, s)))
      return st;
    SB_HIP(hipMemcpyAsync(stk.data(), L.cstuck, B, hipMemcpyDeviceToHost, s));
    SB_HIP(hipMemcpyAsync(cnv.data(), L.cconv, B, hipMemcpyDeviceToHost, s));
    SB_HIP(hipMemcpyAsync(rep_of.data(), L.crep_of, sizeof(int32_t) * B, hipMemcpyDeviceToHost,
                          s));
    SB_HIP(hipMemcpyAsync(reps.data(), L.creps, sizeof(int32_t) * std::max(npk, 1),
                          hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
    Arena ar4(L.dedup_ar.base, L.dedup_ar.cap);
    if ((st = dedup_run((int)B, d, L.Xend, DT_F64, L.lend, DT_F64, L.cconv, rc.dedup_tol_pre,
                        L.crep_of, L.clist, (int)B, &nfound, ar4, s)))
      return st;
    if (gr_used && nfound <= prev_found) gr_enabled = false;
    gr_used = false;
    prev_found = nfound;
    std::vector<int32_t> lost;
    for (int64_t b = 0; b < B; ++b)
      if (stk[b] && rep_of[b] != (int32_t)b) lost.push_back((int32_t)b);
    for (int32_t b : lost) {
      act[b] = 0;
      stk[b] = 0;
    }
    // 4. reseeding
    const uint32_t base = 16u + 8u * (uint32_t)k;
    int kind = 0;
    const int64_t nl = (int64_t)lost.size();
    if (!last && nl > 0) {
      std::vector<int32_t> unc;
      for (int64_t b = 0; b < B; ++b)
        if (act[b] && !cnv[b]) unc.push_back((int32_t)b);
      std::vector<int32_t> slot, orig, coff, ccnt;
      if (unc.size() >= 5) {
        kind = 1;  // Repulse Monkey
        for (int64_t j = 0; j < nl; ++j) {
          slot.push_back(lost[j]);
          orig.push_back(unc[j % (int64_t)unc.size()]);
        }
      } else if (gr_enabled && npk > 0) {
        kind = 2;  // Golden Rooster
        gr_used = true;
        for (int p = 0; p < npk; ++p) {
          std::vector<int32_t> mine;
          for (int64_t j = p; j < nl; j += npk) mine.push_back(lost[j]);
          for (size_t c0 = 0; c0 < mine.size(); c0 += (size_t)d) {
            const size_t c1 = std::min(mine.size(), c0 + (size_t)d);
            coff.push_back((int32_t)slot.size());
            ccnt.push_back((int32_t)(c1 - c0));
            for (size_t q = c0; q < c1; ++q) {
              slot.push_back(mine[q]);
              orig.push_back(reps[p]);
            }
          }
        }
      }
      if (kind) {
        const int64_t n = (int64_t)slot.size();
        int32_t *dslot = L.clist, *dorig = L.clist + B, *doff = L.clist + 2 * B,
                *dcnt = L.clist + 3 * B;
        SB_HIP(hipMemcpyAsync(dslot, slot.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        SB_HIP(hipMemcpyAsync(dorig, orig.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        if ((st = launch_normal_rows(rc.seed, 0u, kind == 1 ? base : base + 2u, n, d, dslot, 0u,
                                     L.U, d, s)))
          return st;
        if (kind == 1) {
          if ((st = launch_normalize_rows(n, d, L.U, s))) return st;
        } else {
          const int nc = (int)coff.size();
          SB_HIP(hipMemcpyAsync(doff, coff.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice,
                                s));
          SB_HIP(hipMemcpyAsync(dcnt, ccnt.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice,
                                s));
          if ((st = launch_mgs_chunks(nc, d, doff, dcnt, L.U, s))) return st;
        }
        if ((st = launch_gather_idx(n, d, dorig, (const double *)L.Xend, L.Xo, s))) return st;
        if ((st = sb_chisao_reseed_dev(&md, P.lo, P.hi, n, L.Xo, L.U, cc.n_reseed_pts, nullptr,
                                       L.reseed_ws, L.reseed_bytes, s)))
          return st;
        *logl_evals += n * cc.n_reseed_pts;
        if ((st = launch_scatter_idx(n, d, dslot, L.Xo, (double *)L.Xend, s))) return st;
        for (int32_t b : lost) act[b] = 1;
        // the upload of the host lists must finish before they are reused
        SB_HIP(hipStreamSynchronize(s));
      }
    }
    SB_HIP(hipMemcpyAsync(L.cactive, act.data(), B, hipMemcpyHostToDevice, s));
    SB_HIP(hipStreamSynchronize(s));
    if (last) {
      // the last dedup's lost duplicates leave the candidates
      if ((st = launch_mask_dead(B, L.cactive, L.status, s))) return st;
      break;
    }
    // 5. Hands Like Clouds and anti-convergence of the free slots
    std::vector<uint8_t> frz(B);
    int64_t nfree = 0;
    for (int64_t b = 0; b < B; ++b) {
      const bool fr = act[b] && !stk[b];
      frz[b] = fr ? 0 : 1;
      nfree += fr ? 1 : 0;
    }
    SB_HIP(hipMemcpyAsync(L.cfrozen, frz.data(), B, hipMemcpyHostToDevice, s));
    double sigma = cc.sigma;
    if (!(sigma > 0)) {
      sigma = 0.0;
      if (nfree >= 2) {
        // the free flags: 1 - frozen, formed on the host beside it
        std::vector<uint8_t> fre(B);
        for (int64_t b = 0; b < B; ++b) fre[b] = (uint8_t)(1 - frz[b]);
        SB_HIP(hipMemcpyAsync(L.cconv, fre.data(), B, hipMemcpyHostToDevice, s));
        if ((st = launch_coord_spread(B, d, (const double *)L.Xend, L.cconv, L.sd, s))) return st;
        std::vector<double> sdh(d);
        SB_HIP(hipMemcpyAsync(sdh.data(), L.sd, sizeof(double) * d, hipMemcpyDeviceToHost, s));
        SB_HIP(hipStreamSynchronize(s));
        std::sort(sdh.begin(), sdh.end());
        const double med = (d % 2) ? sdh[d / 2] : 0.5 * (sdh[d / 2 - 1] + sdh[d / 2]);
        sigma = 0.5 * med;
      }
    }
    for (int c = 0; c < cc.n_cloud; ++c)
      for (int q = 0; q < cc.n_smooth; ++q) {
        const uint32_t i0 = (uint32_t)((c * cc.n_smooth + q) * d);
        if ((st = launch_normal_rows(rc.seed, 0u, base + 4u, B, d, nullptr, i0,
                                     L.Z + ((size_t)c * cc.n_smooth + q) * B * d, d, s)))
          return st;
      }
    if ((st = sb_chisao_explore_dev(&md, P.lo, P.hi, B, (double *)L.Xend, L.cfrozen, cc.n_cloud,
                                    cc.n_smooth, L.Z, sigma, cc.alpha_cloud, cc.n_anti,
                                    cc.alpha_anti, cc.momentum, L.explore_ws, L.explore_bytes,
                                    s)))
      return st;
    *grad_evals += B * ((int64_t)cc.n_cloud * cc.n_smooth + cc.n_anti);
    // the moved points start the next convergence phase
    SB_HIP(hipMemcpyAsync(L.X0, L.Xend, sizeof(double) * B * d, hipMemcpyDeviceToDevice, s));
    SB_HIP(hipStreamSynchronize(s));
  }
  return SB_OK;
}

int run_evidence(const DevProblem &P, const sb_config *cfg, sb_result *res, void *ws,
                 size_t ws_bytes, hipStream_t s, ExecCtx *ex, const sb_chisao_config *cc) {
  const auto t_start = std::chrono::steady_clock::now();
  sb_loglik llh;
  llh.family = P.family;
  llh.norm = P.norm;
  llh.d = P.d;
  llh.K = P.K;
  RunCfg rc = resolve(&llh, cfg, cc);
  const int d = P.d, K = P.K;
  const bool mixed = rc.precision == SB_PREC_MIXED;
  Arena ar(ws, ws_bytes);
  Layout L;
  if (carve_layout(ar, L, &llh, rc) != SB_OK || !ws) {
    set_error("workspace too small: need %zu bytes", evidence_ws_bytes(&llh, cfg, cc));
    return SB_E_NOMEM;
  }
  Timer tm;
  tm.init(ex);
  tm.mark(s);  // 0
  int st;
  // ---------------- A1 prep
  Model m64;
  m64.family = P.family;
  m64.norm = P.norm;
  m64.d = d;
  m64.K = K;
  m64.mu64 = P.mu;
  m64.P64 = P.prec;
  m64.beta = L.beta;
  m64.nu = P.nu;
  m64.c = P.c;
  if ((st = launch_fill_i32(16, 0, L.flags, s))) return st;
  hipLaunchKernelGGL(box_info_kernel, dim3(1), dim3(256), 0, s, d, P.lo, P.hi, L.boxinfo);
  SB_LAUNCH_CHECK();
  if ((st = launch_symmetry_check(P.prec, K, d, L.mx, L.flags, s))) return st;
  if ((st = chol_batched(K, d, P.prec, L.Lprep, L.info, s))) return st;
  if ((st = launch_logdet(K, d, L.Lprep, L.info, L.logdetP, s))) return st;
  if ((st = launch_beta(m64, P.log_w, L.logdetP, L.beta, s))) return st;
  if (mixed) {
    if ((st = launch_convert_model(m64, L.P32, L.Pbf, L.mu32, s))) return st;
    if ((st = launch_split_bf16((int64_t)K * d * d, P.prec, L.Pbf, L.Plo, s))) return st;
    if (L.Uhi && (st = launch_split_upper(K, d, L.Lprep, L.Uhi, L.Ulo, s))) return st;
    if (L.rho) {
      // sigma_k^2: the Gershgorin bound, tightened by a certified power
      // estimate where the polish's Hessian scratch holds the K shifted
      // matrices (SB_LMAX=0: Gershgorin only)
      if ((st = launch_row_abs_max(K, d, P.prec, L.rho, s))) return st;
      const char *e = getenv("SB_LMAX");
      if (rc.polish_chunk >= K && !(e && e[0] == '0') &&
          (st = launch_lmax_bound(K, d, P.prec, L.rho, L.pw, L.H, L.cinfo, s)))
        return st;
    }
  }
  {
    int32_t hflag[1];
    int32_t hinfo[kMaxComp];
    double hmx[kMaxComp], hbox[4];
    SB_HIP(hipMemcpyAsync(hflag, L.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SB_HIP(hipMemcpyAsync(hinfo, L.info, sizeof(int32_t) * K, hipMemcpyDeviceToHost, s));
    SB_HIP(hipMemcpyAsync(hmx, L.mx, sizeof(double) * K, hipMemcpyDeviceToHost, s));
    SB_HIP(hipMemcpyAsync(hbox, L.boxinfo, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
    if (hbox[0] != 0.0) {
      set_error("box: need finite lo_i < hi_i in every coordinate");
      res->log_z = NAN;
      return SB_E_INVAL;
    }
    if (hflag[0]) {
      set_error("precision matrix is not symmetric to 1e-12 relative");
      res->log_z = NAN;
      return SB_E_NOTPD;
    }
    for (int k = 0; k < K; ++k) {
      if (hinfo[k] != 0) {
        set_error("precision matrix %d is not positive definite (pivot %d)", k, hinfo[k]);
        res->log_z = NAN;
        return SB_E_NOTPD;
      }
      if (!std::isfinite(hmx[k])) {
        set_error("precision matrix %d has non-finite entries", k);
        res->log_z = NAN;
        return SB_E_INVAL;
      }
    }
    // FP32 bulk tolerance: its rounding floor 32 u32 max|P| (1 + max|theta|)
    double pmax = 0.0;
    for (int k = 0; k < K; ++k) pmax = std::max(pmax, hmx[k]);
    tm.mark(s);  // 1
    // ---------------- A2 discovery
    const int ddt = mixed ? DT_BF16 : DT_F64;
    if ((st = launch_rays(d, P.lo, P.hi, rc.R, rc.seed, 0u, L.P0, L.P1, L.P0f, L.P1f, s)))
      return st;
    Model md = m64;
    if (mixed) {
      md.mu32 = L.mu32;
      md.Plp = L.Pbf;
      md.Phi = L.Pbf;
    }
    L.disc.m = md;
    if (mixed && rc.n_pts > 3 && quad_gemm_bf16_ok(d)) {
      // the BF16 contraction at three nodes per ray, the samples by interpolation
      if ((st = discover_bf16_nodes(md, L.P0f, L.P1f, rc.R, rc.n_pts, (float *)L.disc.qpart,
                                    (float *)L.lpts, s)))
        return st;
    } else {
      ASrc a;
      a.kind = 1;
      a.P0 = mixed ? (const void *)L.P0f : (const void *)L.P0;
      a.P1 = mixed ? (const void *)L.P1f : (const void *)L.P1;
      a.n_pts = rc.n_pts;
      const int64_t NP = (int64_t)rc.R * rc.n_pts;
      TuneProbe pr;
      pr.a = a;
      pr.o.Y = nullptr;
      pr.o.ldy = L.disc.ldy;
      pr.o.qpart = L.disc.qpart;
      L.disc.tile = autotune_tiles(ddt, md, NP, s, &pr);
      if ((st = L.disc.run(a, NP, nullptr, L.lpts, nullptr, 0, nullptr, nullptr, false, s, false)))
        return st;
    }
    if (rc.cyc && rc.cc.n_ref > 0) {
      // refinement pass (FP64): points at the quantiles of the likelihood on
      // each ray's active cells, scored by the same contraction as rows
      const int nref = rc.cc.n_ref;
      const int64_t NR = (int64_t)rc.R * nref;
      if ((st = launch_refine_t(rc.R, rc.n_pts, nref, rc.cc.ref_delta, (const double *)L.lpts,
                                L.tref, s)))
        return st;
      if ((st = launch_refine_points(rc.R, nref, d, L.P0, L.P1, L.tref, L.Xref, s))) return st;
      ASrc a;
      a.kind = 0;
      a.X = L.Xref;
      a.ldx = d;
      L.refe.m = md;
      TuneProbe pr;
      pr.a = a;
      pr.o.Y = nullptr;
      pr.o.ldy = L.refe.ldy;
      pr.o.qpart = L.refe.qpart;
      L.refe.tile = autotune_tiles(DT_F64, md, NR, s, &pr);
      if ((st = L.refe.run(a, NR, nullptr, L.lref, nullptr, 0, nullptr, nullptr, false, s,
                           false)))
        return st;
      if ((st = launch_refine_best(rc.R, rc.n_pts, nref, (const double *)L.lpts, L.lref, L.tref,
                                   L.best_l, L.best_t, s)))
        return st;
      if ((st = launch_topn(rc.R, rc.n_starts, L.best_l, L.start_ray, s))) return st;
      if ((st = launch_gather_starts_t(d, rc.n_starts, L.start_ray, L.best_t, L.P0, L.P1, L.X0,
                                       s)))
        return st;
    } else {
      if ((st = launch_ray_argmax(rc.R, rc.n_pts, ddt, L.lpts, L.best_l, L.best_j, s)))
        return st;
      if ((st = launch_topn(rc.R, rc.n_starts, L.best_l, L.start_ray, s))) return st;
      if ((st = launch_gather_starts(d, rc.n_pts, rc.n_starts, L.start_ray, L.best_j, L.P0,
                                     L.P1, L.X0, s)))
        return st;
    }
    tm.mark(s);  // 2
    // ---------------- A3-A5 bulk L-BFGS
    Model mb = m64;
    double tol = rc.grad_tol > 0 ? rc.grad_tol : 1e-10;
    if (mixed) {
      mb.mu32 = L.mu32;
      mb.Plp = L.P32;
      mb.Phi = L.Pbf;
      mb.Plo = L.Plo;
      const double maxabs_theta = hbox[1];  // max_i max(|lo_i|, |hi_i|)
      tol = 32.0 * 5.9604644775390625e-08 * pmax * (1.0 + maxabs_theta);
      if (rc.grad_tol > 0) tol = std::max(tol, rc.grad_tol);
      if ((st = launch_cast_f64_f32((int64_t)rc.n_starts * d, L.X0, (float *)L.X0b, s)))
        return st;
    }
    L.bulk.m = mb;
    L.bulk.dtype = mixed ? DT_F32 : DT_F64;
    // mixed bulk: the contraction on the BF16 matrix cores with split operands
    const bool split = bulk_split(&llh, rc);
    L.bulk.gemm_dtype = split ? DT_F32S : -1;
    L.bulk.Uhi = L.Uhi;
    L.bulk.Ulo = L.Ulo;
    L.bulk.rho = L.rho;
    {
      TuneProbe pr;  // timed on the start points and the bulk's own scratch
      pr.a.kind = 0;
      pr.a.X = L.X0b;
      pr.a.ldx = d;
      pr.o.Y = L.bulk.Y;
      pr.o.ldy = L.bulk.ldy;
      pr.o.qpart = L.bulk.qpart;
      L.bulk.tile = autotune_tiles(split ? DT_F32S : L.bulk.dtype, mb, rc.n_starts, s, &pr);
      if (L.bulk.two_stage && !L.bulk.screen) {
        // stage 1 timed in its own mode; stage 2 multiplies about one component's share
        // of the rows per component, where 128 x 128 tiles keep every CU busy
        Model m1 = mb;
        m1.Phi = L.Uhi;
        m1.Plo = L.Ulo;
        TuneProbe p1 = pr;
        p1.o.Y = nullptr;
        p1.o.sumsq = true;
        L.bulk.tile1 = autotune_tiles(DT_F32S, m1, rc.n_starts, s, &p1);
        L.bulk.tile2 = TileCfg();
      } else if (L.bulk.screen) {
        // each component's list holds about its share of the rows: 128 x 128
        // tiles spread the uneven lists over every CU (256 x 256 measured slower)
        L.bulk.tile2 = env_tile("SB_TILE2", TileCfg());
      }
      L.bulk.grad_direct = split && K == 1 && P.family == SB_FAMILY_GAUSS_MIX;
    }
    int64_t bulk_evals = 0;
    int steps = 0;
    BlockKey key;
    memset(&key, 0, sizeof(key));
    key.stream = (void *)s;
    key.ws = ws;
    key.ws_bytes = ws_bytes;
    key.P = P;
    // field by field: the caller's padding bytes stay out of the key
    key.cfg.n_rays = cfg->n_rays;
    key.cfg.n_points = cfg->n_points;
    key.cfg.n_starts = cfg->n_starts;
    key.cfg.m = cfg->m;
    key.cfg.max_iter = cfg->max_iter;
    key.cfg.max_modes = cfg->max_modes;
    key.cfg.precision = cfg->precision;
    key.cfg.grad_tol = cfg->grad_tol;
    key.cfg.dedup_tol = cfg->dedup_tol;
    key.cfg.dedup_tol_pre = cfg->dedup_tol_pre;
    key.cfg.seed = cfg->seed;
    key.tol = tol;
    key.max_iter = rc.max_iter;
    key.blk = rc.blk;
    key.dtype = L.bulk.dtype;
    key.gemm_dtype = L.bulk.gemm_dtype;
    key.two_stage = L.bulk.two_stage;
    key.screen = L.bulk.screen;
    key.grad_direct = L.bulk.grad_direct;
    key.hist_bf16 = L.lb.hist_bf16;
    key.tile = L.bulk.tile;
    key.tile1 = L.bulk.tile1;
    key.tile2 = L.bulk.tile2;
    int64_t cyc_grad_evals = 0, cyc_logl_evals = 0;
    if (!rc.cyc) {
      if ((st = run_bulk(L, rc, tol, s, &bulk_evals, &steps, ex, key))) return st;
    } else if ((st = run_cycle(L, rc, m64, P, tol, s, &bulk_evals, &steps, &cyc_grad_evals,
                               &cyc_logl_evals, key))) {
      return st;
    }
    tm.mark(s);  // 3
    // ---------------- A7 pre-dedup
    const int64_t B = rc.n_starts;
    if ((st = launch_fill_i32(8, 0, L.counts, s))) return st;
    hipLaunchKernelGGL(candidate_flags_kernel<double>, dim3((unsigned)ceil_div(B, 256)),
                       dim3(256), 0, s, B, L.status, (const double *)L.lend, L.valid, L.counts);
    SB_LAUNCH_CHECK();
    int nrep = 0;
    st = dedup_run((int)B, d, L.Xend, L.lb.dtype, L.lend, DT_F64, L.valid, rc.dedup_tol_pre,
                   L.rep_of, L.reps, rc.cap_pre, &nrep, L.dedup_ar, s);
    if (st == SB_E_CAPACITY) {
      set_error("%d representatives after the pre-polish dedup exceed the polish capacity %d",
                nrep, rc.cap_pre);
      res->log_z = NAN;
      return SB_E_CAPACITY;
    }
    if (st) return st;
    tm.mark(s);  // 4
    // ---------------- A6 polish, A8/A9 Hessian + Cholesky, filters (chunks)
    int64_t pol_evals = 0, hess_evals = 0;
    for (int c0 = 0; c0 < nrep; c0 += rc.polish_chunk) {
      const int n = std::min(rc.polish_chunk, nrep - c0);
      if (mixed)
        hipLaunchKernelGGL(gather_reps_kernel<float>, dim3(n), dim3(256), 0, s, d, L.reps + c0,
                           (const float *)L.Xend, L.Xp);
      else
        hipLaunchKernelGGL(gather_reps_kernel<double>, dim3(n), dim3(256), 0, s, d, L.reps + c0,
                           (const double *)L.Xend, L.Xp);
      SB_LAUNCH_CHECK();
      if ((st = polish_chunk(L, m64, P, n, s, &pol_evals, &hess_evals))) return st;
      SB_HIP(hipMemcpyAsync(L.XA + (size_t)c0 * d, L.Xp, sizeof(double) * n * d,
                            hipMemcpyDeviceToDevice, s));
      SB_HIP(hipMemcpyAsync(L.lA + c0, L.lp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      SB_HIP(hipMemcpyAsync(L.ldhA + c0, L.ldh, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      SB_HIP(hipMemcpyAsync(L.okA + c0, L.okp, n, hipMemcpyDeviceToDevice, s));
    }
    tm.mark(s);  // 5
    // ---------------- A7 final dedup
    double tau = rc.dedup_tol;
    if (!(tau > 0)) tau = 1e-6 * hbox[2];  // max_i (hi_i - lo_i)
    Arena ar2(L.dedup_ar.base, L.dedup_ar.cap);
    int nm = 0;
    st = dedup_run(nrep, d, L.XA, DT_F64, L.lA, DT_F64, L.okA, tau, L.rep2_of, L.rep2,
                   rc.cap_pre, &nm, ar2, s);
    if (st && st != SB_E_CAPACITY) return st;
    // ---------------- A10 combine
    int32_t hcounts[8];
    SB_HIP(hipMemcpyAsync(hcounts, L.counts, sizeof(hcounts), hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
    res->n_logl_evals = (int64_t)rc.R * (rc.n_pts + (rc.cyc ? rc.cc.n_ref : 0)) + cyc_logl_evals;
    res->n_grad_evals = bulk_evals + pol_evals + cyc_grad_evals;
    res->n_hess_evals = hess_evals;
    res->iterations = steps;
    res->n_dead_starts = hcounts[0];
    res->n_candidates = hcounts[1];
    res->n_rejected_nonpd = hcounts[4];
    res->n_reps_pre = nrep;
    res->n_modes = nm;
    int ret = SB_OK;
    if (nm == 0) {
      res->log_z = -INFINITY;
      ret = SB_E_NOMODE;
    } else if (nm > rc.max_modes) {
      res->log_z = NAN;
      set_error("%d modes found, max_modes = %d", nm, rc.max_modes);
      ret = SB_E_CAPACITY;
    } else {
      hipLaunchKernelGGL(gather_rows_kernel, dim3(nm), dim3(256), 0, s, d, L.rep2, L.XA, L.Xm);
      hipLaunchKernelGGL(gather_scalars_kernel, dim3((unsigned)ceil_div(nm, 256)), dim3(256), 0,
                         s, nm, L.rep2, L.lA, L.ldhA, L.lm, L.ldm);
      SB_LAUNCH_CHECK();
      if ((st = launch_combine(nm, d, P.lo, P.hi, L.lm, L.ldm, L.Xm, L.order, L.mlz, L.logz, s)))
        return st;
      hipLaunchKernelGGL(gather_rows_kernel, dim3(nm), dim3(256), 0, s, d, L.order, L.Xm, L.Xs);
      hipLaunchKernelGGL(gather_scalars_kernel, dim3((unsigned)ceil_div(nm, 256)), dim3(256), 0,
                         s, nm, L.order, L.lm, L.ldm, L.ls_, L.lds);
      SB_LAUNCH_CHECK();
      tm.mark(s);  // 6
      SB_HIP(hipMemcpyAsync(&res->log_z, L.logz, sizeof(double), hipMemcpyDeviceToHost, s));
      if (res->modes)
        SB_HIP(hipMemcpyAsync(res->modes, L.Xs, sizeof(double) * nm * d, hipMemcpyDeviceToHost,
                              s));
      if (res->mode_log_z)
        SB_HIP(hipMemcpyAsync(res->mode_log_z, L.mlz, sizeof(double) * nm,
                              hipMemcpyDeviceToHost, s));
      if (res->mode_logl)
        SB_HIP(hipMemcpyAsync(res->mode_logl, L.ls_, sizeof(double) * nm, hipMemcpyDeviceToHost,
                              s));
      if (res->log_det_h)
        SB_HIP(hipMemcpyAsync(res->log_det_h, L.lds, sizeof(double) * nm, hipMemcpyDeviceToHost,
                              s));
      SB_HIP(hipStreamSynchronize(s));
    }
    const double total =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (int i = 0; i < 8; ++i) res->seconds[i] = 0.0;
    res->seconds[0] = tm.between(0, 1);
    res->seconds[1] = tm.between(1, 2);
    res->seconds[2] = tm.between(2, 3);
    res->seconds[3] = tm.between(3, 4);
    res->seconds[4] = tm.between(4, 5);
    res->seconds[5] = 0.0;  // Hessian + Cholesky run inside the polish batches
    res->seconds[6] = tm.between(5, 6);
    res->seconds[7] = total;
    return ret;
  }
}

}  // namespace sb
