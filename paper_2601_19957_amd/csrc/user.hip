// Generic user log-likelihoods without an analytic backward (the paper's
// default generality: any l, derivatives by finite differences; appendix
// "Gradient and Hessian Computation" and "Rotation Detection").
//
// The caller's HIP source defines
//   __device__ double NAME(const double *x, int d, const double *params);
// it is compiled at run time for gfx950 with hipRTC (packed FP32 instructions
// off, as for the library) together with a batched evaluation kernel, one
// thread per point.  Derivatives come from batches of perturbed points built
// by the library's own kernels: per base point x the rows
//   0             x
//   1 + 2i, 2+2i  x + eps e_i, x - eps e_i                (i < d)
//   1 + 2d, 2+2d  x + eps v, x - eps v, v = (1..1)/sqrt(d)  (rotation probe)
//   3 + 2d + 4t   x +- eps e_i +- eps e_j, t-th pair i < j  (full Hessian only)
// are evaluated in one launch, and a combine kernel forms the central
// differences: g_i = (f+ - f-)/(2 eps), H_ii = (f+ - 2 f0 + f-)/eps^2,
// H_ij = (f++ - f+- - f-+ + f--)/(4 eps^2), and the probe
// b = (v^T H v - mean H_ii)/(d - 1).
#include <hip/hiprtc.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

struct sb_user_fn {
  hipModule_t mod = nullptr;
  hipFunction_t eval = nullptr;
  int device = -1;
};

namespace sb {

static int64_t fd_rows(int d, bool full) {
  return 3 + 2ll * d + (full ? 2ll * d * (d - 1) : 0);
}

// Row r of base point b, written by one thread (d values).  No contraction
// into FMAs: each coordinate is x_i, x_i +- eps or x_i +- eps v_i, one rounding.
__global__ __launch_bounds__(256) void fd_points_kernel(int64_t B, int d, int64_t R,
                                                        const double *X, double eps, double *P) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= B * R) return;
  const int64_t b = e / R, r = e % R;
  const double *x = X + b * d;
  double *out = P + e * d;
  for (int j = 0; j < d; ++j) out[j] = x[j];
  if (r == 0) return;
  if (r <= 2ll * d) {
    const int i = (int)((r - 1) / 2);
    out[i] = ((r - 1) % 2 == 0) ? x[i] + eps : x[i] - eps;
    return;
  }
  if (r <= 2ll * d + 2) {
    const double vi = 1.0 / sqrt((double)d);
    const double step = eps * vi;
    for (int j = 0; j < d; ++j) out[j] = (r == 2ll * d + 1) ? x[j] + step : x[j] - step;
    return;
  }
  int64_t t = (r - 3 - 2ll * d) / 4;
  const int sgn = (int)((r - 3 - 2ll * d) % 4);  // ++, +-, -+, --
  int i = 0;
  while (t >= d - 1 - i) {
    t -= d - 1 - i;
    ++i;
  }
  const int j = i + 1 + (int)t;
  out[i] = (sgn < 2) ? x[i] + eps : x[i] - eps;
  out[j] = (sgn % 2 == 0) ? x[j] + eps : x[j] - eps;
}

// Thread per (base point, i): l, g_i, H_ii and, for i = 0, the probe.
__global__ __launch_bounds__(256) void fd_combine_kernel(int64_t B, int d, int64_t R,
                                                         const double *F, double eps, double *l,
                                                         double *g, double *hd, double *probe) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= B * d) return;
  const int64_t b = e / d;
  const int i = (int)(e % d);
  const double *f = F + b * R;
  const double f0 = f[0], fp = f[1 + 2 * i], fm = f[2 + 2 * i];
  if (g) g[e] = (fp - fm) / (2.0 * eps);
  const double hii = (fp - 2.0 * f0 + fm) / (eps * eps);
  if (hd) hd[e] = hii;
  if (i == 0) {
    if (l) l[b] = f0;
    if (probe) {
      double pb = 0.0;
      if (d > 1) {
        double a = 0.0;
        for (int k = 0; k < d; ++k)
          a += (f[1 + 2 * k] - 2.0 * f0 + f[2 + 2 * k]) / (eps * eps);
        a /= (double)d;
        const double vhv = (f[1 + 2 * d] - 2.0 * f0 + f[2 + 2 * d]) / (eps * eps);
        pb = (vhv - a) / (double)(d - 1);
      }
      probe[b] = pb;
    }
  }
}

// Thread per (base point, i, j): the full Hessian, diagonal from H_ii.
__global__ __launch_bounds__(256) void fd_hessian_kernel(int64_t B, int d, int64_t R,
                                                         const double *F, double eps, double *H) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= B * d * d) return;
  const int64_t b = e / ((int64_t)d * d);
  const int i = (int)((e / d) % d), j = (int)(e % d);
  const double *f = F + b * R;
  double h;
  if (i == j) {
    h = (f[1 + 2 * i] - 2.0 * f[0] + f[2 + 2 * i]) / (eps * eps);
  } else {
    const int p = i < j ? i : j, q = i < j ? j : i;
    // index of pair (p, q) among i < j in row-major order
    const int64_t t = (int64_t)p * (2 * d - p - 1) / 2 + (q - p - 1);
    const double *v = f + 3 + 2ll * d + 4 * t;
    h = (v[0] - v[1] - v[2] + v[3]) / (4.0 * eps * eps);
  }
  H[e] = h;
}

// Per mode: the rotation decision |b| > rot_tol |mean H_ii| (host), then the
// diagonal modes' log det(-H) = sum log(-H_ii) (NaN if some H_ii >= 0).
__global__ __launch_bounds__(256) void fd_diag_logdet_kernel(int n, int d, const double *hd,
                                                             const int32_t *full,
                                                             double *logdet) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n || full[k]) return;
  double s = 0.0;
  for (int i = 0; i < d; ++i) {
    const double h = -hd[(int64_t)k * d + i];
    s += h > 0.0 ? log(h) : (double)NAN;
  }
  logdet[k] = s;
}

// rows[i] = X[idx[i]] (d values each), thread per element
__global__ __launch_bounds__(256) void gather_rows_kernel(int m, int d, const int32_t *idx,
                                                          const double *X, double *out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)m * d) return;
  out[e] = X[(int64_t)idx[e / d] * d + e % d];
}

// A = -H (the factorisation wants the positive definite -grad^2 l)
__global__ __launch_bounds__(256) void negate_kernel(int64_t n, const double *H, double *A) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) A[e] = -H[e];
}

// logdet[idx[i]] = ld[i], or NaN where the factorisation failed
__global__ __launch_bounds__(256) void scatter_logdet_kernel(int m, const int32_t *idx,
                                                             const double *ld,
                                                             const int32_t *info,
                                                             double *logdet) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < m) logdet[idx[i]] = info[i] ? (double)NAN : ld[i];
}

// Ray point j of ray r, p + t (q - p) with t = (j + 1/2)/n_pts, written out
// for the user kernel (the same two-rounding expression as everywhere).
__global__ __launch_bounds__(256) void ray_points_kernel(int R, int n_pts, int d,
                                                         const double *P0, const double *P1,
                                                         double *X) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)R * n_pts * d) return;
  const int64_t row = e / d;
  const int j = (int)(e % d);
  const int64_t ray = row / n_pts;
  const int jj = (int)(row % n_pts);
  const double t = ((double)jj + 0.5) / (double)n_pts;
  const double p = P0[ray * d + j], q = P1[ray * d + j];
  X[e] = p + t * (q - p);
}

// The L-BFGS rows listed in idx [count] (row r = slot * B + start) gathered
// from the state's points, and their l and gradient scattered back.
__global__ __launch_bounds__(256) void gather_state_rows_kernel(int count, int d,
                                                                const int32_t *idx,
                                                                const double *X, double *out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)count * d) return;
  out[e] = X[(int64_t)idx[e / d] * d + e % d];
}

__global__ __launch_bounds__(256) void scatter_state_rows_kernel(int count, int d,
                                                                 const int32_t *idx,
                                                                 const double *l, const double *g,
                                                                 double *F, double *G) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)count * d) return;
  const int64_t i = e / d;
  const int64_t r = idx[i];
  G[r * d + e % d] = g[e];
  if (e % d == 0) F[r] = l[i];
}

// ------------------------------------------------------------ TrajectoryBank
//
// Step 1 of BendTheBow's geometry detection (section "Automatic Geometry
// Detection"; appendix "Rotation Detection"): GreenDragon's seeds of each
// mode, theta* +- 0.9 w_i e_i with w_i = 1/sqrt(-H_ii) (seed 2i: +, 2i + 1:
// -), run batched L-BFGS on FD gradients; after every batch step each seed's
// newly accepted point (its iteration count advanced) closes a step of its
// trajectory, whose perpendicular fraction in coordinates whitened by
// sqrt(-H_ii) is folded into the seed's maximum.  A step counts while the
// whitened gradient at its start is at least rel_floor of the seed's first.
// The positions and gradients are also written to a caller's bank when one is
// given.

__global__ __launch_bounds__(256) void gd_seeds_kernel(int d, const double *modes,
                                                       const double *hdiag, double *X0) {
#pragma clang fp contract(off)
  const int64_t row = blockIdx.x;
  const int64_t k = row / (2 * d);
  const int j = (int)(row % (2 * d)), i = j / 2;
  for (int c = threadIdx.x; c < d; c += 256) {
    double x = modes[k * d + c];
    if (c == i) {
      const double w = 1.0 / sqrt(-hdiag[k * d + i]);
      x = (j & 1) ? x - 0.9 * w : x + 0.9 * w;
    }
    X0[row * d + c] = x;
  }
}

__global__ __launch_bounds__(256) void traj_step_kernel(
    int64_t S, int d, int n_max, const double *X, const double *G, const int32_t *cur,
    const int32_t *iters, const double *hdiag, double rel_floor, double *xprev, double *gprev,
    int32_t *tprev, double *g0w, double *fmx, int32_t *nct, double *Xbank, double *Gbank,
    int32_t *blen) {
  __shared__ double red[4];
  const int64_t s = blockIdx.x;
  const int64_t k = s / (2 * d);
  const int t = iters[s], tp = tprev[s];
  const int64_t row = (int64_t)cur[s] * S + s;
  const double *x = X + row * d, *g = G + row * d, *hd = hdiag + k * d;
  double *xp = xprev + s * d, *gp = gprev + s * d;
  if (tp >= 0 && t <= tp) return;  // no new accepted point
  if (tp >= 0) {
    // the step from the previous point to this one
    double a = 0.0;
    for (int i = threadIdx.x; i < d; i += 256) {
      const double gw = gp[i] / sqrt(-hd[i]);
      a += gw * gw;
    }
    const double gg = block_sum<256>(a, red);
    const double g0 = g0w[s];
    if (g0 > 0.0 && sqrt(gg) >= rel_floor * g0) {
      double b = 0.0, c = 0.0;
      for (int i = threadIdx.x; i < d; i += 256) {
        const double sh = sqrt(-hd[i]);
        const double du = sh * (x[i] - xp[i]), gw = gp[i] / sh;
        b += du * gw;
        c += du * du;
      }
      const double dg = block_sum<256>(b, red);
      const double dd = block_sum<256>(c, red);
      if (dd > 0.0) {
        const double coef = dg / gg;
        double e = 0.0;
        for (int i = threadIdx.x; i < d; i += 256) {
          const double sh = sqrt(-hd[i]);
          const double pr = sh * (x[i] - xp[i]) - coef * (gp[i] / sh);
          e += pr * pr;
        }
        const double pp = block_sum<256>(e, red);
        if (threadIdx.x == 0) {
          fmx[s] = fmax(fmx[s], sqrt(pp) / sqrt(dd));
          nct[s] += 1;
        }
      }
    }
  } else {
    double a = 0.0;
    for (int i = threadIdx.x; i < d; i += 256) {
      const double gw = g[i] / sqrt(-hd[i]);
      a += gw * gw;
    }
    const double n0 = sqrt(block_sum<256>(a, red));
    if (threadIdx.x == 0) g0w[s] = n0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < d; i += 256) {
    xp[i] = x[i];
    gp[i] = g[i];
  }
  if (Xbank && t <= n_max)
    for (int i = threadIdx.x; i < d; i += 256) {
      Xbank[(s * (n_max + 1) + t) * d + i] = x[i];
      Gbank[(s * (n_max + 1) + t) * d + i] = g[i];
    }
  if (threadIdx.x == 0) {
    tprev[s] = t;
    if (blen) blen[s] = t + 1;
  }
}

__global__ void traj_init_kernel(int64_t S, int32_t *tprev, double *fmx, int32_t *nct) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  tprev[s] = -1;
  fmx[s] = 0.0;
  nct[s] = 0;
}

// f_perp of mode k: the largest seed maximum over its 2d seeds that counted a
// step; NaN when none did.
__global__ void traj_mode_kernel(int n, int d, const double *fmx, const int32_t *nct,
                                 double *fperp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double m = 0.0;
  bool any = false;
  for (int j = 0; j < 2 * d; ++j) {
    const int64_t s = (int64_t)k * 2 * d + j;
    if (nct[s] > 0) {
      any = true;
      m = fmax(m, fmx[s]);
    }
  }
  fperp[k] = any ? m : (double)NAN;
}

__global__ void iota_kernel(int64_t n, int32_t *idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) idx[i] = (int32_t)i;
}

struct TrajBuffers {
  int64_t S = 0;
  LbfgsBuffers lb;
  double *X0 = nullptr, *Xg = nullptr, *lg = nullptr, *gg = nullptr;
  double *xprev = nullptr, *gprev = nullptr, *g0w = nullptr, *fmax = nullptr;
  int32_t *tprev = nullptr, *nct = nullptr, *all = nullptr;
  double *fperp = nullptr;  // [n] per-mode result when the caller keeps none
  void *fd_ws = nullptr;
  size_t fd_bytes = 0;
};

static int traj_layout(Arena &ar, TrajBuffers &T, int n, int d, int m) {
  const int64_t S = 2ll * n * d;
  T.S = S;
  T.X0 = ar.take<double>((size_t)S * d);
  T.Xg = ar.take<double>((size_t)S * d);
  T.lg = ar.take<double>(S);
  T.gg = ar.take<double>((size_t)S * d);
  T.xprev = ar.take<double>((size_t)S * d);
  T.gprev = ar.take<double>((size_t)S * d);
  T.g0w = ar.take<double>(S);
  T.fmax = ar.take<double>(S);
  T.tprev = ar.take<int32_t>(S);
  T.nct = ar.take<int32_t>(S);
  T.all = ar.take<int32_t>(S);
  T.fperp = ar.take<double>(n);
  T.fd_bytes = sb_user_fd_workspace_bytes(S, d, 0);
  T.fd_ws = ar.take<char>(T.fd_bytes);
  T.lb.dtype = DT_F64;
  T.lb.B = S;
  T.lb.d = d;
  T.lb.m = m;
  if (lbfgs_carve(ar, T.lb)) return SB_E_NOMEM;
  return ar.ok() ? SB_OK : SB_E_NOMEM;
}

// FD l and gradient of `count` L-BFGS rows listed in idx into the state's
// slots (gather the rows, one batch of perturbed points, scatter back).
static int eval_state_rows(const sb_user_fn *fn, LbfgsBuffers &lb, int d, const double *params,
                           double eps, const int32_t *idx, int count, double *Xg, double *lg,
                           double *gg, void *fd_ws, size_t fd_bytes, hipStream_t s) {
  if (count <= 0) return SB_OK;
  hipLaunchKernelGGL(gather_state_rows_kernel, dim3((unsigned)ceil_div((int64_t)count * d, 256)),
                     dim3(256), 0, s, count, d, idx, (const double *)lb.X, Xg);
  SB_LAUNCH_CHECK();
  int st = sb_user_fd_dev(fn, count, d, Xg, params, eps, lg, gg, nullptr, nullptr, nullptr,
                          fd_ws, fd_bytes, s);
  if (st) return st;
  hipLaunchKernelGGL(scatter_state_rows_kernel, dim3((unsigned)ceil_div((int64_t)count * d, 256)),
                     dim3(256), 0, s, count, d, idx, lg, gg, (double *)lb.F, (double *)lb.G);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

// The seeds' L-BFGS with the bank recording; fperp [n] (device) per mode.
static int run_trajectories(const sb_user_fn *fn, int n, int d, const double *modes,
                            const double *params, const double *hdiag, double eps, int n_iter,
                            double grad_tol, TrajBuffers &T, double *fperp, double *Xbank,
                            double *Gbank, int32_t *blen, int64_t *evals, hipStream_t s) {
  const int64_t S = T.S;
  LbfgsBuffers &lb = T.lb;
  hipLaunchKernelGGL(gd_seeds_kernel, dim3((unsigned)S), dim3(256), 0, s, d, modes, hdiag, T.X0);
  SB_LAUNCH_CHECK();
  int st;
  if ((st = launch_lbfgs_init(lb, T.X0, s))) return st;
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, s, S, T.all);
  hipLaunchKernelGGL(traj_init_kernel, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, s, S,
                     T.tprev, T.fmax, T.nct);
  SB_LAUNCH_CHECK();
  if ((st = eval_state_rows(fn, lb, d, params, eps, T.all, (int)S, T.Xg, T.lg, T.gg, T.fd_ws,
                            T.fd_bytes, s)))
    return st;
  int64_t ev = S;
  auto record = [&]() {
    hipLaunchKernelGGL(traj_step_kernel, dim3((unsigned)S), dim3(256), 0, s, S, d, n_iter,
                       (const double *)lb.X, (const double *)lb.G, lb.cur, lb.iters, hdiag, 1e-3,
                       T.xprev, T.gprev, T.tprev, T.g0w, T.fmax, T.nct, Xbank, Gbank, blen);
  };
  record();
  SB_LAUNCH_CHECK();
  for (int step = 0; step < 42 * n_iter + 64; ++step) {
    if ((st = launch_lbfgs_step(lb, n_iter, grad_tol, s))) return st;
    record();
    SB_LAUNCH_CHECK();
    if ((st = launch_compact(lb, s))) return st;
    int32_t cnt = 0;
    SB_HIP(hipMemcpyAsync(&cnt, lb.count, 4, hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
    if (cnt <= 0) break;
    if ((st = eval_state_rows(fn, lb, d, params, eps, lb.idx, cnt, T.Xg, T.lg, T.gg, T.fd_ws,
                              T.fd_bytes, s)))
      return st;
    ev += cnt;
  }
  hipLaunchKernelGGL(traj_mode_kernel, dim3((unsigned)ceil_div(n, 64)), dim3(64), 0, s, n, d,
                     T.fmax, T.nct, fperp);
  SB_LAUNCH_CHECK();
  if (evals) *evals = ev;
  return SB_OK;
}

}  // namespace sb

using namespace sb;

static int fail(int st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  char buf[640];
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  set_error("%s", buf);
  return st;
}

static bool valid_name(const char *name) {
  if (!name || !*name || std::strlen(name) > 120) return false;
  if (!(std::isalpha((unsigned char)name[0]) || name[0] == '_')) return false;
  for (const char *c = name; *c; ++c)
    if (!(std::isalnum((unsigned char)*c) || *c == '_')) return false;
  return true;
}

extern "C" {

int32_t sb_user_compile(const char *source, const char *name, sb_user_fn **out) {
  if (!source || !out) return fail(SB_E_INVAL, "NULL source or output");
  *out = nullptr;
  if (!valid_name(name)) return fail(SB_E_INVAL, "the function name must be a C identifier");
  std::string code(source);
  code += "\nextern \"C\" __global__ void sb_user_eval_kernel(long long B, int d, const double *X,"
          " long long ldx, const double *params, double *l) {\n"
          "  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;\n"
          "  if (b < B) l[b] = ";
  code += name;
  code += "(X + b * ldx, d, params);\n}\n";
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, code.c_str(), "sb_user.hip", 0, nullptr, nullptr) !=
      HIPRTC_SUCCESS)
    return fail(SB_E_INVAL, "hipRTC could not create the program");
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult cr = hiprtcCompileProgram(prog, 7, opts);
  if (cr != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    return fail(SB_E_INVAL, "compiling the user likelihood failed: %.400s", log.c_str());
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  std::vector<char> obj(cs);
  hiprtcGetCode(prog, obj.data());
  hiprtcDestroyProgram(&prog);
  sb_user_fn *fn = new sb_user_fn;
  if (hipGetDevice(&fn->device) != hipSuccess || hipModuleLoadData(&fn->mod, obj.data()) !=
                                                       hipSuccess ||
      hipModuleGetFunction(&fn->eval, fn->mod, "sb_user_eval_kernel") != hipSuccess) {
    if (fn->mod) hipModuleUnload(fn->mod);
    delete fn;
    return fail(SB_E_DEVICE, "loading the compiled user likelihood failed");
  }
  *out = fn;
  return SB_OK;
}

void sb_user_release(sb_user_fn *fn) {
  if (!fn) return;
  if (fn->mod) hipModuleUnload(fn->mod);
  delete fn;
}

static int user_eval(const sb_user_fn *fn, int64_t B, int d, const double *X, int64_t ldx,
                     const double *params, double *l, hipStream_t s) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != fn->device)
    return fail(SB_E_DEVICE, "the user likelihood was compiled for device %d", fn->device);
  long long b = (long long)B, lx = (long long)ldx;
  int dd = d;
  void *args[] = {&b, &dd, &X, &lx, &params, &l};
  const unsigned grid = (unsigned)ceil_div(B, 256);
  if (hipModuleLaunchKernel(fn->eval, grid, 1, 1, 256, 1, 1, 0, s, args, nullptr) != hipSuccess)
    return fail(SB_E_DEVICE, "launching the user likelihood failed");
  return SB_OK;
}

int32_t sb_user_logl_dev(const sb_user_fn *fn, int64_t B, int32_t d, const double *X,
                         const double *params, double *l, void *stream) {
  if (!fn || B < 0 || d < 1 || (B > 0 && (!X || !l)))
    return fail(SB_E_INVAL, "bad user likelihood arguments");
  if (B == 0) return SB_OK;
  return user_eval(fn, B, d, X, d, params, l, (hipStream_t)stream);
}

size_t sb_user_fd_workspace_bytes(int64_t B, int32_t d, int32_t full) {
  if (B < 1 || d < 1) return 0;
  const int64_t R = fd_rows(d, full != 0);
  return align_up(8ull * B * R * d) + align_up(8ull * B * R) + 1024;
}

int32_t sb_user_fd_dev(const sb_user_fn *fn, int64_t B, int32_t d, const double *X,
                       const double *params, double eps, double *l, double *grad, double *hdiag,
                       double *H, double *probe_b, void *workspace, size_t ws_bytes,
                       void *stream) {
  if (!fn || B < 1 || d < 1 || !X) return fail(SB_E_INVAL, "bad finite-difference arguments");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(SB_E_INVAL, "eps must be finite and > 0");
  const bool full = H != nullptr;
  if (!workspace || ws_bytes < sb_user_fd_workspace_bytes(B, d, full))
    return fail(SB_E_NOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const int64_t R = fd_rows(d, full);
  Arena ar(workspace, ws_bytes);
  double *P = ar.take<double>((size_t)(B * R * d));
  double *F = ar.take<double>((size_t)(B * R));
  hipLaunchKernelGGL(fd_points_kernel, dim3((unsigned)ceil_div(B * R, 256)), dim3(256), 0, s, B,
                     d, R, X, eps, P);
  SB_LAUNCH_CHECK();
  int st = user_eval(fn, B * R, d, P, d, params, F, s);
  if (st) return st;
  hipLaunchKernelGGL(fd_combine_kernel, dim3((unsigned)ceil_div(B * d, 256)), dim3(256), 0, s, B,
                     d, R, F, eps, l, grad, hdiag, probe_b);
  SB_LAUNCH_CHECK();
  if (full) {
    hipLaunchKernelGGL(fd_hessian_kernel, dim3((unsigned)ceil_div(B * d * d, 256)), dim3(256), 0,
                       s, B, d, R, F, eps, H);
    SB_LAUNCH_CHECK();
  }
  return SB_OK;
}

}  // extern "C"

namespace sb {
// Geometry detection parameters with their defaults filled in.
struct GeoCfg {
  int n_iter, m;
  double grad_tol, eps_axis, eps_rot, rot_tol, eps_grad;
};
static GeoCfg geo_resolve(const sb_geometry_config *gc, int d, double eps_grad) {
  GeoCfg g;
  int lg = 0;
  while ((1 << lg) < d) ++lg;  // ceil(log2 d)
  g.n_iter = gc->n_iter > 0 ? gc->n_iter : std::max(10, 3 * lg);
  g.m = gc->m > 0 ? gc->m : 8;
  g.grad_tol = gc->grad_tol > 0 ? gc->grad_tol : 1e-6;
  g.eps_axis = gc->eps_axis > 0 ? gc->eps_axis : 1e-4;
  g.eps_rot = gc->eps_rot > 0 ? gc->eps_rot : 1e-2;
  g.rot_tol = gc->rot_tol;
  g.eps_grad = eps_grad;
  return g;
}

static size_t traj_bytes(int n, int d, int m) {
  Arena ar(nullptr, 0);
  TrajBuffers T;
  traj_layout(ar, T, n, d, m);
  return ar.off + 1024;
}
}  // namespace sb

extern "C" {

size_t sb_user_mode_evidence_workspace_bytes(int32_t n, int32_t d) {
  if (n < 1 || d < 1) return 0;
  const size_t nd = (size_t)n * d, ndd = nd * d;
  return sb_user_fd_workspace_bytes(n, d, 0) + sb_user_fd_workspace_bytes(n, d, 1) +
         3 * align_up(8 * nd) + 2 * align_up(8 * ndd) + 4 * align_up(8 * (size_t)n) +
         3 * align_up(4 * (size_t)n) + 4096;
}

// Laplace evidence at given modes; geo == nullptr: the probe alone decides
// (Step 2), else Step 1 (the trajectories' perpendicular fraction) and the
// probe only where it is inconclusive.  decision (host, nullable): 0 axis by
// trajectories, 1 rotated by them, 2 axis by the probe, 3 rotated by it.
static int32_t mode_evidence_impl(const sb_user_fn *fn, int32_t n, int32_t d,
                                  const double *modes, const double *params, const double *lo,
                                  const double *hi, double eps, double rot_tol,
                                  const GeoCfg *geo, double *fperp, int32_t *decision,
                                  double *logl, double *logdet, int32_t *full_used,
                                  int32_t *order, double *mode_log_z, double *log_z,
                                  void *workspace, size_t ws_bytes, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  Arena ar(workspace, ws_bytes);
  const size_t ws0 = sb_user_fd_workspace_bytes(n, d, 0), ws1 = sb_user_fd_workspace_bytes(n, d, 1);
  void *w0 = ar.take<char>(ws0);
  void *w1 = ar.take<char>(ws1);
  double *hd = ar.take<double>((size_t)n * d);
  double *hd1 = ar.take<double>((size_t)n * d);
  double *Xf = ar.take<double>((size_t)n * d);
  double *H = ar.take<double>((size_t)n * d * d);
  double *A = ar.take<double>((size_t)n * d * d);
  double *pb = ar.take<double>(n);
  double *l1 = ar.take<double>(n);
  double *ldf = ar.take<double>(n);
  ar.take<double>(n);
  int32_t *fullv = ar.take<int32_t>(n);
  int32_t *idx = ar.take<int32_t>(n);
  int32_t *info = ar.take<int32_t>(n);
  if (!ar.ok()) return fail(SB_E_NOMEM, "workspace too small");
  // diagonal curvature and the rotation probe of every mode (2d + 3 evaluations each)
  int st = sb_user_fd_dev(fn, n, d, modes, params, eps, logl, nullptr, hd, nullptr, pb, w0, ws0,
                          stream);
  if (st) return st;
  std::vector<double> h_hd((size_t)n * d), h_pb(n);
  SB_HIP(hipMemcpyAsync(h_hd.data(), hd, 8 * h_hd.size(), hipMemcpyDeviceToHost, s));
  SB_HIP(hipMemcpyAsync(h_pb.data(), pb, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  SB_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> h_full(n, 0), h_idx, h_dec(n, 2);
  std::vector<double> h_fp(n, (double)NAN);
  if (geo) {
    for (int64_t i = 0; i < (int64_t)n * d; ++i)
      if (!(h_hd[i] < 0.0))
        return fail(SB_E_NOTPD, "mode %lld: H_ii >= 0 (not a maximum)", (long long)(i / d));
    // Step 1: GreenDragon's seeds and the perpendicular step fraction
    const size_t o = align_up(ar.off);
    Arena tar((char *)ar.base + o, ar.cap > o ? ar.cap - o : 0);
    TrajBuffers T;
    if (traj_layout(tar, T, n, d, geo->m)) return fail(SB_E_NOMEM, "workspace too small");
    double *fp = fperp ? fperp : T.fperp;
    if ((st = run_trajectories(fn, n, d, modes, params, hd, geo->eps_grad, geo->n_iter,
                               geo->grad_tol, T, fp, nullptr, nullptr, nullptr, nullptr, s)))
      return st;
    SB_HIP(hipMemcpyAsync(h_fp.data(), fp, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
  }
  for (int k = 0; k < n; ++k) {
    double a = 0.0;
    for (int i = 0; i < d; ++i) a += h_hd[(size_t)k * d + i];
    a /= d;
    int dec;
    if (geo && h_fp[k] > geo->eps_rot)
      dec = 1;
    else if (geo && h_fp[k] <= geo->eps_axis)
      dec = 0;
    else
      dec = std::fabs(h_pb[k]) > rot_tol * std::fabs(a) ? 3 : 2;
    h_dec[k] = dec;
    if (dec == 1 || dec == 3) {
      h_full[k] = 1;
      h_idx.push_back(k);
    }
  }
  if (decision) std::memcpy(decision, h_dec.data(), 4 * (size_t)n);
  if (full_used) std::memcpy(full_used, h_full.data(), 4 * (size_t)n);
  SB_HIP(hipMemcpyAsync(fullv, h_full.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(fd_diag_logdet_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n,
                     d, hd, fullv, logdet);
  SB_LAUNCH_CHECK();
  const int m = (int)h_idx.size();
  if (m > 0) {
    // full FD Hessians of the rotated modes, log det(-H) by Cholesky
    SB_HIP(hipMemcpyAsync(idx, h_idx.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)ceil_div((int64_t)m * d, 256)),
                       dim3(256), 0, s, m, d, idx, modes, Xf);
    SB_LAUNCH_CHECK();
    if ((st = sb_user_fd_dev(fn, m, d, Xf, params, eps, l1, nullptr, hd1, H, nullptr, w1, ws1,
                             stream)))
      return st;
    const int64_t nel = (int64_t)m * d * d;
    hipLaunchKernelGGL(negate_kernel, dim3((unsigned)ceil_div(nel, 256)), dim3(256), 0, s, nel, H,
                       A);
    SB_LAUNCH_CHECK();
    if ((st = chol_batched(m, d, A, A, info, s))) return st;
    if ((st = launch_logdet(m, d, A, info, ldf, s))) return st;
    hipLaunchKernelGGL(scatter_logdet_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s,
                       m, idx, ldf, info, logdet);
    SB_LAUNCH_CHECK();
  }
  if ((st = launch_combine(n, d, lo, hi, logl, logdet, modes, order, mode_log_z, log_z, s)))
    return st;
  std::vector<double> h_ld(n);
  SB_HIP(hipMemcpyAsync(h_ld.data(), logdet, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  SB_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(h_ld[k]))
      return fail(SB_E_NOTPD, "mode %d: -H is not positive definite (not a maximum)", k);
  return SB_OK;
}

int32_t sb_user_mode_evidence_dev(const sb_user_fn *fn, int32_t n, int32_t d,
                                  const double *modes, const double *params, const double *lo,
                                  const double *hi, double eps, double rot_tol, double *logl,
                                  double *logdet, int32_t *full_used, int32_t *order,
                                  double *mode_log_z, double *log_z, void *workspace,
                                  size_t ws_bytes, void *stream) {
  if (!fn || n < 1 || d < 1 || !modes || !lo || !hi || !logl || !logdet || !order ||
      !mode_log_z || !log_z)
    return fail(SB_E_INVAL, "bad evidence-at-modes arguments");
  if (!(eps > 0.0) || !std::isfinite(eps) || !(rot_tol >= 0.0))
    return fail(SB_E_INVAL, "need eps > 0 and rot_tol >= 0");
  if (!workspace || ws_bytes < sb_user_mode_evidence_workspace_bytes(n, d))
    return fail(SB_E_NOMEM, "workspace too small");
  return mode_evidence_impl(fn, n, d, modes, params, lo, hi, eps, rot_tol, nullptr, nullptr,
                            nullptr, logl, logdet, full_used, order, mode_log_z, log_z,
                            workspace, ws_bytes, stream);
}

static bool geo_ok(const sb_geometry_config *gc) {
  return gc && gc->rot_tol >= 0.0 && std::isfinite(gc->rot_tol) && std::isfinite(gc->grad_tol) &&
         std::isfinite(gc->eps_axis) && std::isfinite(gc->eps_rot) && gc->n_iter <= 100000 &&
         gc->m <= kMaxMem;
}

size_t sb_user_mode_evidence_geo_workspace_bytes(int32_t n, int32_t d,
                                                 const sb_geometry_config *gc) {
  if (n < 1 || d < 1 || !geo_ok(gc)) return 0;
  const GeoCfg g = geo_resolve(gc, d, 1.0);
  return sb_user_mode_evidence_workspace_bytes(n, d) + traj_bytes(n, d, g.m);
}

int32_t sb_user_mode_evidence_geo_dev(const sb_user_fn *fn, int32_t n, int32_t d,
                                      const double *modes, const double *params,
                                      const double *lo, const double *hi, double eps_grad,
                                      double eps_hess, const sb_geometry_config *gc,
                                      double *logl, double *logdet, double *fperp,
                                      int32_t *decision, int32_t *order, double *mode_log_z,
                                      double *log_z, void *workspace, size_t ws_bytes,
                                      void *stream) {
  if (!fn || n < 1 || d < 1 || !modes || !lo || !hi || !logl || !logdet || !order ||
      !mode_log_z || !log_z)
    return fail(SB_E_INVAL, "bad evidence-at-modes arguments");
  if (!(eps_grad > 0.0) || !std::isfinite(eps_grad) || !(eps_hess > 0.0) ||
      !std::isfinite(eps_hess) || !geo_ok(gc))
    return fail(SB_E_INVAL, "need eps_grad, eps_hess > 0 and a valid geometry configuration");
  if (!workspace || ws_bytes < sb_user_mode_evidence_geo_workspace_bytes(n, d, gc))
    return fail(SB_E_NOMEM, "workspace too small");
  const GeoCfg g = geo_resolve(gc, d, eps_grad);
  return mode_evidence_impl(fn, n, d, modes, params, lo, hi, eps_hess, g.rot_tol, &g, fperp,
                            decision, logl, logdet, nullptr, order, mode_log_z, log_z,
                            workspace, ws_bytes, stream);
}

size_t sb_user_trajectories_workspace_bytes(int32_t n, int32_t d, int32_t m) {
  if (n < 1 || d < 1 || m < 1 || m > kMaxMem) return 0;
  return traj_bytes(n, d, m);
}

int32_t sb_user_trajectories_dev(const sb_user_fn *fn, int32_t n, int32_t d, const double *modes,
                                 const double *params, const double *hdiag, double eps,
                                 int32_t n_iter, int32_t m, double grad_tol, double *fperp,
                                 double *Xbank, double *Gbank, int32_t *bank_len,
                                 void *workspace, size_t ws_bytes, void *stream) {
  if (!fn || n < 1 || d < 1 || !modes || !hdiag || !fperp || n_iter < 1 || m < 1 ||
      m > kMaxMem || !(eps > 0.0) || !std::isfinite(eps) || !std::isfinite(grad_tol) ||
      (Xbank && !Gbank) || (!Xbank && Gbank))
    return fail(SB_E_INVAL, "bad trajectory arguments");
  if (!workspace || ws_bytes < sb_user_trajectories_workspace_bytes(n, d, m))
    return fail(SB_E_NOMEM, "workspace too small");
  Arena ar(workspace, ws_bytes);
  TrajBuffers T;
  if (traj_layout(ar, T, n, d, m)) return fail(SB_E_NOMEM, "workspace too small");
  return run_trajectories(fn, n, d, modes, params, hdiag, eps, n_iter, grad_tol, T, fperp, Xbank,
                          Gbank, bank_len, nullptr, (hipStream_t)stream);
}

// Rows of the evidence pipeline's workspace for a user likelihood.
struct UserLayout {
  double *P0, *P1, *Xpts, *lpts, *best_l, *X0, *Xg, *lg, *gg, *Xend, *lend, *modes;
  int32_t *best_j, *start_ray, *status, *rep_of, *reps, *order;
  uint8_t *valid;
  double *mlogl, *mlogdet, *mlz, *logz;
  void *fd_ws, *dd_ws, *me_ws;
  size_t fd_bytes, dd_bytes, me_bytes;
  LbfgsBuffers lb;
};

static int user_layout(Arena &ar, UserLayout &U, int d, const sb_config *c) {
  const int64_t R = c->n_rays, NP = (int64_t)c->n_rays * c->n_points, B = c->n_starts;
  const int cap = c->max_modes;
  U.P0 = ar.take<double>((size_t)R * d);
  U.P1 = ar.take<double>((size_t)R * d);
  U.Xpts = ar.take<double>((size_t)NP * d);
  U.lpts = ar.take<double>(NP);
  U.best_l = ar.take<double>(R);
  U.best_j = ar.take<int32_t>(R);
  U.start_ray = ar.take<int32_t>(B);
  U.X0 = ar.take<double>((size_t)B * d);
  U.Xg = ar.take<double>((size_t)2 * B * d);
  U.lg = ar.take<double>(2 * B);
  U.gg = ar.take<double>((size_t)2 * B * d);
  U.Xend = ar.take<double>((size_t)B * d);
  U.lend = ar.take<double>(B);
  U.status = ar.take<int32_t>(B);
  U.valid = ar.take<uint8_t>(B);
  U.rep_of = ar.take<int32_t>(B);
  U.reps = ar.take<int32_t>(cap);
  U.modes = ar.take<double>((size_t)cap * d);
  U.order = ar.take<int32_t>(cap);
  U.mlogl = ar.take<double>(cap);
  U.mlogdet = ar.take<double>(cap);
  U.mlz = ar.take<double>(cap);
  U.logz = ar.take<double>(4);
  U.fd_bytes = sb_user_fd_workspace_bytes(2 * B, d, 0);
  U.fd_ws = ar.take<char>(U.fd_bytes);
  U.dd_bytes = dedup_ws_bytes((int)B) + 1024;
  U.dd_ws = ar.take<char>(U.dd_bytes);
  // the mode evidence with both steps of the geometry detection (defaults)
  sb_geometry_config gc = {0, 0, 0.0, 0.0, 0.0, 0.0};
  U.me_bytes = sb_user_mode_evidence_geo_workspace_bytes(cap, d, &gc);
  U.me_ws = ar.take<char>(U.me_bytes);
  U.lb.dtype = DT_F64;
  U.lb.B = B;
  U.lb.d = d;
  U.lb.m = c->m;
  if (lbfgs_carve(ar, U.lb)) return SB_E_NOMEM;
  return ar.ok() ? SB_OK : SB_E_NOMEM;
}

static bool user_cfg_ok(const sb_config *c) {
  return c && c->n_rays >= 1 && c->n_points >= 1 && c->n_starts >= 1 &&
         c->n_starts <= c->n_rays && c->m >= 1 && c->m <= kMaxMem && c->max_modes >= 1;
}

size_t sb_user_evidence_workspace_bytes(int32_t d, const sb_config *cfg) {
  if (d < 1 || !user_cfg_ok(cfg)) return 0;
  Arena ar(nullptr, 0);
  UserLayout U;
  user_layout(ar, U, d, cfg);
  return ar.off + 4096;
}

// FD l and gradient at `count` L-BFGS rows listed in idx (host count).
static int user_eval_rows(const sb_user_fn *fn, UserLayout &U, int d, const double *params,
                          double eps, const int32_t *idx, int count, hipStream_t s) {
  if (count <= 0) return SB_OK;
  hipLaunchKernelGGL(gather_state_rows_kernel, dim3((unsigned)ceil_div((int64_t)count * d, 256)),
                     dim3(256), 0, s, count, d, idx, (const double *)U.lb.X, U.Xg);
  SB_LAUNCH_CHECK();
  int st = sb_user_fd_dev(fn, count, d, U.Xg, params, eps, U.lg, U.gg, nullptr, nullptr,
                          nullptr, U.fd_ws, U.fd_bytes, s);
  if (st) return st;
  hipLaunchKernelGGL(scatter_state_rows_kernel, dim3((unsigned)ceil_div((int64_t)count * d, 256)),
                     dim3(256), 0, s, count, d, idx, U.lg, U.gg, (double *)U.lb.F,
                     (double *)U.lb.G);
  SB_LAUNCH_CHECK();
  return SB_OK;
}

int32_t sb_user_evidence_dev(const sb_user_fn *fn, int32_t d, const double *params,
                             const double *lo, const double *hi, const sb_config *cfg,
                             double eps, double eps_hess, double rot_tol, sb_result *res,
                             void *workspace, size_t ws_bytes, void *stream) {
  if (!fn || d < 1 || !lo || !hi || !res) return fail(SB_E_INVAL, "bad user evidence arguments");
  if (!user_cfg_ok(cfg)) return fail(SB_E_INVAL, "bad configuration");
  if (!(eps > 0.0) || !std::isfinite(eps) || !(eps_hess > 0.0) || !std::isfinite(eps_hess) ||
      !(rot_tol >= 0.0))
    return fail(SB_E_INVAL, "need eps > 0, eps_hess > 0 and rot_tol >= 0");
  if (!workspace || ws_bytes < sb_user_evidence_workspace_bytes(d, cfg))
    return fail(SB_E_NOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  for (double &t : res->seconds) t = 0.0;
  Arena ar(workspace, ws_bytes);
  UserLayout U;
  if (user_layout(ar, U, d, cfg)) return fail(SB_E_NOMEM, "workspace too small");
  const int R = cfg->n_rays, NPTS = cfg->n_points, B = cfg->n_starts, cap = cfg->max_modes;
  const int max_iter = cfg->max_iter > 0 ? cfg->max_iter : 10 * d + 200;
  const double tol = cfg->grad_tol > 0 ? cfg->grad_tol : 1e-6;
  std::vector<double> hlo(d), hhi(d);
  SB_HIP(hipMemcpyAsync(hlo.data(), lo, 8 * (size_t)d, hipMemcpyDeviceToHost, s));
  SB_HIP(hipMemcpyAsync(hhi.data(), hi, 8 * (size_t)d, hipMemcpyDeviceToHost, s));
  SB_HIP(hipStreamSynchronize(s));
  double wmax = 0.0;
  for (int i = 0; i < d; ++i) {
    if (!(std::isfinite(hlo[i]) && std::isfinite(hhi[i]) && hlo[i] < hhi[i]))
      return fail(SB_E_INVAL, "box coordinate %d is not a finite interval", i);
    wmax = std::max(wmax, hhi[i] - hlo[i]);
  }
  const double tau = cfg->dedup_tol > 0 ? cfg->dedup_tol : 1e-4 * wmax;
  int st;
  // discovery: rays, l at every sample point, per-ray argmax, top starts
  if ((st = launch_rays(d, lo, hi, R, cfg->seed, 0u, U.P0, U.P1, nullptr, nullptr, s)))
    return st;
  const int64_t NP = (int64_t)R * NPTS;
  hipLaunchKernelGGL(ray_points_kernel, dim3((unsigned)ceil_div(NP * d, 256)), dim3(256), 0, s, R,
                     NPTS, d, U.P0, U.P1, U.Xpts);
  SB_LAUNCH_CHECK();
  if ((st = user_eval(fn, NP, d, U.Xpts, d, params, U.lpts, s))) return st;
  if ((st = launch_ray_argmax(R, NPTS, SB_DTYPE_F64, U.lpts, U.best_l, U.best_j, s))) return st;
  if ((st = launch_topn(R, B, U.best_l, U.start_ray, s))) return st;
  if ((st = launch_gather_starts(d, NPTS, B, U.start_ray, U.best_j, U.P0, U.P1, U.X0, s)))
    return st;
  // batched L-BFGS on FD gradients (2d + 3 user evaluations per row)
  LbfgsBuffers &lb = U.lb;
  if ((st = launch_lbfgs_init(lb, U.X0, s))) return st;
  std::vector<int32_t> all(B);
  for (int i = 0; i < B; ++i) all[i] = i;
  SB_HIP(hipMemcpyAsync(lb.idx, all.data(), 4 * (size_t)B, hipMemcpyHostToDevice, s));
  if ((st = user_eval_rows(fn, U, d, params, eps, lb.idx, B, s))) return st;
  int64_t grad_evals = B;
  int steps = 0;
  for (; steps < 42 * max_iter + 64; ++steps) {
    if ((st = launch_lbfgs_step(lb, max_iter, tol, s))) return st;
    if ((st = launch_compact(lb, s))) return st;
    int32_t cnt = 0;
    SB_HIP(hipMemcpyAsync(&cnt, lb.count, 4, hipMemcpyDeviceToHost, s));
    SB_HIP(hipStreamSynchronize(s));
    if (cnt <= 0) break;
    if ((st = user_eval_rows(fn, U, d, params, eps, lb.idx, cnt, s))) return st;
    grad_evals += cnt;
  }
  if ((st = launch_lbfgs_gather(lb, U.Xend, U.lend, true, nullptr, U.status, nullptr, s)))
    return st;
  // converged (or iteration-capped) end points inside the box, leader dedup
  std::vector<int32_t> h_st(B);
  std::vector<double> h_x((size_t)B * d);
  SB_HIP(hipMemcpyAsync(h_st.data(), U.status, 4 * (size_t)B, hipMemcpyDeviceToHost, s));
  SB_HIP(hipMemcpyAsync(h_x.data(), U.Xend, 8 * h_x.size(), hipMemcpyDeviceToHost, s));
  SB_HIP(hipStreamSynchronize(s));
  std::vector<uint8_t> h_valid(B, 0);
  int n_dead = 0;
  for (int b = 0; b < B; ++b) {
    bool ok = h_st[b] == 1;
    for (int i = 0; ok && i < d; ++i)
      ok = h_x[(size_t)b * d + i] >= hlo[i] && h_x[(size_t)b * d + i] <= hhi[i];
    h_valid[b] = ok ? 1 : 0;
    n_dead += h_st[b] == 4;
  }
  SB_HIP(hipMemcpyAsync(U.valid, h_valid.data(), (size_t)B, hipMemcpyHostToDevice, s));
  int n_reps = 0;
  Arena dar(U.dd_ws, U.dd_bytes);
  st = dedup_run(B, d, U.Xend, SB_DTYPE_F64, U.lend, SB_DTYPE_F64, U.valid, tau, U.rep_of, U.reps,
                 cap, &n_reps, dar, s);
  res->n_modes = n_reps;
  res->iterations = steps;
  res->n_logl_evals = NP;
  res->n_grad_evals = grad_evals;
  res->n_dead_starts = n_dead;
  if (st) {
    res->log_z = NAN;
    return st == SB_E_CAPACITY ? fail(st, "%d modes exceed max_modes = %d", n_reps, cap) : st;
  }
  if (n_reps == 0) {
    res->log_z = -INFINITY;
    return fail(SB_E_NOMODE, "no start converged to a maximum inside the box");
  }
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)ceil_div((int64_t)n_reps * d, 256)),
                     dim3(256), 0, s, n_reps, d, U.reps, U.Xend, U.modes);
  SB_LAUNCH_CHECK();
  // geometry by the trajectories of GreenDragon's seeds (FD gradients with
  // step eps), the probe where they are inconclusive
  sb_geometry_config gc = {0, cfg->m, tol, 0.0, 0.0, rot_tol};
  const GeoCfg g = geo_resolve(&gc, d, eps);
  st = mode_evidence_impl(fn, n_reps, d, U.modes, params, lo, hi, eps_hess, rot_tol, &g, nullptr,
                          nullptr, U.mlogl, U.mlogdet, nullptr, U.order, U.mlz, U.logz, U.me_ws,
                          U.me_bytes, s);
  if (st) {
    res->log_z = NAN;
    return st;
  }
  std::vector<int32_t> h_order(n_reps);
  std::vector<double> h_modes((size_t)n_reps * d), h_l(n_reps), h_ld(n_reps), h_mlz(n_reps);
  double h_lz = NAN;
  SB_HIP(hipMemcpyAsync(h_order.data(), U.order, 4 * (size_t)n_reps, hipMemcpyDeviceToHost, s));
  SB_HIP(hipMemcpyAsync(h_modes.data(), U.modes, 8 * h_modes.size(), hipMemcpyDeviceToHost, s));
  SB_HIP(hipMemcpyAsync(h_l.data(), U.mlogl, 8 * (size_t)n_reps, hipMemcpyDeviceToHost, s));
  SB_HIP(hipMemcpyAsync(h_ld.data(), U.mlogdet, 8 * (size_t)n_reps, hipMemcpyDeviceToHost, s));
  SB_HIP(hipMemcpyAsync(h_mlz.data(), U.mlz, 8 * (size_t)n_reps, hipMemcpyDeviceToHost, s));
  SB_HIP(hipMemcpyAsync(&h_lz, U.logz, 8, hipMemcpyDeviceToHost, s));
  SB_HIP(hipStreamSynchronize(s));
  res->log_z = h_lz;
  for (int k = 0; k < n_reps; ++k) {
    const int src = h_order[k];
    if (res->modes)
      std::memcpy(res->modes + (size_t)k * d, h_modes.data() + (size_t)src * d, 8 * (size_t)d);
    if (res->mode_log_z) res->mode_log_z[k] = h_mlz[k];
    if (res->mode_logl) res->mode_logl[k] = h_l[src];
    if (res->log_det_h) res->log_det_h[k] = h_ld[src];
  }
  return SB_OK;
}

}  // extern "C"
