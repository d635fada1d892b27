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

size_t sb_user_mode_evidence_workspace_bytes(int32_t n, int32_t d) {
  if (n < 1 || d < 1) return 0;
  const size_t nd = (size_t)n * d, ndd = nd * d;
  return sb_user_fd_workspace_bytes(n, d, 0) + sb_user_fd_workspace_bytes(n, d, 1) +
         3 * align_up(8 * nd) + 2 * align_up(8 * ndd) + 4 * align_up(8 * (size_t)n) +
         3 * align_up(4 * (size_t)n) + 4096;
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
  std::vector<int32_t> h_full(n, 0), h_idx;
  for (int k = 0; k < n; ++k) {
    double a = 0.0;
    for (int i = 0; i < d; ++i) a += h_hd[(size_t)k * d + i];
    a /= d;
    if (std::fabs(h_pb[k]) > rot_tol * std::fabs(a)) {
      h_full[k] = 1;
      h_idx.push_back(k);
    }
  }
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

}  // extern "C"
