// extern "C" entry points of sb.h: argument validation (before any HIP call),
// device checks, workspace sizing, and dispatch to the kernels.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

using namespace sb;

namespace {

// The library targets gfx950 only; checked once per process.
int device_status() {
  static std::once_flag once;
  static int status = SB_OK;
  static char msg[256] = {0};
  std::call_once(once, [] {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
      status = SB_E_DEVICE;
      snprintf(msg, sizeof(msg), "no HIP device available");
      return;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      status = SB_E_DEVICE;
      snprintf(msg, sizeof(msg), "hipGetDeviceProperties failed");
      return;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      status = SB_E_DEVICE;
      snprintf(msg, sizeof(msg), "device %s is not gfx950 (MI355X)", prop.gcnArchName);
    }
  });
  if (status != SB_OK) set_error("%s", msg);
  return status;
}

int fail(int st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  char buf[512];
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  set_error("%s", buf);
  return st;
}

// Checks that need no array contents.
int validate_shape(const sb_loglik *ll) {
  if (!ll) return fail(SB_E_INVAL, "loglik is NULL");
  if (ll->d < 1) return fail(SB_E_INVAL, "d must be >= 1 (got %d)", ll->d);
  if (ll->K < 1) return fail(SB_E_INVAL, "K must be >= 1 (got %d)", ll->K);
  if (ll->family != SB_FAMILY_GAUSS_MIX && ll->family != SB_FAMILY_STUDENT_T)
    return fail(SB_E_INVAL, "unknown family %d", ll->family);
  if (ll->norm != SB_NORM_PEAK_ZERO && ll->norm != SB_NORM_DENSITY)
    return fail(SB_E_INVAL, "unknown normalisation %d", ll->norm);
  if (!ll->mu || !ll->prec) return fail(SB_E_INVAL, "mu and prec must not be NULL");
  if (ll->family == SB_FAMILY_STUDENT_T) {
    if (ll->K != 1) return fail(SB_E_UNSUPPORTED, "Student-t supports K = 1 only");
    if (!(ll->nu > 0.0) || !std::isfinite(ll->nu)) return fail(SB_E_INVAL, "nu must be > 0");
  }
  if (!std::isfinite(ll->logl_offset)) return fail(SB_E_INVAL, "logl_offset must be finite");
  if (ll->K > 16) return fail(SB_E_UNSUPPORTED, "at most 16 components are supported");
  return SB_OK;
}

int validate_cfg(const sb_loglik *ll, const sb_config *c) {
  if (!c) return fail(SB_E_INVAL, "config is NULL");
  if (c->m < 1 || c->m > kMaxMem)
    return fail(SB_E_INVAL, "m must be in [1, %d] (got %d)", kMaxMem, c->m);
  if (c->n_rays < 1 || c->n_points < 1) return fail(SB_E_INVAL, "n_rays, n_points must be >= 1");
  if (c->n_starts < 1 || c->n_starts > c->n_rays)
    return fail(SB_E_INVAL, "need 1 <= n_starts <= n_rays");
  if (c->max_modes < 1) return fail(SB_E_INVAL, "max_modes must be >= 1");
  if (c->precision != SB_PREC_FP64 && c->precision != SB_PREC_MIXED)
    return fail(SB_E_INVAL, "unknown precision %d", c->precision);
  if (ll->d > 4096) return fail(SB_E_UNSUPPORTED, "d > 4096 is not supported");
  if ((int64_t)c->n_rays * c->n_points > (int64_t)1 << 30)
    return fail(SB_E_INVAL, "n_rays * n_points too large");
  return SB_OK;
}

int validate_box_host(int d, const double *lo, const double *hi) {
  if (!lo || !hi) return fail(SB_E_INVAL, "box bounds must not be NULL");
  for (int i = 0; i < d; ++i)
    if (!std::isfinite(lo[i]) || !std::isfinite(hi[i]) || !(lo[i] < hi[i]))
      return fail(SB_E_INVAL, "box coordinate %d: need finite lo < hi", i);
  return SB_OK;
}

int validate_arrays_host(const sb_loglik *ll) {
  const int64_t d = ll->d, K = ll->K;
  for (int64_t i = 0; i < K * d; ++i)
    if (!std::isfinite(ll->mu[i])) return fail(SB_E_INVAL, "mu has a non-finite entry");
  if (ll->log_w)
    for (int64_t k = 0; k < K; ++k)
      if (!std::isfinite(ll->log_w[k])) return fail(SB_E_INVAL, "log_w has a non-finite entry");
  for (int64_t i = 0; i < K * d * d; ++i)
    if (!std::isfinite(ll->prec[i])) return fail(SB_E_INVAL, "prec has a non-finite entry");
  return SB_OK;
}

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

Model model_from(const sb_model_dev *m) {
  Model r;
  r.family = m->family;
  r.norm = m->norm;
  r.d = m->d;
  r.K = m->K;
  r.mu64 = m->mu;
  r.P64 = m->prec;
  r.beta = m->beta;
  r.mu32 = m->mu_lp;
  r.Plp = m->prec_lp;
  r.nu = m->nu;
  r.c = m->logl_offset;
  return r;
}

// Model for a GEMM dtype: F32_SPLIT reads prec_lp as [2][K][d][d] BF16.
Model model_for(const sb_model_dev *m, int dtype) {
  Model r = model_from(m);
  if (dtype == SB_DTYPE_F32_SPLIT) {
    r.Phi = (const bf16_t *)m->prec_lp;
    r.Plo = r.Phi + (size_t)m->K * m->d * m->d;
    r.Plp = nullptr;
  }
  return r;
}

int check_gemm_dtype(const sb_model_dev *m, int dtype) {
  if (dtype != SB_DTYPE_F64 && dtype != SB_DTYPE_F32 && dtype != SB_DTYPE_F32_SPLIT)
    return fail(SB_E_INVAL, "dtype must be F64, F32 or F32_SPLIT");
  if (dtype != SB_DTYPE_F64 && (!m->prec_lp || !m->mu_lp))
    return fail(SB_E_INVAL, "dtype F32 / F32_SPLIT needs prec_lp and mu_lp");
  if (dtype == SB_DTYPE_F32_SPLIT && m->d % 8 != 0)
    return fail(SB_E_UNSUPPORTED, "F32_SPLIT needs d a multiple of 8 (got %d)", m->d);
  return SB_OK;
}

int validate_model(const sb_model_dev *m) {
  if (!m) return fail(SB_E_INVAL, "model is NULL");
  sb_loglik ll;
  ll.family = m->family;
  ll.norm = m->norm;
  ll.d = m->d;
  ll.K = m->K;
  ll.mu = m->mu;
  ll.prec = m->prec;
  ll.nu = m->nu;
  ll.logl_offset = m->logl_offset;
  ll.log_w = m->log_w;
  int st = validate_shape(&ll);
  if (st) return st;
  if (!m->beta) return fail(SB_E_INVAL, "beta (from sb_prep_dev) must not be NULL");
  return SB_OK;
}

// ------------------------------------------------ allocation-free logL + gradient
//
// For callers that cannot allocate (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc): the contraction's Y rows and q
// partials live in a file-scope device array of kStaticScratchBytes per GPU
// instead of a caller workspace.  In host code the array's name is not a
// device address: its address on the current device is looked up once per
// device (hipGetSymbolAddress with that device current) and only that
// address is handed to the kernels.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;  // 32 MiB per GPU
static __device__ __align__(256) char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address (looked up on its first use there).
int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(SB_E_DEVICE, "no current device for the static scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SB_E_DEVICE, "static scratch address: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SB_OK;
}

size_t eval_bytes(int dtype, int d, int K, int64_t B, bool with_aux) {
  const size_t es = (dtype == SB_DTYPE_F64) ? 8 : 4;
  size_t n = align_up(es * (size_t)B * K * d) + align_up(es * (size_t)B * K * ceil_div(d, 64));
  if (with_aux) n += align_up(es * (size_t)B * K) + align_up(es * (size_t)B * d);
  return n + 1024;
}

}  // namespace

// =====================================================================
extern "C" {

const char *sb_status_string(int32_t st) {
  switch (st) {
    case SB_OK: return "SB_OK";
    case SB_E_INVAL: return "SB_E_INVAL: invalid argument";
    case SB_E_NOTPD: return "SB_E_NOTPD: precision matrix not symmetric positive definite";
    case SB_E_NOMEM: return "SB_E_NOMEM: out of device memory or workspace too small";
    case SB_E_DEVICE: return "SB_E_DEVICE: HIP runtime error or no gfx950 device";
    case SB_E_NOMODE: return "SB_E_NOMODE: no mode passed the filters";
    case SB_E_CAPACITY: return "SB_E_CAPACITY: more modes than max_modes";
    case SB_E_UNSUPPORTED: return "SB_E_UNSUPPORTED: valid but unsupported request";
    case SB_E_NOCONV: return "SB_E_NOCONV: an iteration stopped at its cap above its tolerance";
    default: return "unknown status";
  }
}

const char *sb_last_error(void) { return last_error(); }
int32_t sb_abi_version(void) { return SB_ABI_VERSION; }

size_t sb_evidence_workspace_bytes(const sb_loglik *ll, const sb_config *cfg) {
  if (validate_shape(ll) || validate_cfg(ll, cfg)) return 0;
  return evidence_ws_bytes(ll, cfg);
}

// Shared by sb_evidence_dev and sb_evidence_exec_dev: argument checks that
// need no array contents (the box is checked on the device in prep), then
// the path on the caller's stream.
static int32_t evidence_dev(const sb_loglik *ll, const sb_box *box, const sb_config *cfg,
                            sb_result *res, void *workspace, size_t ws_bytes, void *stream,
                            ExecCtx *ex) {
  int st = validate_shape(ll);
  if (!st) st = validate_cfg(ll, cfg);
  if (!st && (!box || !box->lo || !box->hi)) st = fail(SB_E_INVAL, "box is NULL");
  if (!st && !res) st = fail(SB_E_INVAL, "result is NULL");
  if (st) {
    if (res) res->log_z = NAN;
    return st;
  }
  if ((st = device_status())) {
    res->log_z = NAN;
    return st;
  }
  if (ex) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != ex->device) {
      res->log_z = NAN;
      return fail(SB_E_INVAL, "execution context of device %d used on device %d", ex->device,
                  dev);
    }
  }
  DevProblem P;
  P.family = ll->family;
  P.norm = ll->norm;
  P.d = ll->d;
  P.K = ll->K;
  P.log_w = ll->log_w;
  P.mu = ll->mu;
  P.prec = ll->prec;
  P.lo = box->lo;
  P.hi = box->hi;
  P.nu = ll->nu;
  P.c = ll->logl_offset;
  st = run_evidence(P, cfg, res, workspace, ws_bytes, (hipStream_t)stream, ex);
  if (st && st != SB_E_NOMODE && st != SB_E_CAPACITY) res->log_z = NAN;
  return st;
}

int32_t sb_evidence_dev(const sb_loglik *ll, const sb_box *box, const sb_config *cfg,
                        sb_result *res, void *workspace, size_t ws_bytes, void *stream) {
  return evidence_dev(ll, box, cfg, res, workspace, ws_bytes, stream, nullptr);
}

static int validate_chisao(const sb_config *cfg, const sb_chisao_config *cc) {
  if (!cc) return fail(SB_E_INVAL, "ChiSao configuration is NULL");
  if (cfg->precision != SB_PREC_FP64)
    return fail(SB_E_UNSUPPORTED, "the ChiSao cycle runs in FP64 (precision must be FP64)");
  if (cc->n_osc < 1 || cc->n_osc > 64) return fail(SB_E_INVAL, "n_osc must be in [1, 64]");
  if (cc->n_cloud < 0 || cc->n_anti < 0) return fail(SB_E_INVAL, "negative step counts");
  if (cc->n_smooth > 256 || cc->n_cloud > 256 || cc->n_anti > 100000)
    return fail(SB_E_INVAL, "step counts too large");
  if (!(cc->momentum >= 0.0 && cc->momentum < 1.0))
    return fail(SB_E_INVAL, "momentum must be in [0, 1)");
  if (!std::isfinite(cc->sigma) || !std::isfinite(cc->alpha_cloud) ||
      !std::isfinite(cc->alpha_anti) || !std::isfinite(cc->stick_tol) ||
      !std::isfinite(cc->ref_delta))
    return fail(SB_E_INVAL, "non-finite ChiSao parameter");
  if (cc->n_ref < 0 || cc->n_ref > 4096) return fail(SB_E_INVAL, "n_ref must be in [0, 4096]");
  if ((int64_t)cfg->n_rays * cc->n_ref > (int64_t)1 << 28)
    return fail(SB_E_INVAL, "n_rays * n_ref too large");
  if (cc->n_reseed_pts > 65536) return fail(SB_E_INVAL, "n_reseed_pts too large");
  return SB_OK;
}

size_t sb_evidence_chisao_workspace_bytes(const sb_loglik *ll, const sb_config *cfg,
                                          const sb_chisao_config *cc) {
  if (validate_shape(ll) || validate_cfg(ll, cfg) || validate_chisao(cfg, cc)) return 0;
  return evidence_ws_bytes(ll, cfg, cc);
}

int32_t sb_evidence_chisao_dev(const sb_loglik *ll, const sb_box *box, const sb_config *cfg,
                               const sb_chisao_config *cc, sb_result *res, void *workspace,
                               size_t ws_bytes, void *stream) {
  int st = validate_shape(ll);
  if (!st) st = validate_cfg(ll, cfg);
  if (!st) st = validate_chisao(cfg, cc);
  if (!st && (!box || !box->lo || !box->hi)) st = fail(SB_E_INVAL, "box is NULL");
  if (!st && !res) st = fail(SB_E_INVAL, "result is NULL");
  if (st) {
    if (res) res->log_z = NAN;
    return st;
  }
  if ((st = device_status())) {
    res->log_z = NAN;
    return st;
  }
  DevProblem P;
  P.family = ll->family;
  P.norm = ll->norm;
  P.d = ll->d;
  P.K = ll->K;
  P.log_w = ll->log_w;
  P.mu = ll->mu;
  P.prec = ll->prec;
  P.lo = box->lo;
  P.hi = box->hi;
  P.nu = ll->nu;
  P.c = ll->logl_offset;
  st = run_evidence(P, cfg, res, workspace, ws_bytes, (hipStream_t)stream, nullptr, cc);
  if (st && st != SB_E_NOMODE && st != SB_E_CAPACITY) res->log_z = NAN;
  return st;
}

int32_t sb_exec_create(sb_exec **out) {
  if (!out) return fail(SB_E_INVAL, "out is NULL");
  *out = nullptr;
  int st = device_status();
  if (st) return st;
  ExecCtx *ex = new (std::nothrow) ExecCtx();
  if (!ex) return fail(SB_E_NOMEM, "out of host memory");
  (void)hipGetDevice(&ex->device);
  if (hipHostMalloc((void **)&ex->pinned, sizeof(int32_t) * 16, hipHostMallocDefault) !=
      hipSuccess) {
    delete ex;
    return fail(SB_E_NOMEM, "pinned host allocation failed");
  }
  ex->ev_ok = true;
  int made = 0;
  for (; made < 10; ++made)
    if (hipEventCreate(&ex->ev[made]) != hipSuccess) break;
  if (made < 10) {
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ex->ev[i]);
    (void)hipHostFree(ex->pinned);
    delete ex;
    return fail(SB_E_DEVICE, "event creation failed");
  }
  *out = reinterpret_cast<sb_exec *>(ex);
  return SB_OK;
}

void sb_exec_destroy(sb_exec *h) {
  ExecCtx *ex = reinterpret_cast<ExecCtx *>(h);
  if (!ex) return;
  for (int i = 0; i < ExecCtx::kSlots; ++i)
    if (ex->slot[i].exec) (void)hipGraphExecDestroy(ex->slot[i].exec);
  if (ex->ev_ok)
    for (int i = 0; i < 10; ++i) (void)hipEventDestroy(ex->ev[i]);
  if (ex->pinned) (void)hipHostFree(ex->pinned);
  delete ex;
}

int32_t sb_exec_stats(const sb_exec *h, int32_t *counts) {
  const ExecCtx *ex = reinterpret_cast<const ExecCtx *>(h);
  if (!ex || !counts) return fail(SB_E_INVAL, "bad arguments");
  counts[0] = ex->n_capture;
  counts[1] = ex->n_instantiate;
  counts[2] = ex->n_update;
  counts[3] = ex->n_launch;
  return SB_OK;
}

int32_t sb_evidence_exec_dev(sb_exec *h, const sb_loglik *ll, const sb_box *box,
                             const sb_config *cfg, sb_result *res, void *workspace,
                             size_t ws_bytes, void *stream) {
  if (!h) {
    if (res) res->log_z = NAN;
    return fail(SB_E_INVAL, "execution context is NULL");
  }
  return evidence_dev(ll, box, cfg, res, workspace, ws_bytes, stream,
                      reinterpret_cast<ExecCtx *>(h));
}

int32_t sb_evidence(const sb_loglik *ll, const sb_box *box, const sb_config *cfg,
                    sb_result *res) {
  int st = validate_shape(ll);
  if (!st) st = validate_cfg(ll, cfg);
  if (!st && !box) st = fail(SB_E_INVAL, "box is NULL");
  if (!st) st = validate_box_host(ll->d, box->lo, box->hi);
  if (!st && !res) st = fail(SB_E_INVAL, "result is NULL");
  if (!st) st = validate_arrays_host(ll);
  if (st) {
    if (res) res->log_z = NAN;
    return st;
  }
  if ((st = device_status())) {
    res->log_z = NAN;
    return st;
  }
  const int64_t d = ll->d, K = ll->K;
  const size_t n_prob = align_up(8 * K) + align_up(8 * K * d) + align_up(8 * K * d * d) +
                        2 * align_up(8 * d);
  const size_t ws = evidence_ws_bytes(ll, cfg);
  DevBuf buf;
  if (hipMalloc(&buf.p, n_prob + ws) != hipSuccess) {
    res->log_z = NAN;
    return fail(SB_E_NOMEM, "hipMalloc of %zu bytes failed", n_prob + ws);
  }
  char *p = (char *)buf.p;
  double *lw = (double *)p;
  p += align_up(8 * K);
  double *mu = (double *)p;
  p += align_up(8 * K * d);
  double *prec = (double *)p;
  p += align_up(8 * K * d * d);
  double *lo = (double *)p;
  p += align_up(8 * d);
  double *hi = (double *)p;
  p += align_up(8 * d);
  hipStream_t s;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    res->log_z = NAN;
    return fail(SB_E_DEVICE, "stream creation failed");
  }
  bool ok = true;
  if (ll->log_w) ok &= hipMemcpyAsync(lw, ll->log_w, 8 * K, hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(mu, ll->mu, 8 * K * d, hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(prec, ll->prec, 8 * K * d * d, hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(lo, box->lo, 8 * d, hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(hi, box->hi, 8 * d, hipMemcpyHostToDevice, s) == hipSuccess;
  if (!ok) {
    (void)hipStreamDestroy(s);
    res->log_z = NAN;
    return fail(SB_E_DEVICE, "host-to-device copy failed");
  }
  DevProblem P;
  P.family = ll->family;
  P.norm = ll->norm;
  P.d = ll->d;
  P.K = ll->K;
  P.log_w = ll->log_w ? lw : nullptr;
  P.mu = mu;
  P.prec = prec;
  P.lo = lo;
  P.hi = hi;
  P.nu = ll->nu;
  P.c = ll->logl_offset;
  // a host entry point may allocate: a context of its own for the graphs,
  // the pinned readback word and the phase timing
  sb_exec *ex = nullptr;
  if ((st = sb_exec_create(&ex))) {
    (void)hipStreamDestroy(s);
    res->log_z = NAN;
    return st;
  }
  st = run_evidence(P, cfg, res, p, ws, s, reinterpret_cast<ExecCtx *>(ex));
  (void)hipStreamSynchronize(s);
  sb_exec_destroy(ex);
  (void)hipStreamDestroy(s);
  if (st && st != SB_E_NOMODE && st != SB_E_CAPACITY) res->log_z = NAN;
  return st;
}

int32_t sb_evidence_batch(int32_t n, const sb_loglik *ll, const sb_box *box,
                          const sb_config *cfg, sb_result *res) {
  if (n < 0 || (n > 0 && (!ll || !box || !cfg || !res)))
    return fail(SB_E_INVAL, "invalid batch arguments");
  if (n == 0) return SB_OK;
  for (int j = 0; j < n; ++j) res[j].log_z = NAN;
  for (int j = 0; j < n; ++j) {
    int st = validate_shape(&ll[j]);
    if (!st) st = validate_cfg(&ll[j], &cfg[j]);
    if (!st) st = validate_box_host(ll[j].d, box[j].lo, box[j].hi);
    if (!st) st = validate_arrays_host(&ll[j]);
    if (!st && (cfg[j].precision != cfg[0].precision || cfg[j].m != cfg[0].m))
      st = fail(SB_E_INVAL, "every problem of a batch needs the same precision and m");
    if (st) {
      char msg[512];
      snprintf(msg, sizeof(msg), "problem %d: %s", j, sb::last_error());
      return fail(st, "%s", msg);
    }
  }
  int st = device_status();
  if (st) return st;
  hipStream_t s;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
    return fail(SB_E_DEVICE, "stream creation failed");
  st = sb::run_evidence_batch(n, ll, box, cfg, res, s);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return st;
}

// ------------------------------------------------------------------ prep
size_t sb_prep_workspace_bytes(int32_t d, int32_t K) {
  if (d < 1 || K < 1) return 0;
  return align_up(8ull * K * d * d) + 4 * align_up(8ull * K) + align_up(64) + 1024;
}

int32_t sb_prep_dev(const sb_loglik *ll, double *beta, double *logdet_prec, float *prec_f32,
                    uint16_t *prec_bf16, float *mu_f32, void *workspace, size_t ws_bytes,
                    void *stream) {
  int st = validate_shape(ll);
  if (st) return st;
  if (!beta || !logdet_prec) return fail(SB_E_INVAL, "beta and logdet_prec must not be NULL");
  if (!workspace || ws_bytes < sb_prep_workspace_bytes(ll->d, ll->K))
    return fail(SB_E_NOMEM, "prep workspace too small");
  if ((st = device_status())) return st;
  hipStream_t s = (hipStream_t)stream;
  const int d = ll->d, K = ll->K;
  Arena ar(workspace, ws_bytes);
  double *Lp = ar.take<double>((size_t)K * d * d);
  double *mx = ar.take<double>(K);
  int32_t *info = ar.take<int32_t>(K);
  int32_t *flags = ar.take<int32_t>(16);
  Model m;
  m.family = ll->family;
  m.norm = ll->norm;
  m.d = d;
  m.K = K;
  m.mu64 = ll->mu;
  m.P64 = ll->prec;
  m.nu = ll->nu;
  m.c = ll->logl_offset;
  if ((st = launch_fill_i32(16, 0, flags, s))) return st;
  if ((st = launch_symmetry_check(ll->prec, K, d, mx, flags, s))) return st;
  if ((st = chol_batched(K, d, ll->prec, Lp, info, s))) return st;
  if ((st = launch_logdet(K, d, Lp, info, logdet_prec, s))) return st;
  if ((st = launch_beta(m, ll->log_w, logdet_prec, beta, s))) return st;
  if (prec_f32 || prec_bf16 || mu_f32) {
    if ((st = launch_convert_model(m, prec_f32, (bf16_t *)prec_bf16, mu_f32, s))) return st;
  }
  std::vector<int32_t> hinfo(K);
  int32_t hflag = 0;
  if (hipMemcpyAsync(&hflag, flags, 4, hipMemcpyDeviceToHost, s) ||
      hipMemcpyAsync(hinfo.data(), info, 4 * K, hipMemcpyDeviceToHost, s) ||
      hipStreamSynchronize(s))
    return fail(SB_E_DEVICE, "prep readback failed");
  if (hflag) return fail(SB_E_NOTPD, "precision matrix is not symmetric to 1e-12 relative");
  for (int k = 0; k < K; ++k)
    if (hinfo[k]) return fail(SB_E_NOTPD, "precision matrix %d is not positive definite", k);
  return SB_OK;
}

// ------------------------------------------------------------- logl + grad
size_t sb_logl_grad_workspace_bytes(int32_t d, int32_t K, int64_t B, int32_t dtype) {
  if (d < 1 || K < 1 || B < 0) return 0;
  return eval_bytes(dtype == SB_DTYPE_F64 ? SB_DTYPE_F64 : SB_DTYPE_F32, d, K, B, false);
}

// The contraction and epilogue of sb_logl_grad_dev with Y and the q partials
// carved from `scratch`; tune: time the tile candidates on this launch's
// operands (first call per shape), else the cached choice or the heuristic.
static int32_t logl_grad_core(const sb_model_dev *mdl, int64_t B, const void *X, void *logl,
                              void *grad, int32_t dtype, void *scratch, size_t scratch_bytes,
                              bool tune, void *stream) {
  int st;
  Model m = model_for(mdl, dtype);
  {
    ASrc a;
    a.kind = 0;
    a.X = X;
    a.ldx = m.d;
    // small FP64 problems: contraction and epilogue in one launch, no scratch
    if (dtype == SB_DTYPE_F64 && fused_logl_grad_ok(m, a))
      return launch_fused_logl_grad(m, a, B, nullptr, nullptr, (double *)logl, (double *)grad,
                                    m.d, nullptr, (hipStream_t)stream);
  }
  const size_t es = dtype == SB_DTYPE_F64 ? 8 : 4;
  Arena ar(scratch, scratch_bytes);
  void *Y = ar.take<char>(es * (size_t)B * m.K * m.d);
  void *qp = ar.take<char>(es * (size_t)B * m.K * ceil_div(m.d, 64));
  if (!ar.ok() || !Y || !qp) return fail(SB_E_NOMEM, "scratch too small");
  ASrc a;
  a.kind = 0;
  a.X = X;
  a.ldx = m.d;
  // a single Gaussian's gradient is -Y: the contraction stores it straight
  // into grad and the epilogue forms l only
  const bool direct = grad && m.K == 1 && m.family == SB_FAMILY_GAUSS_MIX;
  QuadOut o;
  o.Y = direct ? grad : Y;
  o.ldy = direct ? (int64_t)m.d : (int64_t)m.K * m.d;
  o.yneg = direct;
  o.qpart = qp;
  const TuneProbe pr{a, o};
  TileCfg t = autotune_tiles(dtype, m, B, (hipStream_t)stream, tune ? &pr : nullptr, false);
  if ((st = launch_quad_gemm(dtype, m, a, B, nullptr, o, t, (hipStream_t)stream))) return st;
  FinishArgs f;
  f.M = B;
  f.qpart = qp;
  f.ntn = o.ntn;
  f.Y = direct ? nullptr : Y;
  f.ldy = o.ldy;
  f.logl = logl;
  f.grad = direct ? nullptr : grad;
  f.ldg = m.d;
  return launch_finish(dtype, m, f, (hipStream_t)stream);
}

int32_t sb_logl_grad_dev(const sb_model_dev *mdl, int64_t B, const void *X, void *logl,
                         void *grad, int32_t dtype, void *workspace, size_t ws_bytes,
                         void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  if (B < 0 || (B > 0 && (!X || !logl))) return fail(SB_E_INVAL, "bad B / X / logl");
  if ((st = check_gemm_dtype(mdl, dtype))) return st;
  if (B == 0) return SB_OK;
  if (!workspace || ws_bytes < sb_logl_grad_workspace_bytes(mdl->d, mdl->K, B, dtype))
    return fail(SB_E_NOMEM, "workspace too small");
  if ((st = device_status())) return st;
  return logl_grad_core(mdl, B, X, logl, grad, dtype, workspace, ws_bytes, true, stream);
}

int32_t sb_logl_grad_noalloc_dev(const sb_model_dev *mdl, int64_t B, const void *X, void *logl,
                                 void *grad, int32_t dtype, void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  if (B < 0 || (B > 0 && (!X || !logl))) return fail(SB_E_INVAL, "bad B / X / logl");
  if ((st = check_gemm_dtype(mdl, dtype))) return st;
  if (B == 0) return SB_OK;
  const size_t need = sb_logl_grad_workspace_bytes(mdl->d, mdl->K, B, dtype);
  if (need > kStaticScratchBytes)
    return fail(SB_E_NOMEM,
                "B = %lld points need %zu bytes of scratch, beyond the static %zu bytes",
                (long long)B, need, kStaticScratchBytes);
  if ((st = device_status())) return st;
  void *p = nullptr;
  if ((st = scratch_address(&p))) return st;
  return logl_grad_core(mdl, B, X, logl, grad, dtype, p, kStaticScratchBytes, false, stream);
}

size_t sb_reduced_logl_workspace_bytes(int32_t d, int32_t K, int64_t B) {
  if (d < 1 || K < 1 || B < 0) return 0;
  return 2 * align_up(8 * (size_t)B * d) + sb_logl_grad_workspace_bytes(d, K, B, SB_DTYPE_F64);
}

int32_t sb_reduced_logl_dev(const sb_model_dev *mdl, const double *theta_star, const double *V,
                            int32_t ldv, int32_t r, int64_t B, const double *phi, double *logl,
                            double *grad_phi, void *workspace, size_t ws_bytes, void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  const int d = mdl->d;
  if (r < 0 || r > d || ldv < (r > 0 ? r : 1) || B < 0 ||
      (B > 0 && (!theta_star || !logl || (r > 0 && (!V || !phi)))))
    return fail(SB_E_INVAL, "bad r / ldv / B / arrays");
  if ((st = check_gemm_dtype(mdl, SB_DTYPE_F64))) return st;
  if (B == 0) return SB_OK;
  if (!workspace || ws_bytes < sb_reduced_logl_workspace_bytes(d, mdl->K, B))
    return fail(SB_E_NOMEM, "workspace too small");
  if ((st = device_status())) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar(workspace, ws_bytes);
  double *X = ar.take<double>((size_t)B * d);
  double *G = ar.take<double>((size_t)B * d);
  const size_t rest = sb_logl_grad_workspace_bytes(d, mdl->K, B, SB_DTYPE_F64);
  char *lw = ar.take<char>(rest);
  if (!ar.ok()) return fail(SB_E_NOMEM, "workspace too small");
  // theta = theta* + V_inform phi: X[b][j] = theta*_j + sum_i phi[b][i] V[j][i]
  if ((st = launch_small_gemm_f64(B, d, r, phi, r, V, 1, ldv, theta_star, X, d, s))) return st;
  if ((st = logl_grad_core(mdl, B, X, logl, grad_phi ? G : nullptr, SB_DTYPE_F64, lw, rest, true,
                           stream)))
    return st;
  // grad_phi[b][i] = sum_j grad[b][j] V[j][i]
  if (grad_phi && r > 0)
    return launch_small_gemm_f64(B, r, d, G, d, V, ldv, 1, nullptr, grad_phi, r, s);
  return SB_OK;
}

int32_t sb_reduced_bounds_dev(int32_t d, const double *theta_star, const double *V, int32_t ldv,
                              int32_t r, const double *lo, const double *hi, double *phi_lo,
                              double *phi_hi, void *stream) {
  if (d < 1 || r < 0 || r > d || ldv < (r > 0 ? r : 1) ||
      (r > 0 && (!theta_star || !V || !lo || !hi || !phi_lo || !phi_hi)))
    return fail(SB_E_INVAL, "bad d / r / ldv / arrays");
  if (r == 0) return SB_OK;
  int st = device_status();
  if (st) return st;
  return launch_reduced_bounds(d, theta_star, V, ldv, r, lo, hi, phi_lo, phi_hi,
                               (hipStream_t)stream);
}

int32_t sb_quadform_dev(const sb_model_dev *mdl, int64_t B, const void *X, int32_t dtype, void *Y,
                        void *qpart, int32_t *n_tiles, void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  if (B < 0 || (B > 0 && (!X || !Y || !qpart))) return fail(SB_E_INVAL, "bad B / X / Y / qpart");
  if ((st = check_gemm_dtype(mdl, dtype))) return st;
  if ((st = device_status())) return st;
  Model m = model_for(mdl, dtype);
  ASrc a;
  a.kind = 0;
  a.X = X;
  a.ldx = m.d;
  QuadOut o;
  o.Y = Y;
  o.ldy = (int64_t)m.K * m.d;
  o.qpart = qpart;
  const TuneProbe pr{a, o};
  TileCfg t = autotune_tiles(dtype, m, B, (hipStream_t)stream, &pr);
  st = launch_quad_gemm(dtype, m, a, B, nullptr, o, t, (hipStream_t)stream);
  if (n_tiles) *n_tiles = o.ntn;
  return st;
}

int32_t sb_quadform_pairs_dev(const sb_model_dev *mdl, int64_t B, const void *X,
                              const int32_t *gcnt, const int32_t *rows, int64_t cap, void *Y,
                              void *qpart, int32_t *n_tiles, void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  if (B < 0 || cap < 0 || (cap > 0 && (!X || !Y || !qpart || !gcnt || !rows)))
    return fail(SB_E_INVAL, "bad B / cap / arrays");
  if ((st = check_gemm_dtype(mdl, SB_DTYPE_F32_SPLIT))) return st;
  if (mdl->family != SB_FAMILY_GAUSS_MIX)
    return fail(SB_E_UNSUPPORTED, "pairs: Gaussian mixtures only");
  if ((st = device_status())) return st;
  if (cap == 0) return SB_OK;
  Model m = model_for(mdl, SB_DTYPE_F32_SPLIT);
  ASrc a;
  a.kind = 0;
  a.X = X;
  a.ldx = m.d;
  a.rowmap = rows;
  a.rows = B;
  QuadOut o;
  o.Y = Y;
  o.ldy = (int64_t)m.K * m.d;
  o.ymap = rows;
  o.gcnt = gcnt;
  o.gcap = cap;
  o.qpart = qpart;
  TileCfg t;  // 128 x 128 (SB_TILE2 overrides it, for measurement)
  (void)parse_tile(getenv("SB_TILE2"), &t);
  st = launch_quad_gemm(DT_F32S, m, a, cap, nullptr, o, t, (hipStream_t)stream);
  if (n_tiles) *n_tiles = o.ntn;
  return st;
}

int32_t sb_split_bf16_dev(int64_t n, const double *x, uint16_t *hi, uint16_t *lo, void *stream) {
  if (n < 0 || (n > 0 && (!x || !hi))) return fail(SB_E_INVAL, "bad n / x / hi");
  if (n == 0) return SB_OK;
  int st = device_status();
  if (st) return st;
  return launch_split_bf16(n, x, hi, lo, (hipStream_t)stream);
}

// ------------------------------------------------------------------- HVP
size_t sb_hvp_workspace_bytes(int32_t d, int32_t K, int64_t B) {
  if (d < 1 || K < 1 || B < 0) return 0;
  return 2 * eval_bytes(SB_DTYPE_F64, d, K, B, false);
}

int32_t sb_hvp_dev(const sb_model_dev *mdl, int64_t B, const double *X, const double *V,
                   double *HV, void *workspace, size_t ws_bytes, void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  if (B < 0 || (B > 0 && (!X || !V || !HV))) return fail(SB_E_INVAL, "bad B / X / V / HV");
  if (B == 0) return SB_OK;
  if (!workspace || ws_bytes < sb_hvp_workspace_bytes(mdl->d, mdl->K, B))
    return fail(SB_E_NOMEM, "workspace too small");
  if ((st = device_status())) return st;
  hipStream_t s = (hipStream_t)stream;
  Model m = model_from(mdl);
  Arena ar(workspace, ws_bytes);
  double *Y = ar.take<double>((size_t)B * m.K * m.d);
  double *Z = ar.take<double>((size_t)B * m.K * m.d);
  double *qp = ar.take<double>((size_t)B * m.K * ceil_div(m.d, 64));
  double *qz = ar.take<double>((size_t)B * m.K * ceil_div(m.d, 64));
  ASrc a;
  a.kind = 0;
  a.X = X;
  a.ldx = m.d;
  QuadOut o;
  o.Y = Y;
  o.ldy = (int64_t)m.K * m.d;
  o.qpart = qp;
  const TuneProbe pr{a, o};
  TileCfg t = autotune_tiles(SB_DTYPE_F64, m, B, s, &pr);
  if ((st = launch_quad_gemm(SB_DTYPE_F64, m, a, B, nullptr, o, t, s))) return st;
  ASrc av = a;
  av.X = V;
  av.zero_mu = true;
  QuadOut oz;
  oz.Y = Z;
  oz.ldy = o.ldy;
  oz.qpart = qz;
  if ((st = launch_quad_gemm(SB_DTYPE_F64, m, av, B, nullptr, oz, t, s))) return st;
  HvpArgs h;
  h.M = B;
  h.qpart = qp;
  h.ntn = o.ntn;
  h.Y = Y;
  h.Z = Z;
  h.ldy = o.ldy;
  h.V = V;
  h.HV = HV;
  return launch_hvp_finish(m, h, s);
}

// ------------------------------------------------------------- discovery
size_t sb_discover_workspace_bytes(int32_t d, int32_t K, int32_t R, int32_t n_pts, int32_t dtype) {
  if (d < 1 || K < 1 || R < 1 || n_pts < 1) return 0;
  const int64_t NP = (int64_t)R * n_pts;
  const size_t es = dtype == SB_DTYPE_F64 ? 8 : 4;
  return 2 * align_up(8ull * R * d) + 2 * align_up(4ull * R * d) + align_up(es * NP) +
         align_up(es * (size_t)NP * K * ceil_div(d, 64)) + 2048;
}

int32_t sb_discover_dev(const sb_model_dev *mdl, const double *lo, const double *hi, int32_t R,
                        int32_t n_pts, int32_t n_starts, uint64_t seed, int32_t dtype, double *P0,
                        double *P1, double *ray_best_l, int32_t *ray_best_j, int32_t *start_ray,
                        double *X0, void *workspace, size_t ws_bytes, void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  if (!lo || !hi || !ray_best_l || !ray_best_j || !start_ray || !X0)
    return fail(SB_E_INVAL, "NULL output");
  if (R < 1 || n_pts < 1 || n_starts < 1 || n_starts > R)
    return fail(SB_E_INVAL, "need R, n_pts >= 1 and 1 <= n_starts <= R");
  if (dtype != SB_DTYPE_F64 && dtype != SB_DTYPE_BF16)
    return fail(SB_E_INVAL, "discovery dtype must be F64 or BF16");
  if (dtype == SB_DTYPE_BF16 && (!mdl->prec_lp || !mdl->mu_lp))
    return fail(SB_E_INVAL, "BF16 needs prec_lp (BF16) and mu_lp");
  if (!workspace || ws_bytes < sb_discover_workspace_bytes(mdl->d, mdl->K, R, n_pts, dtype))
    return fail(SB_E_NOMEM, "workspace too small");
  if ((st = device_status())) return st;
  hipStream_t s = (hipStream_t)stream;
  Model m = model_from(mdl);
  const int d = m.d;
  const int64_t NP = (int64_t)R * n_pts;
  const size_t es = dtype == SB_DTYPE_F64 ? 8 : 4;
  Arena ar(workspace, ws_bytes);
  double *p0 = ar.take<double>((size_t)R * d), *p1 = ar.take<double>((size_t)R * d);
  float *p0f = ar.take<float>((size_t)R * d), *p1f = ar.take<float>((size_t)R * d);
  void *lpts = ar.take<char>(es * NP);
  void *qp = ar.take<char>(es * (size_t)NP * m.K * ceil_div(d, 64));
  if (P0) p0 = P0;
  if (P1) p1 = P1;
  const bool bf = dtype == SB_DTYPE_BF16;
  if ((st = launch_rays(d, lo, hi, R, seed, 0u, p0, p1, bf ? p0f : nullptr, bf ? p1f : nullptr,
                        s)))
    return st;
  if (bf && n_pts > 3 && quad_gemm_bf16_ok(d)) {
    // BF16: the contraction at three nodes per ray, the samples by interpolation
    if ((st = discover_bf16_nodes(m, p0f, p1f, R, n_pts, (float *)qp, (float *)lpts, s)))
      return st;
  } else {
    ASrc a;
    a.kind = 1;
    a.P0 = bf ? (const void *)p0f : (const void *)p0;
    a.P1 = bf ? (const void *)p1f : (const void *)p1;
    a.n_pts = n_pts;
    QuadOut o;
    o.Y = nullptr;
    o.ldy = (int64_t)m.K * d;
    o.qpart = qp;
    const TuneProbe pr{a, o};
    TileCfg t = autotune_tiles(dtype, m, NP, s, &pr);
    if ((st = launch_quad_gemm(dtype, m, a, NP, nullptr, o, t, s))) return st;
    FinishArgs f;
    f.M = NP;
    f.qpart = qp;
    f.ntn = o.ntn;
    f.logl = lpts;
    if ((st = launch_finish(bf ? SB_DTYPE_F32 : SB_DTYPE_F64, m, f, s))) return st;
  }
  if ((st = launch_ray_argmax(R, n_pts, bf ? SB_DTYPE_F32 : SB_DTYPE_F64, lpts, ray_best_l,
                              ray_best_j, s)))
    return st;
  if ((st = launch_topn(R, n_starts, ray_best_l, start_ray, s))) return st;
  return launch_gather_starts(d, n_pts, n_starts, start_ray, ray_best_j, p0, p1, X0, s);
}

// ---------------------------------------------------------- preprocessing
size_t sb_precheck_workspace_bytes(int32_t d, int32_t K) {
  if (d < 1 || K < 1) return 0;
  return precheck_ws_bytes(d, K);
}

int32_t sb_precheck_dev(const sb_model_dev *mdl, const double *lo, const double *hi,
                        double eps_flat, double eps_soft, double *s, int32_t *cls,
                        double *logz_marginal, int32_t *n_flagged, void *workspace,
                        size_t ws_bytes, void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  if (!lo || !hi || !s || !cls || !logz_marginal) return fail(SB_E_INVAL, "NULL argument");
  if (!(eps_flat >= 0.0) || !(eps_soft >= 0.0))
    return fail(SB_E_INVAL, "thresholds must be >= 0 (0: the defaults)");
  if (!workspace || ws_bytes < sb_precheck_workspace_bytes(mdl->d, mdl->K))
    return fail(SB_E_NOMEM, "workspace too small");
  if ((st = device_status())) return st;
  Model m = model_from(mdl);
  int32_t counts[4] = {0, 0, 0, 0};
  st = run_precheck(m, lo, hi, eps_flat > 0.0 ? eps_flat : 1e-6, eps_soft > 0.0 ? eps_soft : 1e-3,
                    s, cls, logz_marginal, counts, workspace, ws_bytes, (hipStream_t)stream);
  if (st) return st;
  if (n_flagged) {
    n_flagged[0] = counts[1];
    n_flagged[1] = counts[2];
  }
  if (counts[3]) return fail(SB_E_INVAL, "non-finite likelihood at %d probe coordinates", counts[3]);
  return SB_OK;
}

// ------------------------------------------------- reduction at the modes
size_t sb_eig_reduce_workspace_bytes(int32_t C, int32_t n) {
  if (C < 1 || n < 1) return 0;
  return reduce_ws_bytes(C, n);
}

int32_t sb_eig_reduce_dev(int32_t C, int32_t n, const double *H, const double *lo,
                          const double *hi, double eps_inform, double eps_nuisance,
                          double *eigval, double *V, int32_t *cls, double *logz_marginal,
                          int32_t *d_eff, int32_t *sweeps, void *workspace, size_t ws_bytes,
                          void *stream) {
  if (C < 1 || n < 1 || !H || !lo || !hi || !eigval || !V || !cls || !logz_marginal)
    return fail(SB_E_INVAL, "bad eigen-reduction arguments");
  if (!(eps_nuisance >= 0.0) || !(eps_inform >= eps_nuisance) || !std::isfinite(eps_inform))
    return fail(SB_E_INVAL, "need 0 <= eps_nuisance <= eps_inform < inf");
  if (!workspace || ws_bytes < sb_eig_reduce_workspace_bytes(C, n))
    return fail(SB_E_NOMEM, "workspace too small");
  int st = device_status();
  if (st) return st;
  return run_eig_reduce(C, n, H, lo, hi, eps_inform, eps_nuisance, eigval, V, cls, logz_marginal,
                        d_eff, sweeps, workspace, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------- L-BFGS
int32_t sb_lbfgs_direction_dev(int64_t B, int32_t d, int32_t m, const int32_t *cnt,
                               const void *S, const void *Y, const void *G, void *P,
                               int32_t dtype, void *stream) {
  if (B < 0 || d < 1 || m < 1 || (B > 0 && (!cnt || !S || !Y || !G || !P)))
    return fail(SB_E_INVAL, "bad two-loop arguments");
  if (dtype != SB_DTYPE_F64 && dtype != SB_DTYPE_F32)
    return fail(SB_E_INVAL, "dtype must be F64 or F32");
  if (m > kMaxMem) return fail(SB_E_INVAL, "m must be in [1, %d]", kMaxMem);
  if (B == 0) return SB_OK;
  int st = device_status();
  if (st) return st;
  return launch_two_loop(B, d, m, cnt, S, Y, G, P, dtype, (hipStream_t)stream);
}

size_t sb_lbfgs_workspace_bytes(int32_t d, int32_t K, int64_t B, int32_t m, int32_t dtype) {
  if (d < 1 || K < 1 || B < 1 || m < 1) return 0;
  const int dt = dtype == SB_DTYPE_F64 ? SB_DTYPE_F64 : SB_DTYPE_F32;
  return lbfgs_state_bytes(dt, B, d, m) + eval_bytes(dt, d, K, B, false) + 4096;
}

// The loop of sb_lbfgs_dev; with n_timed > 0 it records HIP events around
// each of the first n_timed step launches and synchronises after each step.
static int32_t lbfgs_run(const sb_model_dev *mdl, int64_t B, void *X, int32_t m,
                         int32_t max_iter, double grad_tol, int32_t dtype, void *logl,
                         void *grad, int32_t *status, int32_t *iters, int64_t *n_evals,
                         void *workspace, size_t ws_bytes, void *stream, int32_t n_timed,
                         float *step_us, int32_t *step_rows, int32_t *step_full,
                         int32_t *step_back, double *step_bytes) {
  int st = validate_model(mdl);
  if (st) return st;
  if (B < 1 || !X) return fail(SB_E_INVAL, "bad B / X");
  if (m < 1 || m > kMaxMem) return fail(SB_E_INVAL, "m must be in [1, %d]", kMaxMem);
  if (dtype != SB_DTYPE_F64 && dtype != SB_DTYPE_F32 && dtype != SB_DTYPE_F32_H16)
    return fail(SB_E_INVAL, "dtype must be F64, F32 or F32_H16");
  const bool h16 = dtype == SB_DTYPE_F32_H16;
  if (h16 && m > kMaxHist)
    return fail(SB_E_UNSUPPORTED, "F32_H16 (BF16 history) needs m <= %d", kMaxHist);
  if (h16) dtype = SB_DTYPE_F32;
  if (dtype == SB_DTYPE_F32 && (!mdl->prec_lp || !mdl->mu_lp))
    return fail(SB_E_INVAL, "F32 needs prec_lp (FP32) and mu_lp");
  if (!workspace || ws_bytes < sb_lbfgs_workspace_bytes(mdl->d, mdl->K, B, m, dtype))
    return fail(SB_E_NOMEM, "workspace too small");
  if ((st = device_status())) return st;
  hipStream_t s = (hipStream_t)stream;
  Model md = model_from(mdl);
  const int d = md.d;
  Arena ar(workspace, ws_bytes);
  LbfgsBuffers lb;
  lb.dtype = dtype;
  lb.hist_bf16 = h16;
  lb.B = B;
  lb.d = d;
  lb.m = m;
  if ((st = lbfgs_carve(ar, lb))) return fail(st, "workspace too small");
  const size_t es = dtype == SB_DTYPE_F64 ? 8 : 4;
  void *Y = ar.take<char>(es * (size_t)B * md.K * d);
  void *qp = ar.take<char>(es * (size_t)B * md.K * ceil_div(d, 64));
  if ((st = launch_lbfgs_init(lb, X, s))) return st;
  TuneProbe pr;
  pr.a.kind = 0;
  pr.a.X = lb.X;  // slot 0 holds the start points now
  pr.a.ldx = d;
  pr.o.Y = Y;
  pr.o.ldy = (int64_t)md.K * d;
  pr.o.qpart = qp;
  TileCfg t = autotune_tiles(dtype, md, B, s, &pr);
  auto eval = [&](const int32_t *rowmap, const int32_t *count) -> int {
    ASrc a;
    a.kind = 0;
    a.X = lb.X;
    a.ldx = d;
    a.rowmap = rowmap;
    a.rows = 2 * B;  // both slots
    QuadOut o;
    o.Y = Y;
    o.ldy = (int64_t)md.K * d;
    o.qpart = qp;
    int r = launch_quad_gemm(dtype, md, a, B, count, o, t, s);
    if (r) return r;
    FinishArgs f;
    f.M = B;
    f.count = count;
    f.outmap = rowmap;
    f.qpart = qp;
    f.ntn = o.ntn;
    f.Y = Y;
    f.ldy = o.ldy;
    f.logl = lb.F;
    f.logl_f64 = true;
    f.grad = lb.G;
    f.ldg = d;
    return launch_finish(dtype, md, f, s);
  };
  if ((st = eval(nullptr, nullptr))) return st;
  const int mi = max_iter > 0 ? max_iter : 10 * d + 200;
  const double tol = grad_tol > 0 ? grad_tol : 1e-10;
  int32_t hcount = 1;
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<int32_t> h_st, h_ls, h_cnt, p_st, p_cnt;
  if (n_timed > 0) {
    for (int i = 0; i < n_timed; ++i) {
      step_us[i] = 0.f;
      step_rows[i] = 0;
      step_full[i] = step_back[i] = 0;
      if (step_bytes) step_bytes[i] = -1.0;
    }
    h_st.resize(B);
    h_ls.resize(B);
    h_cnt.resize(B);
    p_st.assign(B, 0);  // every start active, no history, before the first step
    p_cnt.assign(B, 0);
    if (hipEventCreate(&ev[0]) || hipEventCreate(&ev[1])) {
      if (ev[0]) hipEventDestroy(ev[0]);
      return fail(SB_E_DEVICE, "event creation failed");
    }
  }
  int32_t rows = (int32_t)B;  // starts active entering the next step
  for (int64_t step = 0; step < 42ll * mi + 64 && hcount > 0; ++step) {
    const bool timed = step < n_timed;
    if (timed && hipEventRecord(ev[0], s)) st = fail(SB_E_DEVICE, "event record failed");
    if (!st) st = launch_lbfgs_step(lb, mi, tol, s);
    if (!st && timed && hipEventRecord(ev[1], s)) st = fail(SB_E_DEVICE, "event record failed");
    if (!st) st = launch_compact(lb, s);
    if (!st) st = eval(lb.idx, lb.count);
    if (!st && timed) {
      float ms = 0.f;
      if (hipMemcpyAsync(&hcount, lb.count, 4, hipMemcpyDeviceToHost, s) ||
          hipStreamSynchronize(s) || hipEventElapsedTime(&ms, ev[0], ev[1]))
        st = fail(SB_E_DEVICE, "step timing readback failed");
      step_us[step] = 1e3f * ms;
      step_rows[step] = rows;
      // after the step: starts that accepted their trial and hold a full
      // history ring, and starts that halved their step (still active)
      if (!st && rows > 0) {
        if (hipMemcpy(h_st.data(), lb.status, 4 * B, hipMemcpyDeviceToHost) ||
            hipMemcpy(h_ls.data(), lb.ls, 4 * B, hipMemcpyDeviceToHost) ||
            hipMemcpy(h_cnt.data(), lb.cnt, 4 * B, hipMemcpyDeviceToHost))
          st = fail(SB_E_DEVICE, "step state readback failed");
        int32_t nf = 0, nb = 0;
        for (int64_t i = 0; !st && i < B; ++i) {
          if (h_st[i] != 0) continue;
          if (h_ls[i] > 0)
            ++nb;
          else if (h_cnt[i] == m)
            ++nf;
        }
        step_full[step] = nf;
        step_back[step] = nb;
        // algorithmic bytes of the launch, when every start active entering it
        // accepted or halved (the first step, a reset (history cleared) or a
        // stop in it leave the entry at -1): a halving start reads the point
        // and direction and writes the trial point (3 d); an accepting start
        // with c pairs in its ring reads them, x and g at both slots, and
        // writes the direction and the trial point, plus s and y when the
        // curvature test stores the new pair (2 c + 6 (+ 2)) d; with the ring
        // full the pair the new one evicts is read only when the new one is
        // kept out, so (2 m + 6) d either way
        if (step_bytes && !st && step > 0) {
          // (d-vectors of the dtype; ring pairs of the ring's element type)
          const double vec = (double)d * (dtype == SB_DTYPE_F64 ? 8.0 : 4.0);
          const double rv = h16 ? (double)d * 2.0 : vec;
          double bytes = 0.0;
          bool exact = true;
          for (int64_t i = 0; i < B && exact; ++i) {
            if (p_st[i] != 0) continue;  // stopped before this step
            if (h_st[i] != 0 || (h_ls[i] == 0 && h_cnt[i] < p_cnt[i])) {
              exact = false;
            } else if (h_ls[i] > 0) {
              bytes += 3.0 * vec;
            } else if (p_cnt[i] == m) {
              bytes += 2.0 * m * rv + 6.0 * vec;
            } else {
              bytes += (2.0 * p_cnt[i] + (h_cnt[i] > p_cnt[i] ? 2.0 : 0.0)) * rv + 6.0 * vec;
            }
          }
          step_bytes[step] = exact ? bytes : -1.0;
        }
        p_st.swap(h_st);
        p_cnt.swap(h_cnt);
      }
      rows = hcount;
    } else if (!st && (step & 7) == 7) {
      if (hipMemcpyAsync(&hcount, lb.count, 4, hipMemcpyDeviceToHost, s) ||
          hipStreamSynchronize(s))
        st = fail(SB_E_DEVICE, "count readback failed");
    }
    if (st) break;
  }
  if (ev[0]) hipEventDestroy(ev[0]);
  if (ev[1]) hipEventDestroy(ev[1]);
  if (st) return st;
  if ((st = launch_lbfgs_gather(lb, X, logl, false, grad, status, iters, s))) return st;
  if (n_evals) {
    if (hipMemcpyAsync(n_evals, lb.evals, 8, hipMemcpyDeviceToHost, s) || hipStreamSynchronize(s))
      return fail(SB_E_DEVICE, "eval count readback failed");
  }
  return SB_OK;
}

int32_t sb_lbfgs_dev(const sb_model_dev *mdl, int64_t B, void *X, int32_t m, int32_t max_iter,
                     double grad_tol, int32_t dtype, void *logl, void *grad, int32_t *status,
                     int32_t *iters, int64_t *n_evals, void *workspace, size_t ws_bytes,
                     void *stream) {
  return lbfgs_run(mdl, B, X, m, max_iter, grad_tol, dtype, logl, grad, status, iters, n_evals,
                   workspace, ws_bytes, stream, 0, nullptr, nullptr, nullptr, nullptr, nullptr);
}

int32_t sb_lbfgs_timed_dev(const sb_model_dev *mdl, int64_t B, void *X, int32_t m,
                           int32_t max_iter, double grad_tol, int32_t dtype, void *logl,
                           void *grad, int32_t *status, int32_t *iters, int64_t *n_evals,
                           void *workspace, size_t ws_bytes, void *stream, int32_t n_timed,
                           float *step_us, int32_t *step_rows, int32_t *step_full,
                           int32_t *step_back, double *step_bytes) {
  if (n_timed < 0 || (n_timed > 0 && (!step_us || !step_rows || !step_full || !step_back)))
    return fail(SB_E_INVAL, "n_timed must be >= 0 with the four timing arrays given");
  return lbfgs_run(mdl, B, X, m, max_iter, grad_tol, dtype, logl, grad, status, iters, n_evals,
                   workspace, ws_bytes, stream, n_timed, step_us, step_rows, step_full,
                   step_back, step_bytes);
}

// ----------------------------------------------------------------- dedup
size_t sb_dedup_workspace_bytes(int32_t C) { return dedup_ws_bytes(C) + 1024; }

int32_t sb_dedup_dev(int32_t C, int32_t d, const void *X, const void *l, const uint8_t *valid,
                     double tau, int32_t dtype, int32_t *rep_of, int32_t *reps, int32_t max_reps,
                     int32_t *n_reps, void *workspace, size_t ws_bytes, void *stream) {
  if (C < 0 || d < 1 || (C > 0 && (!X || !l || !rep_of || !reps)) || max_reps < 1 || !n_reps)
    return fail(SB_E_INVAL, "bad dedup arguments");
  if (!(tau >= 0.0)) return fail(SB_E_INVAL, "tau must be >= 0");
  if (dtype != SB_DTYPE_F64 && dtype != SB_DTYPE_F32)
    return fail(SB_E_INVAL, "dtype must be F64 or F32");
  if (!workspace || ws_bytes < sb_dedup_workspace_bytes(C))
    return fail(SB_E_NOMEM, "workspace too small");
  int st = device_status();
  if (st) return st;
  Arena ar(workspace, ws_bytes);
  int n = 0;
  st = dedup_run(C, d, X, dtype, l, dtype, valid, tau, rep_of, reps, max_reps, &n, ar,
                 (hipStream_t)stream);
  *n_reps = n;
  if (st == SB_E_CAPACITY) set_error("%d representatives exceed max_reps = %d", n, max_reps);
  return st;
}

// --------------------------------------------------------------- Hessian
size_t sb_hessian_workspace_bytes(int32_t d, int32_t K, int32_t C) {
  if (d < 1 || K < 1 || C < 0) return 0;
  return eval_bytes(SB_DTYPE_F64, d, K, C, true) + align_up(8ull * C) + 1024;
}

int32_t sb_hessian_dev(const sb_model_dev *mdl, int32_t C, const double *X, double *H,
                       void *workspace, size_t ws_bytes, void *stream) {
  int st = validate_model(mdl);
  if (st) return st;
  if (C < 0 || (C > 0 && (!X || !H))) return fail(SB_E_INVAL, "bad C / X / H");
  if (C == 0) return SB_OK;
  if (!workspace || ws_bytes < sb_hessian_workspace_bytes(mdl->d, mdl->K, C))
    return fail(SB_E_NOMEM, "workspace too small");
  if ((st = device_status())) return st;
  hipStream_t s = (hipStream_t)stream;
  Model m = model_from(mdl);
  Arena ar(workspace, ws_bytes);
  double *Y = ar.take<double>((size_t)C * m.K * m.d);
  double *qp = ar.take<double>((size_t)C * m.K * ceil_div(m.d, 64));
  double *aux = ar.take<double>((size_t)C * m.K);
  double *G = ar.take<double>((size_t)C * m.d);
  double *l = ar.take<double>(C);
  ASrc a;
  a.kind = 0;
  a.X = X;
  a.ldx = m.d;
  QuadOut o;
  o.Y = Y;
  o.ldy = (int64_t)m.K * m.d;
  o.qpart = qp;
  const TuneProbe pr{a, o};
  TileCfg t = autotune_tiles(SB_DTYPE_F64, m, C, s, &pr);
  if ((st = launch_quad_gemm(SB_DTYPE_F64, m, a, C, nullptr, o, t, s))) return st;
  FinishArgs f;
  f.M = C;
  f.qpart = qp;
  f.ntn = o.ntn;
  f.Y = Y;
  f.ldy = o.ldy;
  f.logl = l;
  f.grad = G;
  f.ldg = m.d;
  f.aux = aux;
  if ((st = launch_finish(SB_DTYPE_F64, m, f, s))) return st;
  return launch_hessian_assemble(m, C, Y, o.ldy, aux, G, H, s);
}

// -------------------------------------------------------------- Cholesky
int32_t sb_cholesky_logdet_dev(int32_t C, int32_t n, const double *A, double *L, double *logdet,
                               int32_t *info, void *stream) {
  if (C < 0 || n < 1 || (C > 0 && (!A || !L || !logdet || !info)))
    return fail(SB_E_INVAL, "bad Cholesky arguments");
  if (C == 0) return SB_OK;
  int st = device_status();
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = chol_batched(C, n, A, L, info, s))) return st;
  return launch_logdet(C, n, L, info, logdet, s);
}

int32_t sb_cholesky_solve_dev(int32_t C, int32_t n, const double *L, const double *b, double *x,
                              void *stream) {
  if (C < 0 || n < 1 || (C > 0 && (!L || !b || !x))) return fail(SB_E_INVAL, "bad solve arguments");
  if (C == 0) return SB_OK;
  int st = device_status();
  if (st) return st;
  return launch_chol_solve(C, n, L, b, x, nullptr, (hipStream_t)stream);
}

// --------------------------------------------------------------- combine
int32_t sb_combine_dev(int32_t n, int32_t d, const double *lo, const double *hi,
                       const double *logl, const double *logdet, const double *modes,
                       int32_t *order, double *mode_log_z, double *log_z, void *stream) {
  if (n < 0 || d < 1 || !lo || !hi || !log_z ||
      (n > 0 && (!logl || !logdet || !modes || !order || !mode_log_z)))
    return fail(SB_E_INVAL, "bad combine arguments");
  int st = device_status();
  if (st) return st;
  return launch_combine(n, d, lo, hi, logl, logdet, modes, order, mode_log_z, log_z,
                        (hipStream_t)stream);
}

}  // extern "C"
