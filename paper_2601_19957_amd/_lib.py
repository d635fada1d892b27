"""ctypes binding of libsb.so (the C ABI in include/sb.h).

Argument marshalling only: every computation runs in the library's gfx950
kernels.  Device buffers and streams come from PyTorch (``torch.cuda`` is
HIP on ROCm).  Importing this module loads the library and fails loudly if
it has not been built; it never falls back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsb.so")

OK, E_INVAL, E_NOTPD, E_NOMEM, E_DEVICE, E_NOMODE, E_CAPACITY, E_UNSUPPORTED, E_NOCONV = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
FAMILY_GAUSS_MIX, FAMILY_STUDENT_T = 0, 1
NORM_PEAK_ZERO, NORM_DENSITY = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
DTYPE_F64, DTYPE_F32, DTYPE_BF16, DTYPE_F32_SPLIT, DTYPE_F32_H16 = 0, 1, 2, 3, 4
ST_CONVERGED, ST_STALLED, ST_MAXITER, ST_DEAD = 1, 2, 3, 4

# every extern "C" symbol declared in include/sb.h
EXPORTS = [
    "sb_evidence", "sb_evidence_batch", "sb_evidence_workspace_bytes", "sb_evidence_dev",
    "sb_exec_create", "sb_exec_destroy", "sb_exec_stats", "sb_evidence_exec_dev",
    "sb_evidence_chisao_workspace_bytes", "sb_evidence_chisao_dev",
    "sb_user_trajectories_workspace_bytes", "sb_user_trajectories_dev",
    "sb_user_mode_evidence_geo_workspace_bytes", "sb_user_mode_evidence_geo_dev",
    "sb_prep_workspace_bytes", "sb_prep_dev", "sb_logl_grad_workspace_bytes", "sb_logl_grad_dev",
    "sb_logl_grad_noalloc_dev",
    "sb_quadform_dev", "sb_quadform_pairs_dev", "sb_split_bf16_dev", "sb_hvp_workspace_bytes", "sb_hvp_dev", "sb_discover_workspace_bytes", "sb_discover_dev",
    "sb_lbfgs_direction_dev", "sb_lbfgs_workspace_bytes", "sb_lbfgs_dev",
    "sb_lbfgs_timed_dev", "sb_precheck_workspace_bytes", "sb_precheck_dev",
    "sb_eig_reduce_workspace_bytes", "sb_eig_reduce_dev", "sb_reduced_logl_workspace_bytes",
    "sb_reduced_logl_dev", "sb_reduced_bounds_dev", "sb_chisao_stick_dev",
    "sb_chisao_explore_workspace_bytes", "sb_chisao_explore_dev",
    "sb_chisao_reseed_workspace_bytes", "sb_chisao_reseed_dev", "sb_chisao_orthonormal_dev",
    "sb_user_compile", "sb_user_release",
    "sb_user_logl_dev", "sb_user_fd_workspace_bytes", "sb_user_fd_dev",
    "sb_user_mode_evidence_workspace_bytes", "sb_user_mode_evidence_dev",
    "sb_user_evidence_workspace_bytes", "sb_user_evidence_dev",
    "sb_dedup_workspace_bytes", "sb_dedup_dev", "sb_hessian_workspace_bytes", "sb_hessian_dev",
    "sb_cholesky_logdet_dev", "sb_cholesky_solve_dev", "sb_combine_dev", "sb_status_string",
    "sb_last_error", "sb_abi_version",
]


class sb_geometry_config(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("m", C.c_int32), ("grad_tol", C.c_double),
                ("eps_axis", C.c_double), ("eps_rot", C.c_double), ("rot_tol", C.c_double)]


class sb_chisao_config(C.Structure):
    _fields_ = [("n_osc", C.c_int32), ("n_conv", C.c_int32), ("stick_tol", C.c_double),
                ("n_reseed_pts", C.c_int32), ("n_cloud", C.c_int32), ("n_smooth", C.c_int32),
                ("sigma", C.c_double), ("alpha_cloud", C.c_double), ("n_anti", C.c_int32),
                ("alpha_anti", C.c_double), ("momentum", C.c_double), ("n_ref", C.c_int32),
                ("ref_delta", C.c_double)]


@dataclass
class ChiSaoConfig:
    """Parameters of the ChiSao cycle and the refinement pass (sb_chisao_config)."""
    n_osc: int = 3
    n_conv: int = 0
    stick_tol: float = 1e-6
    n_reseed_pts: int = 32
    n_cloud: int = 1
    n_smooth: int = 4
    sigma: float = 0.0
    alpha_cloud: float = 0.01
    n_anti: int = 8
    alpha_anti: float = 0.01
    momentum: float = 0.9
    n_ref: int = 0
    ref_delta: float = 10.0

    def c(self) -> sb_chisao_config:
        return sb_chisao_config(self.n_osc, self.n_conv, self.stick_tol, self.n_reseed_pts,
                                self.n_cloud, self.n_smooth, self.sigma, self.alpha_cloud,
                                self.n_anti, self.alpha_anti, self.momentum, self.n_ref,
                                self.ref_delta)


class SbError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({last_error()})")


class sb_loglik(C.Structure):
    _fields_ = [("family", C.c_int32), ("norm", C.c_int32), ("d", C.c_int32), ("K", C.c_int32),
                ("log_w", C.c_void_p), ("mu", C.c_void_p), ("prec", C.c_void_p),
                ("nu", C.c_double), ("logl_offset", C.c_double)]


class sb_box(C.Structure):
    _fields_ = [("lo", C.c_void_p), ("hi", C.c_void_p)]


class sb_config(C.Structure):
    _fields_ = [("n_rays", C.c_int32), ("n_points", C.c_int32), ("n_starts", C.c_int32),
                ("m", C.c_int32), ("max_iter", C.c_int32), ("max_modes", C.c_int32),
                ("precision", C.c_int32), ("grad_tol", C.c_double), ("dedup_tol", C.c_double),
                ("dedup_tol_pre", C.c_double), ("seed", C.c_uint64)]


class sb_result(C.Structure):
    _fields_ = [("log_z", C.c_double), ("n_modes", C.c_int32), ("modes", C.c_void_p),
                ("mode_log_z", C.c_void_p), ("mode_logl", C.c_void_p), ("log_det_h", C.c_void_p),
                ("n_logl_evals", C.c_int64), ("n_grad_evals", C.c_int64),
                ("n_hess_evals", C.c_int64), ("iterations", C.c_int32),
                ("n_rejected_nonpd", C.c_int32), ("n_dead_starts", C.c_int32),
                ("n_candidates", C.c_int32), ("n_reps_pre", C.c_int32),
                ("seconds", C.c_double * 8)]


class sb_model_dev(C.Structure):
    _fields_ = [("family", C.c_int32), ("norm", C.c_int32), ("d", C.c_int32), ("K", C.c_int32),
                ("log_w", C.c_void_p), ("mu", C.c_void_p), ("prec", C.c_void_p),
                ("nu", C.c_double), ("logl_offset", C.c_double), ("beta", C.c_void_p),
                ("prec_lp", C.c_void_p), ("mu_lp", C.c_void_p)]


_lib = None


def lib():
    """Load libsb.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        # torch first: libsb.so then binds to the HIP runtime torch has loaded (torch
        # carries its own copy; two runtimes in one process do not share devices)
        import torch  # noqa: F401

        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f64, u64, sz = (C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64,
                                      C.c_size_t)
        sig = {
            "sb_evidence": (i32, [vp, vp, vp, vp]),
            "sb_evidence_batch": (i32, [i32, vp, vp, vp, vp]),
            "sb_evidence_workspace_bytes": (sz, [vp, vp]),
            "sb_evidence_dev": (i32, [vp, vp, vp, vp, vp, sz, vp]),
            "sb_exec_create": (i32, [vp]),
            "sb_exec_destroy": (None, [vp]),
            "sb_exec_stats": (i32, [vp, vp]),
            "sb_evidence_exec_dev": (i32, [vp, vp, vp, vp, vp, vp, sz, vp]),
            "sb_evidence_chisao_workspace_bytes": (sz, [vp, vp, vp]),
            "sb_evidence_chisao_dev": (i32, [vp, vp, vp, vp, vp, vp, sz, vp]),
            "sb_user_trajectories_workspace_bytes": (sz, [i32, i32, i32]),
            "sb_user_trajectories_dev": (i32, [vp, i32, i32, vp, vp, vp, f64, i32, i32, f64, vp,
                                               vp, vp, vp, vp, sz, vp]),
            "sb_user_mode_evidence_geo_workspace_bytes": (sz, [i32, i32, vp]),
            "sb_user_mode_evidence_geo_dev": (i32, [vp, i32, i32, vp, vp, vp, vp, f64, f64, vp,
                                                    vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
            "sb_prep_workspace_bytes": (sz, [i32, i32]),
            "sb_prep_dev": (i32, [vp, vp, vp, vp, vp, vp, vp, sz, vp]),
            "sb_logl_grad_workspace_bytes": (sz, [i32, i32, i64, i32]),
            "sb_logl_grad_dev": (i32, [vp, i64, vp, vp, vp, i32, vp, sz, vp]),
            "sb_logl_grad_noalloc_dev": (i32, [vp, i64, vp, vp, vp, i32, vp]),
            "sb_quadform_dev": (i32, [vp, i64, vp, i32, vp, vp, vp, vp]),
            "sb_quadform_pairs_dev": (i32, [vp, i64, vp, vp, vp, i64, vp, vp, vp, vp]),
            "sb_split_bf16_dev": (i32, [i64, vp, vp, vp, vp]),
            "sb_hvp_workspace_bytes": (sz, [i32, i32, i64]),
            "sb_hvp_dev": (i32, [vp, i64, vp, vp, vp, vp, sz, vp]),
            "sb_discover_workspace_bytes": (sz, [i32, i32, i32, i32, i32]),
            "sb_discover_dev": (i32, [vp, vp, vp, i32, i32, i32, u64, i32, vp, vp, vp, vp, vp, vp,
                                      vp, sz, vp]),
            "sb_lbfgs_direction_dev": (i32, [i64, i32, i32, vp, vp, vp, vp, vp, i32, vp]),
            "sb_lbfgs_workspace_bytes": (sz, [i32, i32, i64, i32, i32]),
            "sb_lbfgs_dev": (i32, [vp, i64, vp, i32, i32, f64, i32, vp, vp, vp, vp, vp, vp, sz,
                                   vp]),
            "sb_lbfgs_timed_dev": (i32, [vp, i64, vp, i32, i32, f64, i32, vp, vp, vp, vp, vp,
                                         vp, sz, vp, i32, vp, vp, vp, vp, vp]),
            "sb_precheck_workspace_bytes": (sz, [i32, i32]),
            "sb_precheck_dev": (i32, [vp, vp, vp, f64, f64, vp, vp, vp, vp, vp, sz, vp]),
            "sb_eig_reduce_workspace_bytes": (sz, [i32, i32]),
            "sb_reduced_logl_workspace_bytes": (sz, [i32, i32, i64]),
            "sb_reduced_logl_dev": (i32, [vp, vp, vp, i32, i32, i64, vp, vp, vp, vp, sz, vp]),
            "sb_reduced_bounds_dev": (i32, [i32, vp, vp, i32, i32, vp, vp, vp, vp, vp]),
            "sb_eig_reduce_dev": (i32, [i32, i32, vp, vp, vp, f64, f64, vp, vp, vp, vp, vp, vp,
                                        vp, sz, vp]),
            "sb_chisao_stick_dev": (i32, [i64, i32, vp, vp, f64, vp, vp, sz, vp]),
            "sb_chisao_explore_workspace_bytes": (sz, [i32, i32, i64, i32]),
            "sb_chisao_explore_dev": (i32, [vp, vp, vp, i64, vp, vp, i32, i32, vp, f64, f64, i32,
                                            f64, f64, vp, sz, vp]),
            "sb_chisao_reseed_workspace_bytes": (sz, [i32, i32, i64, i32]),
            "sb_chisao_reseed_dev": (i32, [vp, vp, vp, i64, vp, vp, i32, vp, vp, sz, vp]),
            "sb_chisao_orthonormal_dev": (i32, [i32, i32, i32, vp, vp]),
            "sb_user_compile": (i32, [C.c_char_p, C.c_char_p, vp]),
            "sb_user_release": (None, [vp]),
            "sb_user_logl_dev": (i32, [vp, i64, i32, vp, vp, vp, vp]),
            "sb_user_fd_workspace_bytes": (sz, [i64, i32, i32]),
            "sb_user_fd_dev": (i32, [vp, i64, i32, vp, vp, f64, vp, vp, vp, vp, vp, vp, sz, vp]),
            "sb_user_mode_evidence_workspace_bytes": (sz, [i32, i32]),
            "sb_user_mode_evidence_dev": (i32, [vp, i32, i32, vp, vp, vp, vp, f64, f64, vp, vp,
                                                vp, vp, vp, vp, vp, sz, vp]),
            "sb_user_evidence_workspace_bytes": (sz, [i32, vp]),
            "sb_user_evidence_dev": (i32, [vp, i32, vp, vp, vp, vp, f64, f64, f64, vp, vp, sz,
                                           vp]),
            "sb_dedup_workspace_bytes": (sz, [i32]),
            "sb_dedup_dev": (i32, [i32, i32, vp, vp, vp, f64, i32, vp, vp, i32, vp, vp, sz, vp]),
            "sb_hessian_workspace_bytes": (sz, [i32, i32, i32]),
            "sb_hessian_dev": (i32, [vp, i32, vp, vp, vp, sz, vp]),
            "sb_cholesky_logdet_dev": (i32, [i32, i32, vp, vp, vp, vp, vp]),
            "sb_cholesky_solve_dev": (i32, [i32, i32, vp, vp, vp, vp]),
            "sb_combine_dev": (i32, [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
            "sb_status_string": (C.c_char_p, [i32]),
            "sb_last_error": (C.c_char_p, []),
            "sb_abi_version": (i32, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return lib().sb_status_string(st).decode()


def last_error() -> str:
    return lib().sb_last_error().decode()


def _check(st: int, where: str, ok=(OK,)):
    if st not in ok:
        raise SbError(st, where)
    return st


# ---------------------------------------------------------------- host path

def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class EvidenceResult:
    status: int
    log_z: float
    n_modes: int
    modes: np.ndarray
    mode_log_z: np.ndarray
    mode_logl: np.ndarray
    log_det_h: np.ndarray
    n_logl_evals: int
    n_grad_evals: int
    n_hess_evals: int
    iterations: int
    n_rejected_nonpd: int
    n_dead_starts: int
    n_candidates: int
    n_reps_pre: int
    seconds: list = field(default_factory=list)


def make_config(cfg) -> sb_config:
    return sb_config(cfg.n_rays, cfg.n_points, cfg.n_starts, cfg.m, cfg.max_iter, cfg.max_modes,
                     cfg.precision, cfg.grad_tol, cfg.dedup_tol,
                     getattr(cfg, "dedup_tol_pre", 0.0), cfg.seed)


class _HostProblem:
    def __init__(self, prob):
        self.log_w = _f64(prob.log_w)
        self.mu = _f64(prob.mu)
        self.prec = _f64(prob.prec)
        self.lo = _f64(prob.lo)
        self.hi = _f64(prob.hi)
        self.ll = sb_loglik(prob.family, prob.norm, prob.d, prob.K, self.log_w.ctypes.data,
                            self.mu.ctypes.data, self.prec.ctypes.data, float(prob.nu),
                            float(prob.logl_offset))
        self.box = sb_box(self.lo.ctypes.data, self.hi.ctypes.data)


def _result_arrays(cap: int, d: int):
    return (np.zeros((cap, d)), np.zeros(cap), np.zeros(cap), np.zeros(cap))


def _to_result(st, r, cap, arrs) -> EvidenceResult:
    modes, mlz, mll, ldh = arrs
    n = min(r.n_modes, cap) if st == OK else 0
    return EvidenceResult(st, r.log_z, r.n_modes, modes[:n].copy(), mlz[:n].copy(),
                          mll[:n].copy(), ldh[:n].copy(), r.n_logl_evals, r.n_grad_evals,
                          r.n_hess_evals, r.iterations, r.n_rejected_nonpd, r.n_dead_starts,
                          r.n_candidates, r.n_reps_pre, list(r.seconds))


def _new_result(cap, d):
    arrs = _result_arrays(cap, d)
    r = sb_result()
    r.modes, r.mode_log_z, r.mode_logl, r.log_det_h = (a.ctypes.data for a in arrs)
    return r, arrs


def sb_evidence(prob, cfg) -> EvidenceResult:
    """Evidence of one problem from host arrays (the library allocates device memory)."""
    hp = _HostProblem(prob)
    c = make_config(cfg)
    r, arrs = _new_result(cfg.max_modes, prob.d)
    st = lib().sb_evidence(C.byref(hp.ll), C.byref(hp.box), C.byref(c), C.byref(r))
    return _to_result(st, r, cfg.max_modes, arrs)


def sb_evidence_batch(probs: Sequence, cfgs: Sequence) -> list:
    """Evidence of independent problems in one batched run (host arrays).

    Returns one result per problem; a problem without modes has status
    E_NOMODE, one over its capacity E_CAPACITY (log Z NaN).  Errors that stop
    the whole batch (invalid input, device failure) raise SbError."""
    n = len(probs)
    if n != len(cfgs):
        raise ValueError("one config per problem")
    hps = [_HostProblem(p) for p in probs]
    LL = (sb_loglik * n)(*[h.ll for h in hps])
    BX = (sb_box * n)(*[h.box for h in hps])
    CF = (sb_config * n)(*[make_config(c) for c in cfgs])
    RS = (sb_result * n)()
    keep = []
    for j in range(n):
        r, arrs = _new_result(cfgs[j].max_modes, probs[j].d)
        RS[j] = r
        keep.append(arrs)
    st_all = lib().sb_evidence_batch(n, LL, BX, CF, RS)
    if st_all not in (OK, E_NOMODE, E_CAPACITY):
        raise SbError(st_all, "sb_evidence_batch")
    out = []
    for j in range(n):
        st = OK
        if RS[j].log_z == -math.inf:
            st = E_NOMODE
        elif math.isnan(RS[j].log_z):
            st = E_CAPACITY
        out.append(_to_result(st, RS[j], cfgs[j].max_modes, keep[j]))
    return out


# ---------------------------------------------------------------- device path

def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class DeviceModel:
    """Likelihood parameters resident on the GPU plus the prep outputs (beta, log det P)."""

    def __init__(self, prob, device="cuda", low_precision: bool = False):
        """low_precision also builds the FP32 / BF16 copies and the split
        [2][K][d][d] BF16 hi/lo copy (dtype F32_SPLIT) of the precisions."""
        import torch

        self.prob = prob
        dev = torch.device(device)
        self.d, self.K = prob.d, prob.K
        self.log_w = torch.as_tensor(_f64(prob.log_w), device=dev)
        self.mu = torch.as_tensor(_f64(prob.mu), device=dev)
        self.prec = torch.as_tensor(_f64(prob.prec), device=dev)
        self.lo = torch.as_tensor(_f64(prob.lo), device=dev)
        self.hi = torch.as_tensor(_f64(prob.hi), device=dev)
        self.beta = torch.zeros(self.K, dtype=torch.float64, device=dev)
        self.logdet_prec = torch.zeros(self.K, dtype=torch.float64, device=dev)
        self.prec_f32 = self.prec_bf16 = self.mu_f32 = self.prec_split = None
        if low_precision:
            self.prec_f32 = torch.empty(self.prec.shape, dtype=torch.float32, device=dev)
            self.prec_bf16 = torch.empty(self.prec.shape, dtype=torch.int16, device=dev)
            self.mu_f32 = torch.empty(self.mu.shape, dtype=torch.float32, device=dev)
            self.prec_split = torch.empty((2,) + tuple(self.prec.shape), dtype=torch.int16,
                                          device=dev)
        self.ll = sb_loglik(prob.family, prob.norm, prob.d, prob.K, self.log_w.data_ptr(),
                            self.mu.data_ptr(), self.prec.data_ptr(), float(prob.nu),
                            float(prob.logl_offset))
        ws = torch.empty(int(lib().sb_prep_workspace_bytes(self.d, self.K)), dtype=torch.uint8,
                         device=dev)
        st = lib().sb_prep_dev(C.byref(self.ll), self.beta.data_ptr(),
                               self.logdet_prec.data_ptr(), _ptr(self.prec_f32),
                               _ptr(self.prec_bf16), _ptr(self.mu_f32), ws.data_ptr(), ws.numel(),
                               _stream())
        _check(st, "sb_prep_dev")
        if low_precision:
            n = self.prec.numel()
            st = lib().sb_split_bf16_dev(n, self.prec.data_ptr(), self.prec_split[0].data_ptr(),
                                         self.prec_split[1].data_ptr(), _stream())
            _check(st, "sb_split_bf16_dev")

    def view(self, dtype: int = DTYPE_F64) -> sb_model_dev:
        lp = None
        if dtype in (DTYPE_F32, DTYPE_F32_H16):
            lp = _ptr(self.prec_f32)
        elif dtype == DTYPE_BF16:
            lp = _ptr(self.prec_bf16)
        elif dtype == DTYPE_F32_SPLIT:
            lp = _ptr(self.prec_split)
        return sb_model_dev(self.prob.family, self.prob.norm, self.d, self.K,
                            self.log_w.data_ptr(), self.mu.data_ptr(), self.prec.data_ptr(),
                            float(self.prob.nu), float(self.prob.logl_offset),
                            self.beta.data_ptr(), lp, _ptr(self.mu_f32))


def _ws(nbytes: int, device):
    import torch

    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def sb_logl_grad_dev(model: DeviceModel, X, grad: bool = True, dtype=None):
    """l (and grad l) at the rows of X (float64 -> FP64 path, float32 -> FP32 path, or
    DTYPE_F32_SPLIT for float32 data through the split BF16 contraction)."""
    import torch

    dt = dtype if dtype is not None else (DTYPE_F64 if X.dtype == torch.float64 else DTYPE_F32)
    X = X.contiguous()
    B = X.shape[0]
    l = torch.empty(B, dtype=X.dtype, device=X.device)
    g = torch.empty_like(X) if grad else None
    ws = _ws(lib().sb_logl_grad_workspace_bytes(model.d, model.K, B, dt), X.device)
    mv = model.view(dt)
    st = lib().sb_logl_grad_dev(C.byref(mv), B, X.data_ptr(), l.data_ptr(), _ptr(g), dt,
                                ws.data_ptr(), ws.numel(), _stream())
    _check(st, "sb_logl_grad_dev")
    return (l, g) if grad else l


def sb_logl_grad_noalloc_dev(model: DeviceModel, X, l, g=None, dtype=None, stream=None):
    """sb_logl_grad_dev into caller tensors l (and g) with the library's static scratch:
    nothing is allocated (the caller allocates l and g beforehand)."""
    import torch

    dt = dtype if dtype is not None else (DTYPE_F64 if X.dtype == torch.float64 else DTYPE_F32)
    mv = model.view(dt)
    st = lib().sb_logl_grad_noalloc_dev(C.byref(mv), X.shape[0], X.data_ptr(), l.data_ptr(),
                                        _ptr(g), dt, _stream(stream))
    _check(st, "sb_logl_grad_noalloc_dev")


class LoglGrad:
    """Repeated sb_logl_grad_dev calls on fixed buffers (outputs and workspace allocated once),
    so that a timing loop measures the launches, not the allocations."""

    def __init__(self, model: DeviceModel, X, dtype=None, grad: bool = True):
        import torch

        self.dt = dtype if dtype is not None else (
            DTYPE_F64 if X.dtype == torch.float64 else DTYPE_F32)
        self.X = X.contiguous()
        B = X.shape[0]
        self.l = torch.empty(B, dtype=X.dtype, device=X.device)
        self.g = torch.empty_like(self.X) if grad else None
        self.ws = _ws(lib().sb_logl_grad_workspace_bytes(model.d, model.K, B, self.dt), X.device)
        self.mv = model.view(self.dt)
        self.args = (C.byref(self.mv), B, self.X.data_ptr(), self.l.data_ptr(), _ptr(self.g),
                     self.dt, self.ws.data_ptr(), self.ws.numel())

    def __call__(self, stream=None):
        st = lib().sb_logl_grad_dev(*self.args, _stream(stream))
        _check(st, "sb_logl_grad_dev")


class QuadForm:
    """Repeated launches of the A3 contraction alone (sb_quadform_dev) on fixed buffers."""

    def __init__(self, model: DeviceModel, X, dtype=None):
        import torch

        self.model = model
        self.dt = dtype if dtype is not None else (
            DTYPE_F64 if X.dtype == torch.float64 else DTYPE_F32)
        self.X = X.contiguous()
        B = X.shape[0]
        self.Y = torch.empty((B, model.K * model.d), dtype=X.dtype, device=X.device)
        self.qpart = torch.empty((B, model.K, (model.d + 63) // 64), dtype=X.dtype,
                                 device=X.device)
        self.mv = model.view(self.dt)
        self.n_tiles = C.c_int32()

    def __call__(self, stream=None):
        st = lib().sb_quadform_dev(C.byref(self.mv), self.X.shape[0], self.X.data_ptr(), self.dt,
                                   self.Y.data_ptr(), self.qpart.data_ptr(),
                                   C.byref(self.n_tiles), _stream(stream))
        _check(st, "sb_quadform_dev")


def sb_hvp_dev(model: DeviceModel, X, V):
    import torch

    X = X.contiguous().to(torch.float64)
    V = V.contiguous().to(torch.float64)
    B = X.shape[0]
    HV = torch.empty_like(X)
    ws = _ws(lib().sb_hvp_workspace_bytes(model.d, model.K, B), X.device)
    mv = model.view(DTYPE_F64)
    st = lib().sb_hvp_dev(C.byref(mv), B, X.data_ptr(), V.data_ptr(), HV.data_ptr(),
                          ws.data_ptr(), ws.numel(), _stream())
    _check(st, "sb_hvp_dev")
    return HV


def sb_discover_dev(model: DeviceModel, R: int, n_pts: int, n_starts: int, seed: int,
                    dtype: int = DTYPE_F64):
    import torch

    dev = model.mu.device
    d = model.d
    P0 = torch.empty((R, d), dtype=torch.float64, device=dev)
    P1 = torch.empty((R, d), dtype=torch.float64, device=dev)
    bl = torch.empty(R, dtype=torch.float64, device=dev)
    bj = torch.empty(R, dtype=torch.int32, device=dev)
    sr = torch.empty(n_starts, dtype=torch.int32, device=dev)
    X0 = torch.empty((n_starts, d), dtype=torch.float64, device=dev)
    ws = _ws(lib().sb_discover_workspace_bytes(d, model.K, R, n_pts, dtype), dev)
    mv = model.view(dtype)
    st = lib().sb_discover_dev(C.byref(mv), model.lo.data_ptr(), model.hi.data_ptr(), R, n_pts,
                               n_starts, seed, dtype, P0.data_ptr(), P1.data_ptr(), bl.data_ptr(),
                               bj.data_ptr(), sr.data_ptr(), X0.data_ptr(), ws.data_ptr(),
                               ws.numel(), _stream())
    _check(st, "sb_discover_dev")
    return dict(P0=P0, P1=P1, ray_best_l=bl, ray_best_j=bj, start_ray=sr, X0=X0)


def sb_lbfgs_direction_dev(S, Y, G, cnt):
    import torch

    B, m, d = S.shape
    dt = DTYPE_F64 if S.dtype == torch.float64 else DTYPE_F32
    P = torch.empty_like(G)
    st = lib().sb_lbfgs_direction_dev(B, d, m, cnt.data_ptr(), S.contiguous().data_ptr(),
                                      Y.contiguous().data_ptr(), G.contiguous().data_ptr(),
                                      P.data_ptr(), dt, _stream())
    _check(st, "sb_lbfgs_direction_dev")
    return P


def sb_lbfgs_dev(model: DeviceModel, X0, m: int = 8, max_iter: int = 0, grad_tol: float = 0.0,
                 hist_bf16: bool = False):
    """Batched L-BFGS from X0 (float64: FP64; float32: FP32, with hist_bf16 the BF16 history
    ring of dtype F32_H16)."""
    import torch

    dt = DTYPE_F64 if X0.dtype == torch.float64 else (DTYPE_F32_H16 if hist_bf16 else DTYPE_F32)
    X = X0.clone().contiguous()
    B, d = X.shape
    l = torch.empty(B, dtype=X.dtype, device=X.device)
    g = torch.empty_like(X)
    status = torch.empty(B, dtype=torch.int32, device=X.device)
    iters = torch.empty(B, dtype=torch.int32, device=X.device)
    nev = C.c_int64()
    ws = _ws(lib().sb_lbfgs_workspace_bytes(d, model.K, B, m, dt), X.device)
    mv = model.view(dt)
    st = lib().sb_lbfgs_dev(C.byref(mv), B, X.data_ptr(), m, max_iter, grad_tol, dt, l.data_ptr(),
                            g.data_ptr(), status.data_ptr(), iters.data_ptr(), C.byref(nev),
                            ws.data_ptr(), ws.numel(), _stream())
    _check(st, "sb_lbfgs_dev")
    return dict(x=X, logl=l, grad=g, status=status, iters=iters, n_evals=nev.value)


def sb_lbfgs_timed_dev(model: DeviceModel, X0, m: int = 8, max_iter: int = 0,
                       grad_tol: float = 0.0, n_timed: int = 32, hist_bf16: bool = False):
    """sb_lbfgs_dev plus, for each of the first n_timed L-BFGS step launches, its duration
    (us), the number of starts active when it began, the number that accepted their trial and
    hold a full history ring after it, the number that halved their step in it, and its
    algorithmic bytes (-1 where some start reset or stopped in it, and for the first)."""
    import torch

    dt = DTYPE_F64 if X0.dtype == torch.float64 else (DTYPE_F32_H16 if hist_bf16 else DTYPE_F32)
    X = X0.clone().contiguous()
    B, d = X.shape
    l = torch.empty(B, dtype=X.dtype, device=X.device)
    g = torch.empty_like(X)
    status = torch.empty(B, dtype=torch.int32, device=X.device)
    iters = torch.empty(B, dtype=torch.int32, device=X.device)
    nev = C.c_int64()
    us = np.zeros(max(n_timed, 1), dtype=np.float32)
    rows = np.zeros(max(n_timed, 1), dtype=np.int32)
    full = np.zeros(max(n_timed, 1), dtype=np.int32)
    back = np.zeros(max(n_timed, 1), dtype=np.int32)
    nbytes = np.zeros(max(n_timed, 1), dtype=np.float64)
    ws = _ws(lib().sb_lbfgs_workspace_bytes(d, model.K, B, m, dt), X.device)
    mv = model.view(dt)
    st = lib().sb_lbfgs_timed_dev(C.byref(mv), B, X.data_ptr(), m, max_iter, grad_tol, dt,
                                  l.data_ptr(), g.data_ptr(), status.data_ptr(), iters.data_ptr(),
                                  C.byref(nev), ws.data_ptr(), ws.numel(), _stream(), n_timed,
                                  us.ctypes.data, rows.ctypes.data, full.ctypes.data,
                                  back.ctypes.data, nbytes.ctypes.data)
    _check(st, "sb_lbfgs_timed_dev")
    return dict(x=X, logl=l, grad=g, status=status, iters=iters, n_evals=nev.value,
                step_us=us[:n_timed], step_rows=rows[:n_timed], step_full=full[:n_timed],
                step_back=back[:n_timed], step_bytes=nbytes[:n_timed])


def sb_precheck_dev(model: DeviceModel, eps_flat: float = 0.0, eps_soft: float = 0.0,
                    lo=None, hi=None):
    """Preprocessing probe on the model's box (or lo/hi device tensors): sensitivities s,
    classes (0 active, 1 flat, 2 soft nuisance), marginal log-evidence of the flagged
    coordinates, and the flat and soft counts."""
    import torch

    dev = model.mu.device
    d = model.d
    lo = model.lo if lo is None else lo
    hi = model.hi if hi is None else hi
    s = torch.empty(d, dtype=torch.float64, device=dev)
    cls = torch.empty(d, dtype=torch.int32, device=dev)
    lz = torch.empty(1, dtype=torch.float64, device=dev)
    nfl = (C.c_int32 * 2)()
    ws = _ws(lib().sb_precheck_workspace_bytes(d, model.K), dev)
    mv = model.view(DTYPE_F64)
    st = lib().sb_precheck_dev(C.byref(mv), lo.data_ptr(), hi.data_ptr(), eps_flat, eps_soft,
                               s.data_ptr(), cls.data_ptr(), lz.data_ptr(), nfl, ws.data_ptr(),
                               ws.numel(), _stream())
    _check(st, "sb_precheck_dev")
    return dict(s=s, cls=cls, logz_marginal=lz, n_flat=nfl[0], n_soft=nfl[1])


def sb_reduced_logl_dev(model: DeviceModel, theta_star, V, r: int, phi, grad: bool = True):
    """The reduced likelihood l(theta* + V[:, :r] phi) (device FP64) and its gradient in phi."""
    import torch

    dev = model.mu.device
    th = theta_star.to(device=dev, dtype=torch.float64).contiguous()
    Vd = V.to(device=dev, dtype=torch.float64).contiguous()
    P = phi.to(device=dev, dtype=torch.float64).contiguous().reshape(-1, max(r, 1))[:, :r]
    P = P.contiguous()
    B, d = P.shape[0], model.d
    logl = torch.empty(B, dtype=torch.float64, device=dev)
    gp = torch.empty((B, r), dtype=torch.float64, device=dev) if grad else None
    ws = _ws(lib().sb_reduced_logl_workspace_bytes(d, model.K, B), dev)
    st = lib().sb_reduced_logl_dev(C.byref(model.view(DTYPE_F64)), th.data_ptr(), Vd.data_ptr(),
                                   Vd.shape[1], r, B, P.data_ptr(), logl.data_ptr(),
                                   gp.data_ptr() if grad else None, ws.data_ptr(), ws.numel(),
                                   _stream())
    _check(st, "sb_reduced_logl_dev")
    return (logl, gp) if grad else logl


def sb_reduced_bounds_dev(theta_star, V, r: int, lo, hi):
    """Per direction i < r the interval of t with theta* + t V[:, i] inside [lo, hi]."""
    import torch

    dev = theta_star.device
    Vd = V.to(dtype=torch.float64).contiguous()
    d = Vd.shape[0]
    plo = torch.empty(r, dtype=torch.float64, device=dev)
    phi = torch.empty(r, dtype=torch.float64, device=dev)
    st = lib().sb_reduced_bounds_dev(d, theta_star.contiguous().data_ptr(), Vd.data_ptr(),
                                     Vd.shape[1], r, lo.contiguous().data_ptr(),
                                     hi.contiguous().data_ptr(), plo.data_ptr(), phi.data_ptr(),
                                     _stream())
    _check(st, "sb_reduced_bounds_dev")
    return plo, phi


def sb_eig_reduce_dev(H, lo, hi, eps_inform: float, eps_nuisance: float):
    """Eigendecomposition of C symmetric matrices H [C][n][n] (device FP64), direction classes
    (0 informative, 1 nuisance, 2 degenerate), marginal log-evidence of the non-informative
    directions, d_eff and the Jacobi sweeps used."""
    import torch

    H = H.contiguous()
    Cn, n, _ = H.shape
    dev = H.device
    ev = torch.empty((Cn, n), dtype=torch.float64, device=dev)
    V = torch.empty((Cn, n, n), dtype=torch.float64, device=dev)
    cls = torch.empty((Cn, n), dtype=torch.int32, device=dev)
    lz = torch.empty(Cn, dtype=torch.float64, device=dev)
    deff = (C.c_int32 * Cn)()
    sweeps = C.c_int32(0)
    ws = _ws(lib().sb_eig_reduce_workspace_bytes(Cn, n), dev)
    st = lib().sb_eig_reduce_dev(Cn, n, H.data_ptr(), lo.data_ptr(), hi.data_ptr(), eps_inform,
                                 eps_nuisance, ev.data_ptr(), V.data_ptr(), cls.data_ptr(),
                                 lz.data_ptr(), deff, C.byref(sweeps), ws.data_ptr(), ws.numel(),
                                 _stream())
    _check(st, "sb_eig_reduce_dev")
    return dict(eigval=ev, V=V, cls=cls, logz_marginal=lz, d_eff=list(deff),
                sweeps=sweeps.value)


def sb_chisao_stick_dev(logl, grad, grad_tol: float):
    """ChiSao stick mask [B] (uint8, device) of samples with values logl [B] and gradients
    grad [B][d] (device FP64)."""
    import torch

    logl = logl.contiguous()
    grad = grad.contiguous()
    B, d = grad.shape
    dev = grad.device
    stuck = torch.empty(B, dtype=torch.uint8, device=dev)
    ws = _ws(256, dev)
    st = lib().sb_chisao_stick_dev(B, d, logl.data_ptr(), grad.data_ptr(), grad_tol,
                                   stuck.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    _check(st, "sb_chisao_stick_dev")
    return stuck


def sb_chisao_explore_dev(model: DeviceModel, X, stuck, Z, sigma: float, alpha_cloud: float,
                          n_anti: int, alpha: float, mu: float, lo=None, hi=None):
    """ChiSao moves of the free samples, in place on X [B][d] (device FP64): Z [n_cloud]
    [n_smooth][B][d] Hands Like Clouds draws, then n_anti anti-convergence steps.  Returns X."""
    import torch

    assert X.is_contiguous() and X.dtype == torch.float64
    B, d = X.shape
    dev = X.device
    lo = model.lo if lo is None else lo
    hi = model.hi if hi is None else hi
    stuck = stuck.to(torch.uint8).contiguous()
    n_cloud, n_smooth = (Z.shape[0], Z.shape[1]) if Z is not None else (0, 1)
    Zp = Z.contiguous().data_ptr() if Z is not None and Z.numel() else None
    if n_cloud == 0:
        Zp = None
    ws = _ws(lib().sb_chisao_explore_workspace_bytes(d, model.K, max(B, 1), n_smooth), dev)
    mv = model.view(DTYPE_F64)
    st = lib().sb_chisao_explore_dev(C.byref(mv), lo.data_ptr(), hi.data_ptr(), B, X.data_ptr(),
                                     stuck.data_ptr(), n_cloud, n_smooth, Zp, sigma, alpha_cloud,
                                     n_anti, alpha, mu, ws.data_ptr(), ws.numel(), _stream())
    _check(st, "sb_chisao_explore_dev")
    return X


def sb_chisao_reseed_dev(model: DeviceModel, X, U, n_pts: int, lo=None, hi=None):
    """ChiSao reseeding rays from the samples X [B][d] (device FP64, replaced in place by the
    best point of each ray) along directions U [B][d]; returns (X, best_l)."""
    import torch

    assert X.is_contiguous() and X.dtype == torch.float64
    U = U.contiguous()
    B, d = X.shape
    dev = X.device
    lo = model.lo if lo is None else lo
    hi = model.hi if hi is None else hi
    best = torch.empty(B, dtype=torch.float64, device=dev)
    ws = _ws(lib().sb_chisao_reseed_workspace_bytes(d, model.K, max(B, 1), max(n_pts, 1)), dev)
    mv = model.view(DTYPE_F64)
    st = lib().sb_chisao_reseed_dev(C.byref(mv), lo.data_ptr(), hi.data_ptr(), B, X.data_ptr(),
                                    U.data_ptr(), n_pts, best.data_ptr(), ws.data_ptr(),
                                    ws.numel(), _stream())
    _check(st, "sb_chisao_reseed_dev")
    return X, best


def sb_chisao_orthonormal_dev(G):
    """Golden Rooster directions: the rows of each G [C][n][d] (device FP64) made orthonormal
    in place (QR with a positive R diagonal).  Returns G."""
    assert G.is_contiguous() and G.dtype == __import__("torch").float64 and G.dim() == 3
    Cn, n, d = G.shape
    _check(lib().sb_chisao_orthonormal_dev(Cn, n, d, G.data_ptr(), _stream()),
           "sb_chisao_orthonormal_dev")
    return G


class UserLogL:
    """A generic log-likelihood given as HIP source defining
    ``__device__ double NAME(const double *x, int d, const double *params)``, compiled for the
    current device at construction."""

    def __init__(self, source: str, name: str):
        self.h = C.c_void_p()
        st = lib().sb_user_compile(source.encode(), name.encode(), C.byref(self.h))
        _check(st, "sb_user_compile")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sb_user_release(self.h)
            self.h = None

    def logl(self, X, params=None):
        import torch

        X = X.contiguous().to(torch.float64)
        B, d = X.shape
        l = torch.empty(B, dtype=torch.float64, device=X.device)
        st = lib().sb_user_logl_dev(self.h, B, d, X.data_ptr(), _ptr(params), l.data_ptr(),
                                    _stream())
        _check(st, "sb_user_logl_dev")
        return l

    def fd(self, X, eps: float, params=None, full: bool = False):
        """Central finite differences at the rows of X: l, grad, hdiag, probe_b and, with
        full, the Hessian H [B][d][d]."""
        import torch

        X = X.contiguous().to(torch.float64)
        B, d = X.shape
        f64 = dict(dtype=torch.float64, device=X.device)
        l = torch.empty(B, **f64)
        g = torch.empty((B, d), **f64)
        hd = torch.empty((B, d), **f64)
        pb = torch.empty(B, **f64)
        H = torch.empty((B, d, d), **f64) if full else None
        ws = _ws(lib().sb_user_fd_workspace_bytes(B, d, int(full)), X.device)
        st = lib().sb_user_fd_dev(self.h, B, d, X.data_ptr(), _ptr(params), eps, l.data_ptr(),
                                  g.data_ptr(), hd.data_ptr(), _ptr(H), pb.data_ptr(),
                                  ws.data_ptr(), ws.numel(), _stream())
        _check(st, "sb_user_fd_dev")
        return dict(l=l, grad=g, hdiag=hd, H=H, probe_b=pb)

    def mode_evidence(self, modes, lo, hi, eps: float, rot_tol: float, params=None):
        """Laplace evidence at the given modes with FD curvature: log Z, per-mode log Z
        (sorted), the sort order, l and log det per mode, and which modes took the full
        Hessian."""
        import torch

        modes = modes.contiguous().to(torch.float64)
        n, d = modes.shape
        f64 = dict(dtype=torch.float64, device=modes.device)
        l = torch.empty(n, **f64)
        ld = torch.empty(n, **f64)
        order = torch.empty(n, dtype=torch.int32, device=modes.device)
        mlz = torch.empty(n, **f64)
        lz = torch.empty(1, **f64)
        full = (C.c_int32 * n)()
        ws = _ws(lib().sb_user_mode_evidence_workspace_bytes(n, d), modes.device)
        st = lib().sb_user_mode_evidence_dev(self.h, n, d, modes.data_ptr(), _ptr(params),
                                             lo.data_ptr(), hi.data_ptr(), eps, rot_tol,
                                             l.data_ptr(), ld.data_ptr(), full, order.data_ptr(),
                                             mlz.data_ptr(), lz.data_ptr(), ws.data_ptr(),
                                             ws.numel(), _stream())
        _check(st, "sb_user_mode_evidence_dev")
        return dict(log_z=float(lz.cpu()[0]), mode_log_z=mlz, order=order, logl=l, logdet=ld,
                    full=list(full))

    def trajectories(self, modes, hdiag, eps: float, n_iter: int, m: int = 8,
                     grad_tol: float = 1e-6, params=None, bank: bool = False):
        """Step 1 of the geometry detection: the perpendicular step fraction per mode of the
        trajectories of GreenDragon's seeds (and, with bank, the recorded positions, gradients
        and lengths)."""
        import torch

        modes = modes.contiguous().to(torch.float64)
        n, d = modes.shape
        f64 = dict(dtype=torch.float64, device=modes.device)
        fp = torch.empty(n, **f64)
        Xb = Gb = bl = None
        if bank:
            Xb = torch.empty((n, 2 * d, n_iter + 1, d), **f64)
            Gb = torch.empty_like(Xb)
            bl = torch.zeros((n, 2 * d), dtype=torch.int32, device=modes.device)
        ws = _ws(lib().sb_user_trajectories_workspace_bytes(n, d, m), modes.device)
        st = lib().sb_user_trajectories_dev(self.h, n, d, modes.data_ptr(), _ptr(params),
                                            hdiag.contiguous().data_ptr(), eps, n_iter, m,
                                            grad_tol, fp.data_ptr(), _ptr(Xb), _ptr(Gb),
                                            _ptr(bl), ws.data_ptr(), ws.numel(), _stream())
        _check(st, "sb_user_trajectories_dev")
        return dict(fperp=fp, X=Xb, G=Gb, length=bl)

    def mode_evidence_geo(self, modes, lo, hi, eps_grad: float, eps_hess: float,
                          rot_tol: float, n_iter: int = 0, m: int = 0, grad_tol: float = 0.0,
                          eps_axis: float = 0.0, eps_rot: float = 0.0, params=None):
        """Laplace evidence at the given modes with both steps of the geometry detection."""
        import torch

        modes = modes.contiguous().to(torch.float64)
        n, d = modes.shape
        f64 = dict(dtype=torch.float64, device=modes.device)
        l = torch.empty(n, **f64)
        ld = torch.empty(n, **f64)
        fp = torch.empty(n, **f64)
        order = torch.empty(n, dtype=torch.int32, device=modes.device)
        mlz = torch.empty(n, **f64)
        lz = torch.empty(1, **f64)
        dec = (C.c_int32 * n)()
        gc = sb_geometry_config(n_iter, m, grad_tol, eps_axis, eps_rot, rot_tol)
        ws = _ws(lib().sb_user_mode_evidence_geo_workspace_bytes(n, d, C.byref(gc)),
                 modes.device)
        st = lib().sb_user_mode_evidence_geo_dev(self.h, n, d, modes.data_ptr(), _ptr(params),
                                                 lo.data_ptr(), hi.data_ptr(), eps_grad,
                                                 eps_hess, C.byref(gc), l.data_ptr(),
                                                 ld.data_ptr(), fp.data_ptr(), dec,
                                                 order.data_ptr(), mlz.data_ptr(),
                                                 lz.data_ptr(), ws.data_ptr(), ws.numel(),
                                                 _stream())
        _check(st, "sb_user_mode_evidence_geo_dev")
        return dict(log_z=float(lz.cpu()[0]), mode_log_z=mlz, order=order, logl=l, logdet=ld,
                    fperp=fp, decision=list(dec))

    def evidence(self, d: int, lo, hi, cfg, eps: float, eps_hess: float, rot_tol: float,
                 params=None):
        """The evidence path on this likelihood (discovery, FD L-BFGS, dedup, Laplace with FD
        curvature); lo, hi device tensors, cfg a RunConfig."""
        import torch

        c = make_config(cfg)
        cap = cfg.max_modes
        r, arrs = _new_result(cap, d)
        ws = _ws(lib().sb_user_evidence_workspace_bytes(d, C.byref(c)), lo.device)
        st = lib().sb_user_evidence_dev(self.h, d, _ptr(params), lo.data_ptr(), hi.data_ptr(),
                                        C.byref(c), eps, eps_hess, rot_tol, C.byref(r),
                                        ws.data_ptr(), ws.numel(), _stream())
        torch.cuda.synchronize()
        return _to_result(st, r, cap, arrs)


def sb_dedup_dev(X, l, tau: float, valid=None, max_reps: int = 1024):
    import torch

    Cn, d = X.shape
    dt = DTYPE_F64 if X.dtype == torch.float64 else DTYPE_F32
    rep_of = torch.empty(Cn, dtype=torch.int32, device=X.device)
    reps = torch.empty(max_reps, dtype=torch.int32, device=X.device)
    n = C.c_int32()
    ws = _ws(lib().sb_dedup_workspace_bytes(Cn), X.device)
    v = None if valid is None else valid.to(torch.uint8).contiguous()
    st = lib().sb_dedup_dev(Cn, d, X.contiguous().data_ptr(), l.contiguous().data_ptr(), _ptr(v),
                            tau, dt, rep_of.data_ptr(), reps.data_ptr(), max_reps, C.byref(n),
                            ws.data_ptr(), ws.numel(), _stream())
    _check(st, "sb_dedup_dev")
    return rep_of, reps[:n.value]


def sb_hessian_dev(model: DeviceModel, X):
    import torch

    X = X.contiguous().to(torch.float64)
    Cn = X.shape[0]
    H = torch.empty((Cn, model.d, model.d), dtype=torch.float64, device=X.device)
    ws = _ws(lib().sb_hessian_workspace_bytes(model.d, model.K, Cn), X.device)
    mv = model.view(DTYPE_F64)
    st = lib().sb_hessian_dev(C.byref(mv), Cn, X.data_ptr(), H.data_ptr(), ws.data_ptr(),
                              ws.numel(), _stream())
    _check(st, "sb_hessian_dev")
    return H


def sb_cholesky_logdet_dev(A):
    import torch

    A = A.contiguous().to(torch.float64)
    Cn, n, _ = A.shape
    L = torch.empty_like(A)
    ld = torch.empty(Cn, dtype=torch.float64, device=A.device)
    info = torch.empty(Cn, dtype=torch.int32, device=A.device)
    st = lib().sb_cholesky_logdet_dev(Cn, n, A.data_ptr(), L.data_ptr(), ld.data_ptr(),
                                      info.data_ptr(), _stream())
    _check(st, "sb_cholesky_logdet_dev")
    return L, ld, info


def sb_cholesky_solve_dev(L, b):
    import torch

    L = L.contiguous()
    b = b.contiguous().to(torch.float64)
    x = torch.empty_like(b)
    Cn, n, _ = L.shape
    st = lib().sb_cholesky_solve_dev(Cn, n, L.data_ptr(), b.data_ptr(), x.data_ptr(), _stream())
    _check(st, "sb_cholesky_solve_dev")
    return x


def sb_combine_dev(lo, hi, logl, logdet, modes):
    import torch

    n, d = modes.shape
    order = torch.empty(n, dtype=torch.int32, device=modes.device)
    mlz = torch.empty(n, dtype=torch.float64, device=modes.device)
    lz = torch.empty(1, dtype=torch.float64, device=modes.device)
    st = lib().sb_combine_dev(n, d, lo.data_ptr(), hi.data_ptr(), logl.contiguous().data_ptr(),
                              logdet.contiguous().data_ptr(), modes.contiguous().data_ptr(),
                              order.data_ptr(), mlz.data_ptr(), lz.data_ptr(), _stream())
    _check(st, "sb_combine_dev")
    return order, mlz, lz


class ExecContext:
    """sb_exec: pinned readback word, timing events and instantiated block graphs kept
    across whole-path calls on one device (created on the current device)."""

    def __init__(self):
        h = C.c_void_p()
        _check(lib().sb_exec_create(C.byref(h)), "sb_exec_create")
        self.handle = h

    def stats(self) -> dict:
        c = (C.c_int32 * 4)()
        _check(lib().sb_exec_stats(self.handle, c), "sb_exec_stats")
        return {"captured": c[0], "instantiated": c[1], "updated": c[2], "launched": c[3]}

    def close(self):
        if self.handle:
            lib().sb_exec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EvidenceRunner:
    """Device-resident evidence: inputs in HBM, workspace allocated once.  Without an
    execution context run() calls sb_evidence_dev (allocation-free, blocks launched
    directly); with one (exec=True: a context of its own, or an ExecContext) it calls
    sb_evidence_exec_dev (iteration blocks as the context's HIP graphs)."""

    def __init__(self, prob, cfg, device="cuda", exec=None, chisao: "ChiSaoConfig" = None):
        import torch

        self.prob, self.cfg = prob, cfg
        self.chisao = chisao.c() if chisao is not None else None
        dev = torch.device(device)
        if exec is True:
            with torch.cuda.device(dev):
                exec = ExecContext()
        self.exec = exec or None
        self.log_w = torch.as_tensor(_f64(prob.log_w), device=dev)
        self.mu = torch.as_tensor(_f64(prob.mu), device=dev)
        self.prec = torch.as_tensor(_f64(prob.prec), device=dev)
        self.lo = torch.as_tensor(_f64(prob.lo), device=dev)
        self.hi = torch.as_tensor(_f64(prob.hi), device=dev)
        self.ll = sb_loglik(prob.family, prob.norm, prob.d, prob.K, self.log_w.data_ptr(),
                            self.mu.data_ptr(), self.prec.data_ptr(), float(prob.nu),
                            float(prob.logl_offset))
        self.box = sb_box(self.lo.data_ptr(), self.hi.data_ptr())
        self.c = make_config(cfg)
        if self.chisao is not None:
            nb = lib().sb_evidence_chisao_workspace_bytes(C.byref(self.ll), C.byref(self.c),
                                                          C.byref(self.chisao))
        else:
            nb = lib().sb_evidence_workspace_bytes(C.byref(self.ll), C.byref(self.c))
        if nb == 0:
            raise SbError(E_INVAL, "sb_evidence_workspace_bytes")
        self.ws = torch.empty(int(nb), dtype=torch.uint8, device=dev)

    def run(self, stream=None) -> EvidenceResult:
        r, arrs = _new_result(self.cfg.max_modes, self.prob.d)
        if self.chisao is not None:
            st = lib().sb_evidence_chisao_dev(C.byref(self.ll), C.byref(self.box),
                                              C.byref(self.c), C.byref(self.chisao), C.byref(r),
                                              self.ws.data_ptr(), self.ws.numel(),
                                              _stream(stream))
        elif self.exec is not None:
            st = lib().sb_evidence_exec_dev(self.exec.handle, C.byref(self.ll),
                                            C.byref(self.box), C.byref(self.c), C.byref(r),
                                            self.ws.data_ptr(), self.ws.numel(),
                                            _stream(stream))
        else:
            st = lib().sb_evidence_dev(C.byref(self.ll), C.byref(self.box), C.byref(self.c),
                                       C.byref(r), self.ws.data_ptr(), self.ws.numel(),
                                       _stream(stream))
        return _to_result(st, r, self.cfg.max_modes, arrs)
