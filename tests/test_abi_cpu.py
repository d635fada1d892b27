"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/sb.h declares, and rejects invalid arguments before touching a device."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2601_19957_amd import _lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sb.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(sb_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_and_exports_agree():
    decl = declared_functions()
    assert len(decl) >= 20
    assert sorted(_lib.EXPORTS) == decl
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sb_[a-z0-9_]+)\b", out))
    assert set(decl) <= exported


def test_library_loads_and_reports():
    L = _lib.lib()
    assert L.sb_abi_version() == 1
    for st in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert _lib.status_string(st) and "unknown" not in _lib.status_string(st)
    assert "unknown" in _lib.status_string(17)


def _status(mod=None, cfg_mod=None, name="c0"):
    prob, cfg = synth.make_workload(name)
    if mod:
        mod(prob)
    if cfg_mod:
        cfg_mod(cfg)
    return _lib.sb_evidence(prob, cfg)


def test_validation_before_device():
    # each invalid input is rejected on the host, before any device call
    cases = [
        (lambda p: setattr(p, "d", 0), None, _lib.E_INVAL),
        (lambda p: setattr(p, "K", 0), None, _lib.E_INVAL),
        (lambda p: setattr(p, "family", 7), None, _lib.E_INVAL),
        (lambda p: p.lo.__setitem__(0, 11.0), None, _lib.E_INVAL),
        (lambda p: p.hi.__setitem__(2, np.nan), None, _lib.E_INVAL),
        (lambda p: p.mu.__setitem__((0, 1), np.inf), None, _lib.E_INVAL),
        (lambda p: p.prec.__setitem__((0, 1, 1), np.nan), None, _lib.E_INVAL),
        (None, lambda c: setattr(c, "m", 0), _lib.E_INVAL),
        (None, lambda c: setattr(c, "m", 33), _lib.E_INVAL),
        (None, lambda c: setattr(c, "max_modes", 0), _lib.E_INVAL),
        (None, lambda c: setattr(c, "n_starts", 10 ** 6), _lib.E_INVAL),
        (None, lambda c: setattr(c, "n_points", 0), _lib.E_INVAL),
        (None, lambda c: setattr(c, "precision", 5), _lib.E_INVAL),
    ]
    for mod, cmod, expect in cases:
        r = _status(mod, cmod)
        assert r.status == expect, (mod, cmod, r.status, _lib.last_error())
        assert math.isnan(r.log_z)


def test_student_t_validation():
    rng = np.random.Generator(np.random.PCG64(1))
    t = synth.student_t(rng, 4, 0.0, -1, 1, 0.5, 1.0, 10.0)
    cfg = synth.RunConfig(n_rays=8, n_points=4, n_starts=4)
    assert _lib.sb_evidence(t, cfg).status == _lib.E_INVAL
    t.nu = 5.0
    t.K = 2
    t.mu = np.concatenate([t.mu, t.mu])
    t.prec = np.concatenate([t.prec, t.prec])
    t.log_w = np.zeros(2)
    assert _lib.sb_evidence(t, cfg).status == _lib.E_UNSUPPORTED


def test_null_arguments():
    L = _lib.lib()
    assert L.sb_evidence(None, None, None, None) == _lib.E_INVAL
    assert L.sb_exec_create(None) == _lib.E_INVAL
    assert L.sb_exec_stats(None, None) == _lib.E_INVAL
    L.sb_exec_destroy(None)
    prob, cfg = synth.make_workload("c0")
    hp = _lib._HostProblem(prob)
    r = _lib.sb_result()
    assert L.sb_evidence_exec_dev(None, C.byref(hp.ll), C.byref(hp.box),
                                  C.byref(_lib.make_config(cfg)), C.byref(r), None, 0,
                                  None) == _lib.E_INVAL
    assert math.isnan(r.log_z)
    assert L.sb_evidence_workspace_bytes(None, None) == 0
    assert L.sb_lbfgs_direction_dev(1, 4, 8, None, None, None, None, None, 0, None) == _lib.E_INVAL
    assert L.sb_cholesky_logdet_dev(1, 0, None, None, None, None, None) == _lib.E_INVAL
    assert L.sb_precheck_dev(None, None, None, 0.0, 0.0, None, None, None, None, None, 0,
                             None) == _lib.E_INVAL
    assert L.sb_precheck_workspace_bytes(0, 1) == 0
    assert L.sb_eig_reduce_dev(0, 4, None, None, None, 1.0, 0.1, None, None, None, None, None,
                               None, None, 0, None) == _lib.E_INVAL
    assert L.sb_eig_reduce_workspace_bytes(1, 0) == 0
    h = C.c_void_p()
    assert L.sb_user_compile(None, b"f", C.byref(h)) == _lib.E_INVAL
    assert L.sb_user_compile(b"__device__ double f(const double *x, int d, const double *p)"
                             b" { return 0.0; }", b"1f", C.byref(h)) == _lib.E_INVAL
    assert L.sb_user_fd_workspace_bytes(0, 3, 0) == 0
    assert L.sb_user_mode_evidence_dev(None, 1, 2, None, None, None, None, 1e-3, 1e-3, None, None,
                                       None, None, None, None, None, 0, None) == _lib.E_INVAL
    assert L.sb_user_mode_evidence_workspace_bytes(0, 2) == 0
    assert L.sb_user_evidence_workspace_bytes(3, None) == 0
    assert L.sb_user_evidence_dev(None, 3, None, None, None, None, 1e-5, 1e-3, 1e-3, None, None,
                                  0, None) == _lib.E_INVAL


def test_user_likelihood_compiles_on_the_host():
    """The run-time compilation of a user likelihood needs no GPU: a syntax error is reported
    with the compiler's message; a valid source compiles and then needs a device to load."""
    L = _lib.lib()
    h = C.c_void_p()
    bad = b"__device__ double f(const double *x, int d, const double *p) { return x[0] + ; }"
    assert L.sb_user_compile(bad, b"f", C.byref(h)) == _lib.E_INVAL
    assert "error" in _lib.last_error()
    good = b"__device__ double f(const double *x, int d, const double *p) { return -x[0]; }"
    st = L.sb_user_compile(good, b"f", C.byref(h))
    assert st in (_lib.OK, _lib.E_DEVICE)
    if st == _lib.OK:
        L.sb_user_release(h)
    for n_timed in (-1, 4):  # negative count, or timing arrays missing
        assert L.sb_lbfgs_timed_dev(None, 1, None, 8, 0, 0.0, 1, None, None, None, None, None,
                                    None, 0, None, n_timed, None, None, None,
                                    None, None) == _lib.E_INVAL
    assert L.sb_dedup_dev(4, 2, None, None, None, 0.1, 0, None, None, 4, None, None, 0,
                          None) == _lib.E_INVAL
    assert L.sb_combine_dev(1, 0, None, None, None, None, None, None, None, None,
                            None) == _lib.E_INVAL


def test_workspace_sizes_scale():
    prob, cfg = synth.make_workload("c1")
    ll = _lib._HostProblem(prob).ll
    small = _lib.lib().sb_evidence_workspace_bytes(C.byref(ll), C.byref(_lib.make_config(cfg)))
    cfg.n_starts = cfg.n_rays = 8192
    big = _lib.lib().sb_evidence_workspace_bytes(C.byref(ll), C.byref(_lib.make_config(cfg)))
    assert 0 < small < big
    assert _lib.lib().sb_logl_grad_workspace_bytes(64, 4, 1000, 0) > 8 * 1000 * 256


def test_batch_validation_before_device():
    """Mismatched precisions in one batch are rejected before any device work."""
    import numpy as np
    from paper_2601_19957_amd import _lib, synth

    p = synth.make_problem("c0")
    c0 = synth.make_run_config("c0", precision=0)
    c1 = synth.make_run_config("c0", precision=1)
    try:
        _lib.sb_evidence_batch([p, p], [c0, c1])
    except _lib.SbError as e:
        assert e.status == _lib.E_INVAL and "problem 1" in str(e)
    else:
        raise AssertionError("expected SbError")
    assert np.isfinite(p.lo).all()
