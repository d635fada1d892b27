"""CPU oracle of the Laplace-evidence hot path -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes) to the plain FP64 C oracle in ``oracle.c``.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg use this package;
the product library and its binding never import it.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

ST_ACTIVE, ST_CONVERGED, ST_STALLED, ST_MAXITER, ST_DEAD = 0, 1, 2, 3, 4
OK, E_INVAL, E_NOTPD, E_NOMEM, E_NOMODE, E_CAPACITY, E_UNSUPPORTED = 0, -1, -2, -3, -5, -6, -7


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, OpenMP across starts)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Problem(C.Structure):
    _fields_ = [("family", C.c_int32), ("norm", C.c_int32), ("d", C.c_int32), ("K", C.c_int32),
                ("log_w", C.c_void_p), ("mu", C.c_void_p), ("prec", C.c_void_p),
                ("nu", C.c_double), ("logl_offset", C.c_double)]


class _Config(C.Structure):
    _fields_ = [("n_rays", C.c_int32), ("n_points", C.c_int32), ("n_starts", C.c_int32),
                ("m", C.c_int32), ("max_iter", C.c_int32), ("max_modes", C.c_int32),
                ("grad_tol", C.c_double), ("dedup_tol", C.c_double),
                ("dedup_tol_pre", C.c_double), ("seed", C.c_uint64), ("n_threads", C.c_int32),
                ("problem", C.c_uint32)]


class _Result(C.Structure):
    _fields_ = [("log_z", C.c_double), ("n_modes", C.c_int32), ("modes", C.c_void_p),
                ("mode_log_z", C.c_void_p), ("mode_logl", C.c_void_p), ("log_det_h", C.c_void_p),
                ("n_logl_evals", C.c_int64), ("n_grad_evals", C.c_int64),
                ("n_hess_evals", C.c_int64), ("iterations", C.c_int32),
                ("n_rejected_nonpd", C.c_int32), ("n_dead_starts", C.c_int32),
                ("n_candidates", C.c_int32), ("n_reps_pre", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f64, u64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64, C.c_uint32
        L.or_pairwise_sum.restype = f64
        L.or_pairwise_sum.argtypes = [vp, i64]
        L.or_logsumexp.restype = f64
        L.or_logsumexp.argtypes = [vp, i32]
        L.or_cholesky.restype = i32
        L.or_cholesky.argtypes = [i32, vp, vp]
        L.or_logdet_from_chol.restype = f64
        L.or_logdet_from_chol.argtypes = [i32, vp]
        L.or_chol_solve.argtypes = [i32, vp, vp, vp]
        L.or_validate_problem.restype = i32
        L.or_validate_problem.argtypes = [vp]
        L.or_prep.restype = i32
        L.or_prep.argtypes = [vp, vp, vp]
        L.or_logl.argtypes = [vp, vp, i64, vp, vp, vp]
        L.or_hvp.argtypes = [vp, vp, i64, vp, vp, vp]
        L.or_neg_hessian.argtypes = [vp, vp, vp, vp]
        L.or_philox4x32_10.argtypes = [vp, vp, vp]
        L.or_rng_word.restype = u32
        L.or_rng_word.argtypes = [u64, u32, u32, u32, u32]
        L.or_rng_uniform.restype = f64
        L.or_rng_uniform.argtypes = [u64, u32, u32, u32, u32]
        L.or_rays.argtypes = [i32, vp, vp, i32, u64, u32, vp, vp]
        L.or_discover.restype = i32
        L.or_discover.argtypes = [vp, vp, vp, vp, i32, i32, i32, u64, u32, vp, vp, vp, vp]
        L.or_two_loop.argtypes = [i32, i32, vp, vp, vp, vp]
        L.or_lbfgs.restype = i32
        L.or_lbfgs.argtypes = [vp, vp, vp, i32, i32, f64, vp, vp, vp, vp]
        L.or_newton.restype = i32
        L.or_newton.argtypes = [vp, vp, vp, i32, vp]
        L.or_dedup.restype = i32
        L.or_dedup.argtypes = [i32, i32, vp, vp, vp, f64, vp, vp]
        L.or_log_volume.restype = f64
        L.or_log_volume.argtypes = [i32, vp, vp]
        L.or_precheck.restype = i32
        L.or_precheck.argtypes = [vp, vp, vp, vp, f64, f64, vp, vp, vp]
        L.or_mode_log_z.restype = f64
        L.or_mode_log_z.argtypes = [i32, f64, f64, f64]
        L.or_evidence.restype = i32
        L.or_evidence.argtypes = [vp, vp, vp, vp, vp]
        L.or_reference_modes.restype = i32
        L.or_reference_modes.argtypes = [vp, vp, vp, f64, i32, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleProblem:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, prob):
        self.prob = prob
        self.log_w = _f64(prob.log_w)
        self.mu = _f64(prob.mu)
        self.prec = _f64(prob.prec)
        self.lo = _f64(prob.lo)
        self.hi = _f64(prob.hi)
        self.s = _Problem(prob.family, prob.norm, prob.d, prob.K, _p(self.log_w).value,
                          _p(self.mu).value, _p(self.prec).value, float(prob.nu),
                          float(prob.logl_offset))
        self._beta = None

    @property
    def ptr(self):
        return C.byref(self.s)

    def beta(self) -> np.ndarray:
        if self._beta is None:
            b = np.zeros(self.prob.K)
            st = lib().or_prep(self.ptr, _p(b), None)
            if st != OK:
                raise ValueError(f"oracle prep failed: {st}")
            self._beta = b
        return self._beta


def pairwise_sum(x) -> float:
    x = _f64(x)
    return lib().or_pairwise_sum(_p(x), x.size)


def logsumexp(x) -> float:
    x = _f64(x)
    return lib().or_logsumexp(_p(x), x.size)


def cholesky(A):
    A = _f64(A)
    n = A.shape[0]
    L = np.zeros_like(A)
    st = lib().or_cholesky(n, _p(A), _p(L))
    return st, L


def logdet_spd(A) -> float:
    st, L = cholesky(A)
    if st:
        raise ValueError("not positive definite")
    return lib().or_logdet_from_chol(A.shape[0], _p(L))


def chol_solve(L, b):
    L = _f64(L)
    b = _f64(b)
    x = np.zeros_like(b)
    lib().or_chol_solve(L.shape[0], _p(L), _p(b), _p(x))
    return x


def validate_problem(prob) -> int:
    op = OracleProblem(prob)
    return lib().or_validate_problem(op.ptr)


def prep(prob):
    op = OracleProblem(prob)
    beta = np.zeros(prob.K)
    ld = np.zeros(prob.K)
    st = lib().or_prep(op.ptr, _p(beta), _p(ld))
    return st, beta, ld


def logl(prob, X, grad: bool = True, op: Optional[OracleProblem] = None):
    op = op or OracleProblem(prob)
    X = _f64(np.atleast_2d(X))
    B = X.shape[0]
    l = np.zeros(B)
    g = np.zeros_like(X) if grad else None
    lib().or_logl(op.ptr, _p(op.beta()), B, _p(X), _p(l), _p(g) if grad else None)
    return (l, g) if grad else l


def hvp(prob, X, V, op: Optional[OracleProblem] = None):
    op = op or OracleProblem(prob)
    X = _f64(np.atleast_2d(X))
    V = _f64(np.atleast_2d(V))
    HV = np.zeros_like(X)
    lib().or_hvp(op.ptr, _p(op.beta()), X.shape[0], _p(X), _p(V), _p(HV))
    return HV


def neg_hessian(prob, x, op: Optional[OracleProblem] = None):
    op = op or OracleProblem(prob)
    x = _f64(x)
    H = np.zeros((prob.d, prob.d))
    lib().or_neg_hessian(op.ptr, _p(op.beta()), _p(x), _p(H))
    return H


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def rng_word(seed, problem, ray, stream, i) -> int:
    return lib().or_rng_word(seed, problem, ray, stream, i)


def rng_uniform(seed, problem, ray, stream, i) -> float:
    return lib().or_rng_uniform(seed, problem, ray, stream, i)


def rays(d, lo, hi, R, seed, problem=0):
    lo = _f64(lo)
    hi = _f64(hi)
    P0 = np.zeros((R, d))
    P1 = np.zeros((R, d))
    lib().or_rays(d, _p(lo), _p(hi), R, seed, problem, _p(P0), _p(P1))
    return P0, P1


def discover(prob, R, n_pts, n_starts, seed, problem=0):
    op = OracleProblem(prob)
    bl = np.zeros(R)
    bj = np.zeros(R, dtype=np.int32)
    sr = np.zeros(n_starts, dtype=np.int32)
    X0 = np.zeros((n_starts, prob.d))
    st = lib().or_discover(op.ptr, _p(op.beta()), _p(op.lo), _p(op.hi), R, n_pts, n_starts, seed,
                           problem, _p(bl), _p(bj), _p(sr), _p(X0))
    if st != OK:
        raise ValueError(f"discover failed {st}")
    return dict(ray_best_l=bl, ray_best_j=bj, start_ray=sr, X0=X0)


def two_loop(S, Y, g):
    S = _f64(S)
    Y = _f64(Y)
    g = _f64(g)
    cnt, d = S.shape
    p = np.zeros(d)
    lib().or_two_loop(d, cnt, _p(S), _p(Y), _p(g), _p(p))
    return p


def lbfgs(prob, x0, m=8, max_iter=None, grad_tol=1e-10, op=None):
    op = op or OracleProblem(prob)
    x = _f64(x0).copy()
    l = C.c_double()
    g = np.zeros(prob.d)
    it = C.c_int32()
    ev = C.c_int64()
    mi = max_iter if max_iter is not None else 10 * prob.d + 200
    st = lib().or_lbfgs(op.ptr, _p(op.beta()), _p(x), m, mi, grad_tol, C.byref(l), _p(g),
                        C.byref(it), C.byref(ev))
    return dict(status=st, x=x, logl=l.value, grad=g, iters=it.value, evals=ev.value)


def newton(prob, x0, max_steps=20, op=None):
    op = op or OracleProblem(prob)
    x = _f64(x0).copy()
    steps = C.c_int32()
    st = lib().or_newton(op.ptr, _p(op.beta()), _p(x), max_steps, C.byref(steps))
    return st, x, steps.value


def dedup(X, l, tau, valid=None):
    X = _f64(X)
    l = _f64(l)
    Cn, d = X.shape
    rep_of = np.zeros(Cn, dtype=np.int32)
    reps = np.zeros(max(Cn, 1), dtype=np.int32)
    v = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    n = lib().or_dedup(Cn, d, _p(X), _p(l), _p(v) if v is not None else None, tau, _p(rep_of),
                       _p(reps))
    return rep_of, reps[:n].copy()


def chisao_stick(l, G, grad_tol):
    """Stick detection of the ChiSao cycle (section "ChiSao Exploration", the oscillation
    cycle's second step and the algorithm summary of CarryTiger): a sample sticks when its
    gradient's L-infinity norm is below grad_tol and its l is at least l_max + log 0.1, with
    l_max the largest finite l of the batch.  Readings: log 0.1 is -ln 10 (a tenth of the
    maximum likelihood, exactly), in FP64 the correctly rounded -ln 10, not the logarithm of the
    double nearest 0.1 (one unit in the last place apart); a sample with a non-finite l or
    gradient entry never sticks."""
    l = _f64(l)
    G = _f64(np.atleast_2d(G))
    stuck = np.zeros(l.size, dtype=np.uint8)
    fin = [i for i in range(l.size) if math.isfinite(l[i])]
    if not fin:
        return stuck
    lmax = max(l[i] for i in fin)
    thr = lmax - math.log(10.0)
    for i in fin:
        g = G[i]
        if not np.all(np.isfinite(g)):
            continue
        if float(np.max(np.abs(g))) < grad_tol and l[i] >= thr:
            stuck[i] = 1
    return stuck


def chisao_explore(prob, X, stuck, Z, sigma, alpha_cloud, n_anti, alpha, mu,
                   op: Optional[OracleProblem] = None):
    """The ChiSao cycle's moves of the samples that are not stuck (section "ChiSao
    Exploration"): Hands Like Clouds, then the anti-convergence phase.

    Hands Like Clouds: for each of Z's n_cloud steps, the smoothed gradient is the mean over
    its K perturbations of grad l(x + sigma z_k) (the equation of that step; Z [n_cloud][K]
    [B][d] holds the standard normal draws), and the sample moves x <- x + alpha_cloud times
    it.  Anti-convergence: n_anti momentum descent steps v <- mu v - alpha grad l(x),
    x <- x + v (the momentum equation of that phase), from v = 0.  Readings: the step sizes
    are parameters; every move is clipped to the prior box; stuck samples do not move."""
    op = op or OracleProblem(prob)
    X = _f64(np.atleast_2d(X)).copy()
    free = np.asarray(stuck).reshape(-1) == 0
    lo, hi = op.lo, op.hi
    Z = _f64(Z)
    n_cloud, K = Z.shape[0], Z.shape[1]
    for s in range(n_cloud):
        acc = np.zeros_like(X)
        for k in range(K):
            _, g = logl(prob, X + sigma * Z[s, k], op=op)
            acc = acc + g
        step = alpha_cloud * (acc / K)
        X[free] = np.minimum(np.maximum(X[free] + step[free], lo), hi)
    V = np.zeros_like(X)
    for _ in range(n_anti):
        _, g = logl(prob, X, op=op)
        V = mu * V - alpha * g
        X[free] = np.minimum(np.maximum(X[free] + V[free], lo), hi)
    return X


def chisao_reseed(prob, X, U, n_pts, op: Optional[OracleProblem] = None):
    """The reseeding ray of the ChiSao cycle (section "ChiSao Exploration", the Repulse Monkey /
    Golden Rooster step: rays shot from existing samples in given directions), sampled as the
    coarse pass samples a ray (section "Ray Generation": uniform points along r(t), keep the
    best).  From origin x along direction u the ray ends where it leaves the box, at
    t_exit = min over u_i != 0 of (hi_i - x_i)/u_i (u_i > 0) or (lo_i - x_i)/u_i (u_i < 0),
    at least 0 (0 when u = 0); its points are x + (t_j t_exit) u with t_j = (j + 1/2)/n_pts; the
    new sample is the point of highest l (ties: lowest j; non-finite l never chosen; none
    finite: x stays).  Returns the new samples and their l (NaN where x stayed)."""
    op = op or OracleProblem(prob)
    X = _f64(np.atleast_2d(X))
    U = _f64(np.atleast_2d(U))
    lo, hi = op.lo, op.hi
    out = X.copy()
    best = np.full(X.shape[0], np.nan)
    for b in range(X.shape[0]):
        x, u = X[b], U[b]
        te = math.inf
        for i in range(x.size):
            if u[i] > 0:
                te = min(te, (hi[i] - x[i]) / u[i])
            elif u[i] < 0:
                te = min(te, (lo[i] - x[i]) / u[i])
        te = 0.0 if te == math.inf else max(te, 0.0)
        P = np.empty((n_pts, x.size))
        for j in range(n_pts):
            s = ((j + 0.5) / n_pts) * te
            P[j] = x + s * u
        l = logl(prob, P, grad=False, op=op)
        jb = -1
        for j in range(n_pts):
            if math.isfinite(l[j]) and (jb < 0 or l[j] > l[jb]):
                jb = j
        if jb >= 0:
            out[b] = P[jb]
            best[b] = l[jb]
    return out, best


def chisao_orthonormal(G):
    """Golden Rooster's orthonormal ray directions (section "ChiSao Exploration": the
    near-exhaustion refill shoots rays in orthonormal directions obtained by QR): for each
    peak c, the n <= d rows of G [C][n][d] (Gaussian draws) are replaced by the rows of Q from
    G_c^T = Q R with R's diagonal positive, which makes Q unique.  Reading: a row whose
    |R_kk| (its norm after removing the earlier directions) is at most 1e-12 of its own norm
    depends on the earlier rows; it and every later row become NaN, since the rows after it
    have no well-defined orthonormal completion from these draws."""
    G = _f64(G)
    out = np.empty_like(G)
    for c in range(G.shape[0]):
        Q, R = np.linalg.qr(G[c].T)
        r = np.diag(R)
        sgn = np.where(r < 0, -1.0, 1.0)
        out[c] = (Q * sgn).T
        bad = np.abs(r) <= 1e-12 * np.linalg.norm(G[c], axis=1)
        if bad.any():
            out[c, int(np.argmax(bad)):] = np.nan
    return out


def log_volume(lo, hi) -> float:
    lo = _f64(lo)
    hi = _f64(hi)
    return lib().or_log_volume(lo.size, _p(lo), _p(hi))


def precheck(prob, eps_flat=0.0, eps_soft=0.0, op: Optional[OracleProblem] = None):
    """Preprocessing: sensitivities s, classes (0 active, 1 flat, 2 soft nuisance) and the
    marginal log-evidence of the flagged coordinates."""
    op = op or OracleProblem(prob)
    d = prob.d
    s = np.zeros(d)
    cls = np.zeros(d, dtype=np.int32)
    lz = C.c_double(np.nan)
    st = lib().or_precheck(op.ptr, _p(op.beta()), _p(op.lo), _p(op.hi), eps_flat, eps_soft,
                           _p(s), _p(cls), C.byref(lz))
    return dict(status=st, s=s, cls=cls, logz_marginal=lz.value)


def eig_reduce(H, lo, hi, eps_inform, eps_nuisance):
    """Dimensional reduction at a mode (section "Module 4: GraspBirdsTail", its algorithm
    summary): eigendecomposition of the symmetric part of H = -grad^2 l (numpy.linalg.eigh as
    the library primitive), eigenvalues in descending order, classes 0 informative
    (lambda > eps_inform), 1 nuisance (eps_nuisance < lambda <= eps_inform), 2 degenerate
    (lambda <= eps_nuisance), the marginal log-evidence: 1/2 log(2 pi / lambda) per nuisance
    direction and, per degenerate direction, the log of the box's extent along it,
    sum_j |v_j| (hi_j - lo_j) (the paper's prior width Delta_i, read for a rotated direction),
    summed pairwise in index order; d_eff = number of informative directions."""
    Hs = 0.5 * (_f64(H) + _f64(H).T)
    w, V = np.linalg.eigh(Hs)
    order = np.argsort(-w, kind="stable")
    w, V = w[order], V[:, order]
    cls = np.where(w > eps_inform, 0, np.where(w > eps_nuisance, 1, 2)).astype(np.int32)
    width = np.abs(V).T @ (_f64(hi) - _f64(lo))
    safe_w = np.where(cls == 1, w, 1.0)
    terms = np.where(cls == 1, 0.5 * np.log(2.0 * np.pi / safe_w),
                     np.where(cls == 2, np.log(width), 0.0))
    return dict(eigval=w, V=V, cls=cls, logz_marginal=pairwise_sum(terms),
                d_eff=int(np.sum(cls == 0)))


def fd_derivatives(f, X, eps, full=False):
    """Finite-difference derivatives of a generic log-likelihood f (a Python callable on one
    point) at each row of X (appendix "Gradient and Hessian Computation": central-difference
    gradient, diagonal Hessian from the same perturbations, off-diagonal entries from the four
    points x +- eps e_i +- eps e_j), plain loops in the formulas' order.  Returns l [B],
    grad [B][d], hdiag [B][d] and, with full, H [B][d][d] (symmetric, diagonal = hdiag).
    Parity unpinned only in the sense that the stencils are the method; they are checked
    against analytic derivatives in the CPU tests."""
    X = np.atleast_2d(_f64(X))
    B, d = X.shape
    l = np.zeros(B)
    g = np.zeros((B, d))
    hd = np.zeros((B, d))
    H = np.zeros((B, d, d)) if full else None
    for b in range(B):
        x = X[b]
        f0 = f(x)
        l[b] = f0
        for i in range(d):
            xp = x.copy()
            xp[i] = x[i] + eps
            xm = x.copy()
            xm[i] = x[i] - eps
            fp, fm = f(xp), f(xm)
            g[b, i] = (fp - fm) / (2.0 * eps)
            hd[b, i] = (fp - 2.0 * f0 + fm) / (eps * eps)
        if full:
            for i in range(d):
                H[b, i, i] = hd[b, i]
                for j in range(i + 1, d):
                    v = {}
                    for si in (1.0, -1.0):
                        for sj in (1.0, -1.0):
                            xx = x.copy()
                            xx[i] = x[i] + si * eps
                            xx[j] = x[j] + sj * eps
                            v[(si, sj)] = f(xx)
                    h = (v[(1.0, 1.0)] - v[(1.0, -1.0)] - v[(-1.0, 1.0)] + v[(-1.0, -1.0)]) / (
                        4.0 * eps * eps)
                    H[b, i, j] = H[b, j, i] = h
    return dict(l=l, grad=g, hdiag=hd, H=H, probe_b=_fd_probe(f, X, eps, l, hd))


def _fd_probe(f, X, eps, l, hd):
    """Off-diagonal probe of the rotation detection (appendix "Rotation Detection"):
    b = (v^T H v - a) / (d - 1), v = (1, ..., 1) / sqrt(d), a = mean(H_ii), with v^T H v from
    the central second difference along v (two more evaluations); 0 for d = 1."""
    B, d = X.shape
    out = np.zeros(B)
    if d == 1:
        return out
    vi = 1.0 / math.sqrt(d)
    for b in range(B):
        x = X[b]
        fp = f(x + eps * vi)
        fm = f(x - eps * vi)
        vhv = (fp - 2.0 * l[b] + fm) / (eps * eps)
        out[b] = (vhv - float(np.mean(hd[b]))) / (d - 1)
    return out


def user_mode_evidence(f, modes, lo, hi, eps, rot_tol):
    """Laplace evidence of a generic log-likelihood at given modes with finite-difference
    curvature (module BendTheBow's geometry detection and evidence calculation): per mode the
    diagonal H_ii and the probe b from one batch of perturbations; when |b| > rot_tol * |mean
    H_ii| the full FD Hessian and log det(-H) by a Cholesky factorisation (numpy), else
    sum log(-H_ii); log Z_k = l + (d/2) log 2 pi - log det / 2 - log V; log Z = logsumexp.
    Returns None for a mode whose -H is not positive definite."""
    modes = np.atleast_2d(_f64(modes))
    n, d = modes.shape
    lv = log_volume(lo, hi)
    r = fd_derivatives(f, modes, eps, full=False)
    out = dict(logl=r["l"].copy(), logdet=np.zeros(n), full=np.zeros(n, dtype=bool),
               mode_log_z=np.zeros(n))
    for k in range(n):
        a = float(np.mean(r["hdiag"][k]))
        if abs(r["probe_b"][k]) > rot_tol * abs(a):
            out["full"][k] = True
            Hk = fd_derivatives(f, modes[k:k + 1], eps, full=True)["H"][0]
            st, _ = cholesky(-Hk)
            if st:
                return None
            out["logdet"][k] = logdet_spd(-Hk)
        else:
            if np.any(r["hdiag"][k] >= 0):
                return None
            out["logdet"][k] = pairwise_sum(np.log(-r["hdiag"][k]))
        out["mode_log_z"][k] = mode_log_z(d, out["logl"][k], out["logdet"][k], lv)
    out["log_z"] = logsumexp(np.sort(out["mode_log_z"])[::-1])
    return out


def mode_log_z(d, logl_v, log_det_h, log_vol) -> float:
    return lib().or_mode_log_z(d, logl_v, log_det_h, log_vol)


@dataclass
class OracleResult:
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


def _result(st, r, d, cap, modes, mlz, mll, ldh) -> OracleResult:
    n = min(r.n_modes, cap) if st == OK else 0
    return OracleResult(st, r.log_z, r.n_modes, modes[:n].copy(), mlz[:n].copy(), mll[:n].copy(),
                        ldh[:n].copy(), r.n_logl_evals, r.n_grad_evals, r.n_hess_evals,
                        r.iterations, r.n_rejected_nonpd, r.n_dead_starts, r.n_candidates,
                        r.n_reps_pre)


def evidence(prob, cfg, n_threads: int = 0, n_starts: Optional[int] = None,
             problem: int = 0) -> OracleResult:
    """Run the whole path on the CPU.  ``n_starts`` overrides cfg.n_starts (fewer rays too);
    ``problem`` is the problem's index within a batch (Philox counter word 3)."""
    op = OracleProblem(prob)
    ns = cfg.n_starts if n_starts is None else n_starts
    nr = cfg.n_rays if n_starts is None else max(ns, cfg.n_rays * ns // cfg.n_starts)
    c = _Config(nr, cfg.n_points, ns, cfg.m, cfg.max_iter, cfg.max_modes, cfg.grad_tol,
                cfg.dedup_tol, cfg.dedup_tol_pre, cfg.seed, n_threads, problem)
    cap = cfg.max_modes
    d = prob.d
    modes = np.zeros((cap, d))
    mlz = np.zeros(cap)
    mll = np.zeros(cap)
    ldh = np.zeros(cap)
    r = _Result()
    r.modes, r.mode_log_z, r.mode_logl, r.log_det_h = (_p(modes).value, _p(mlz).value,
                                                       _p(mll).value, _p(ldh).value)
    st = lib().or_evidence(op.ptr, _p(op.lo), _p(op.hi), C.byref(c), C.byref(r))
    return _result(st, r, d, cap, modes, mlz, mll, ldh)


def reference_modes(prob, dedup_tol: float = 0.0, max_modes: int = 64) -> OracleResult:
    """Expected mode set of a synthetic problem: Newton from each mu_k, filtered and deduplicated."""
    op = OracleProblem(prob)
    d = prob.d
    modes = np.zeros((max_modes, d))
    mlz = np.zeros(max_modes)
    mll = np.zeros(max_modes)
    ldh = np.zeros(max_modes)
    r = _Result()
    r.modes, r.mode_log_z, r.mode_logl, r.log_det_h = (_p(modes).value, _p(mlz).value,
                                                       _p(mll).value, _p(ldh).value)
    st = lib().or_reference_modes(op.ptr, _p(op.lo), _p(op.hi), dedup_tol, max_modes, C.byref(r))
    return _result(st, r, d, max_modes, modes, mlz, mll, ldh)
