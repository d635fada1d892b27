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
        L.or_finish_points.restype = i32
        L.or_finish_points.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp]
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
    |R_kk| (its norm after removing the earlier directions) is at most 8 n eps of its own norm
    (eps = 2^-52) depends on the earlier rows: removing n projections leaves a rounding residue
    of order n eps |g_k| even from an exactly dependent row, so a residual at that level carries
    no direction of its own.  It and every later row become NaN, since the rows after it have no
    well-defined orthonormal completion from these draws."""
    G = _f64(G)
    out = np.empty_like(G)
    n = G.shape[1]
    thr = 8.0 * n * np.finfo(np.float64).eps
    for c in range(G.shape[0]):
        Q, R = np.linalg.qr(G[c].T)
        r = np.diag(R)
        sgn = np.where(r < 0, -1.0, 1.0)
        out[c] = (Q * sgn).T
        bad = np.abs(r) <= thr * np.linalg.norm(G[c], axis=1)
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


def reduced_logl(prob, theta_star, V, r, Phi):
    """The reduced likelihood of section "Module 4: GraspBirdsTail" (compacted likelihood and
    algorithm summary): l_red(phi) = l(theta* + V_inform phi) with V_inform the first r
    columns of V (the informative eigenvectors, eigenvalues in descending order), phi in R^r;
    the paper writes the displacement as V_info^T phi, read here as the combination of the
    informative columns (the only product whose shapes agree).  Returns l_red [B] and its
    gradient V_inform^T grad l [B][r] (chain rule)."""
    th = _f64(theta_star)
    Vi = _f64(V)[:, :r]
    P = np.atleast_2d(_f64(Phi))
    X = th[None, :] + P @ Vi.T
    l, g = logl(prob, X)
    return l, g @ Vi


def reduced_bounds(theta_star, V, r, lo, hi):
    """Bounds in the reduced space (section "Module 4: GraspBirdsTail", its exports): for each
    informative direction i the interval of t with theta* + t V[:, i] inside the box, i.e.
    the intersection over coordinates j with V_ji != 0 of the t where lo_j <= theta*_j +
    t V_ji <= hi_j (a direction that never leaves the box along some coordinate puts no
    bound there).  Returns (phi_lo [r], phi_hi [r])."""
    th, Vm, lo, hi = _f64(theta_star), _f64(V), _f64(lo), _f64(hi)
    plo = np.full(r, -np.inf)
    phi = np.full(r, np.inf)
    for i in range(r):
        for j in range(th.size):
            v = Vm[j, i]
            if v == 0.0:
                continue
            a, b = (lo[j] - th[j]) / v, (hi[j] - th[j]) / v
            plo[i] = max(plo[i], min(a, b))
            phi[i] = min(phi[i], max(a, b))
    return plo, phi


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


# ------------------------------------------------------------- ChiSao cycle

# Counter word 2 of the cycle's draws: CHISAO_STREAM0 + 8 * oscillation + purpose, purpose 0
# (Repulse Monkey directions), 2 (Golden Rooster rows), 4 (Hands Like Clouds perturbations);
# each normal takes the uniforms of streams s and s + 1 (the discovery rays use 0..2).
CHISAO_STREAM0 = 16


def chisao_normal(seed, problem, row, stream, i) -> float:
    """Standard normal draw i of counter row `row`: the cosine branch of Box-Muller, as the
    sunburst rays draw their directions, from uniform i of streams `stream` and `stream` + 1."""
    u1 = rng_uniform(seed, problem, row, stream, i)
    u2 = rng_uniform(seed, problem, row, stream + 1, i)
    return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)


@dataclass
class ChiSaoParams:
    """Parameters of the oscillation cycle (section "ChiSao Exploration").  The paper gives
    n_osc = 3 and the momentum 0.9; the rest are left open there and are parameters here."""
    n_osc: int = 3
    n_conv: int = 0            # L-BFGS steps per convergence phase (<= 0: the run's max_iter)
    stick_tol: float = 1e-6    # gradient L-infinity tolerance of stick detection
    n_reseed_pts: int = 32     # samples along a reseeding ray
    n_cloud: int = 1           # Hands Like Clouds steps
    n_smooth: int = 4          # perturbations per smoothed gradient
    sigma: float = 0.0         # smoothing scale (<= 0: from the free samples' spread)
    alpha_cloud: float = 0.01  # ascent step of Hands Like Clouds
    n_anti: int = 8            # anti-convergence steps
    alpha_anti: float = 0.01   # descent step of the anti-convergence phase
    momentum: float = 0.9


def chisao_sigma(X, free) -> float:
    """Automatic smoothing scale (reading of "auto-estimated from sample spread"): half the
    median over coordinates of the population standard deviation of the free samples'
    coordinates; 0 with fewer than two free samples."""
    F = _f64(np.atleast_2d(X))[np.asarray(free, dtype=bool)]
    if F.shape[0] < 2:
        return 0.0
    sd = np.sqrt(np.mean((F - np.mean(F, axis=0)) ** 2, axis=0))
    return 0.5 * float(np.median(sd))


def chisao_cycle(prob, X0, prm: ChiSaoParams, m=8, max_iter=None, grad_tol=1e-10,
                 dedup_tol=0.25, seed=0, problem=0, op: Optional[OracleProblem] = None):
    """The oscillation cycle of CarryTiger (section "ChiSao Exploration": the oscillation
    cycle and the algorithm summary of CarryTiger) on samples X0 [N][d], FP64.

    For oscillation k = 0 .. n_osc - 1:
      1. convergence: every active sample runs L-BFGS (fresh history, memory m) for at most
         n_conv accepted steps toward a local maximum (all stuck masks released);
      2. stick detection: converged-to-stick_tol and l >= l_max - ln 10 (chisao_stick over
         the active samples);
      3. dedup of the stuck samples by L-infinity leader clustering (radius dedup_tol,
         highest l first): every stuck sample that joins another's cluster is lost (its slot
         is freed); the leaders are the distinct peaks;
      4. unless k is the last oscillation and if samples were lost: with >= 5 active samples
         that did not converge, Repulse Monkey refills lost slot j (in slot order) with the
         best point of a ray from unconverged sample j mod n_unconv (slot order) in a random
         direction (chisao_reseed); with fewer, Golden Rooster (unless disabled) refills the
         lost slots round-robin over the peaks (l descending), each peak's slots taking the
         rows of QR-orthonormalised Gaussian draws (chisao_orthonormal, in chunks of d rows)
         as directions of rays from the peak; otherwise the lost slots stay empty.  Refilled
         slots are active and not stuck.  Golden Rooster disables itself for the remaining
         oscillations when the oscillation after one in which it refilled ends with no more
         distinct converged peaks (leaders of the converged samples, stuck or not) than the
         one before;
      5. unless k is the last oscillation: the free samples (active, not stuck) take n_cloud
         Hands Like Clouds steps and n_anti anti-convergence steps (chisao_explore).
    Draws: Repulse Monkey direction of slot b, coordinate i: chisao_normal(seed, problem, b,
    CHISAO_STREAM0 + 8k, i), normalised; Golden Rooster row of slot b: stream + 2; Hands Like
    Clouds perturbation (step c, draw q) of slot b: stream + 4, index (c n_smooth + q) d + i.
    Returns a dict: X [N][d], l [N], status [N] of the last convergence phase (ST_* codes,
    ST_DEAD for empty slots), active [N], and per-oscillation counts (peaks, lost, reseed
    kind: 0 none, 1 Repulse Monkey, 2 Golden Rooster)."""
    op = op or OracleProblem(prob)
    d = prob.d
    X = _f64(np.atleast_2d(X0)).copy()
    N = X.shape[0]
    lo, hi = op.lo, op.hi
    mi = max_iter if max_iter is not None else 10 * d + 200
    n_conv = prm.n_conv if prm.n_conv > 0 else mi
    active = np.ones(N, dtype=bool)
    l = np.full(N, np.nan)
    G = np.zeros((N, d))
    status = np.full(N, ST_DEAD, dtype=np.int32)
    gr_enabled, gr_used, prev_peaks = True, False, -1
    log = []
    for k in range(prm.n_osc):
        # 1. convergence phase
        for b in range(N):
            if not active[b]:
                status[b] = ST_DEAD
                continue
            r = lbfgs(prob, X[b], m=m, max_iter=n_conv, grad_tol=grad_tol, op=op)
            X[b], l[b], G[b], status[b] = r["x"], r["logl"], r["grad"], r["status"]
        conv = active & (status == ST_CONVERGED)
        # 2. stick detection over the active samples
        idx = np.flatnonzero(active)
        stuck = np.zeros(N, dtype=bool)
        if idx.size:
            stuck[idx] = chisao_stick(l[idx], G[idx], prm.stick_tol).astype(bool)
        # 3. dedup of the stuck samples
        rep_of, reps = dedup(X, l, dedup_tol, valid=stuck.astype(np.uint8))
        lost = [b for b in range(N) if stuck[b] and rep_of[b] != b]
        peaks = list(reps)
        # distinct peaks the converged samples reached (stuck or below the stick threshold)
        n_found = len(dedup(X, l, dedup_tol, valid=conv.astype(np.uint8))[1])
        if gr_used and n_found <= prev_peaks:
            gr_enabled = False
        gr_used = False
        prev_peaks = n_found
        for b in lost:
            active[b] = False
            stuck[b] = False
        kind = 0
        last = k == prm.n_osc - 1
        if not last and lost:
            base = CHISAO_STREAM0 + 8 * k
            unconv = [b for b in range(N) if active[b] and not conv[b]]
            if len(unconv) >= 5:
                kind = 1
                O_ = np.array([X[unconv[j % len(unconv)]] for j in range(len(lost))])
                U = np.zeros((len(lost), d))
                for j, b in enumerate(lost):
                    z = np.array([chisao_normal(seed, problem, b, base, i) for i in range(d)])
                    U[j] = z / np.linalg.norm(z)
                newx, _ = chisao_reseed(prob, O_, U, prm.n_reseed_pts, op=op)
                for j, b in enumerate(lost):
                    X[b] = newx[j]
            elif gr_enabled and peaks:
                kind = 2
                gr_used = True
                P = len(peaks)
                for p in range(P):
                    slots = lost[p::P]
                    for c0 in range(0, len(slots), d):
                        chunk = slots[c0:c0 + d]
                        Gr = np.array([[chisao_normal(seed, problem, b, base + 2, i)
                                        for i in range(d)] for b in chunk])
                        U = chisao_orthonormal(Gr[None])[0]
                        O_ = np.repeat(X[peaks[p]][None], len(chunk), axis=0)
                        newx, _ = chisao_reseed(prob, O_, U, prm.n_reseed_pts, op=op)
                        for j, b in enumerate(chunk):
                            X[b] = newx[j]
            if kind:
                for b in lost:
                    active[b] = True
        log.append(dict(peaks=len(peaks), found=n_found, lost=len(lost), reseed=kind,
                        converged=int(conv.sum()), golden_rooster=gr_enabled))
        if last:
            break
        # 5. Hands Like Clouds and anti-convergence on the free samples
        free = active & ~stuck
        sigma = prm.sigma if prm.sigma > 0 else chisao_sigma(X, free)
        base = CHISAO_STREAM0 + 8 * k + 4
        Z = np.zeros((prm.n_cloud, prm.n_smooth, N, d))
        for c in range(prm.n_cloud):
            for q in range(prm.n_smooth):
                for b in range(N):
                    if free[b]:
                        for i in range(d):
                            Z[c, q, b, i] = chisao_normal(seed, problem, b, base,
                                                          (c * prm.n_smooth + q) * d + i)
        frozen = (~free).astype(np.uint8)
        X = chisao_explore(prob, X, frozen, Z, sigma, prm.alpha_cloud, prm.n_anti,
                           prm.alpha_anti, prm.momentum, op=op)
    return dict(X=X, l=l, status=status, active=active, log=log)


def refine_rays(prob, P0, P1, n_pts, n_ref, delta, op: Optional[OracleProblem] = None):
    """Two-pass sampling along rays (section "Two-Pass Sampling").  Coarse pass: l at
    t_j = (j + 1/2)/n_pts.  Active region of a ray: the cells [t_j - h/2, t_j + h/2]
    (h = 1/n_pts) of its coarse samples with l_j > l_max - delta, l_max the ray's coarse
    maximum.  Refinement pass: n_ref points placed with density proportional to the
    likelihood within the active region, read as the piecewise-constant density
    exp(l_j - l_max) on the active cells and its quantiles (i + 1/2)/n_ref (stratified, so
    deterministic).  Returns per ray the best point over the coarse and refined samples
    (highest l; ties: coarse before refined, then lowest index), its l and its t."""
    op = op or OracleProblem(prob)
    P0, P1 = _f64(np.atleast_2d(P0)), _f64(np.atleast_2d(P1))
    R = P0.shape[0]
    h = 1.0 / n_pts
    best_t = np.zeros(R)
    best_l = np.full(R, -np.inf)
    T = np.zeros((R, n_ref))
    for r in range(R):
        tc = (np.arange(n_pts) + 0.5) / n_pts
        lc = logl(prob, P0[r] + tc[:, None] * (P1[r] - P0[r]), grad=False, op=op)
        fin = np.isfinite(lc)
        if not fin.any():
            best_l[r] = np.nan
            continue
        lmax = float(np.max(lc[fin]))
        act = [j for j in range(n_pts) if fin[j] and lc[j] > lmax - delta]
        w = np.array([math.exp(lc[j] - lmax) * h for j in act])
        cw = np.concatenate([[0.0], np.cumsum(w)])
        tot = cw[-1]
        tr = np.zeros(n_ref)
        for i in range(n_ref):
            u = (i + 0.5) / n_ref * tot
            a = int(np.searchsorted(cw, u, side="right")) - 1
            a = min(max(a, 0), len(act) - 1)
            tr[i] = tc[act[a]] - 0.5 * h + (u - cw[a]) / w[a] * h
        T[r] = tr
        lr = logl(prob, P0[r] + tr[:, None] * (P1[r] - P0[r]), grad=False, op=op) \
            if n_ref else np.zeros(0)
        cand_t = np.concatenate([tc, tr])
        cand_l = np.concatenate([lc, lr])
        jb = -1
        for j in range(cand_l.size):
            if math.isfinite(cand_l[j]) and (jb < 0 or cand_l[j] > cand_l[jb]):
                jb = j
        best_t[r], best_l[r] = cand_t[jb], cand_l[jb]
    return dict(best_t=best_t, best_l=best_l, t_refined=T)


def finish_points(prob, cfg, X, l, valid, n_threads: int = 0, problem: int = 0) -> OracleResult:
    """The whole path's tail from given end points (or_finish_points): pre-dedup, Newton
    polish, filters, final dedup and the Laplace combine."""
    op = OracleProblem(prob)
    X = _f64(np.atleast_2d(X))
    n = X.shape[0]
    c = _Config(cfg.n_rays, cfg.n_points, cfg.n_starts, cfg.m, cfg.max_iter, cfg.max_modes,
                cfg.grad_tol, cfg.dedup_tol, cfg.dedup_tol_pre, cfg.seed, n_threads, problem)
    cap = cfg.max_modes
    d = prob.d
    modes = np.zeros((cap, d))
    mlz = np.zeros(cap)
    mll = np.zeros(cap)
    ldh = np.zeros(cap)
    r = _Result()
    r.modes, r.mode_log_z, r.mode_logl, r.log_det_h = (_p(modes).value, _p(mlz).value,
                                                       _p(mll).value, _p(ldh).value)
    v = np.ascontiguousarray(valid, dtype=np.uint8)
    lv = _f64(l)
    st = lib().or_finish_points(op.ptr, _p(op.lo), _p(op.hi), C.byref(c), n, _p(X), _p(lv),
                                _p(v), C.byref(r))
    return _result(st, r, d, cap, modes, mlz, mll, ldh)


def evidence_chisao(prob, cfg, prm: ChiSaoParams, n_ref: int = 0, delta: float = 10.0,
                    problem: int = 0) -> OracleResult:
    """The whole path with the ChiSao cycle as its convergence (CarryTiger's algorithm
    summary): rays (or_rays), the coarse pass and, with n_ref > 0, the refinement pass
    (refine_rays); the n_starts rays of highest best l (ties: lowest ray) seed the cycle
    from their best points; the cycle's end points that are active with a finite l enter the
    tail of the single-phase path (finish_points).  FP64 throughout."""
    op = OracleProblem(prob)
    P0, P1 = rays(prob.d, prob.lo, prob.hi, cfg.n_rays, cfg.seed, problem)
    rf = refine_rays(prob, P0, P1, cfg.n_points, n_ref, delta, op=op)
    key = np.where(np.isfinite(rf["best_l"]), rf["best_l"], -np.inf)
    order = sorted(range(cfg.n_rays), key=lambda r: (-key[r], r))[:cfg.n_starts]
    X0 = np.array([P0[r] + rf["best_t"][r] * (P1[r] - P0[r]) for r in order])
    tol = cfg.grad_tol if cfg.grad_tol > 0 else 1e-10
    tau_pre = cfg.dedup_tol_pre if cfg.dedup_tol_pre > 0 else 0.25
    cyc = chisao_cycle(prob, X0, prm, m=cfg.m, max_iter=cfg.max_iter or None, grad_tol=tol,
                       dedup_tol=tau_pre, seed=cfg.seed, problem=problem, op=op)
    valid = cyc["active"] & np.isfinite(cyc["l"]) & (cyc["status"] != ST_DEAD)
    res = finish_points(prob, cfg, cyc["X"], cyc["l"], valid, problem=problem)
    res.cycle = cyc["log"]
    return res


# ------------------------------------------------ trajectory-based geometry detection

def lbfgs_user(f, x0, eps, m=8, max_iter=20, grad_tol=0.0):
    """L-BFGS on -f for a generic log-likelihood f with central finite-difference gradients
    (the rules of or_lbfgs: first step -grad f / max(1, |grad f|_inf), Armijo c1 = 1e-4 with
    halving up to 40 times, history reset then stall on failure, curvature skip
    s^T y > 1e-10 |s| |y|, stop at |grad l|_inf <= grad_tol or max_iter accepted steps),
    recording its trajectory: the start and every accepted point, with the gradient of l
    there (the TrajectoryBank of module GreenDragon, section "Trajectory Storage").
    Returns dict(X [T+1][d], G [T+1][d], status)."""
    x = _f64(x0).copy()
    d = x.size

    def lg(p):
        r = fd_derivatives(f, p[None], eps)
        return float(r["l"][0]), r["grad"][0].copy()

    l, gl = lg(x)
    Xs, Gs = [x.copy()], [gl.copy()]
    if not (math.isfinite(l) and np.all(np.isfinite(gl))):
        return dict(X=np.array(Xs), G=np.array(Gs), status=ST_DEAD)
    S, Y = [], []
    it = 0
    status = ST_MAXITER
    while True:
        g = -gl
        gn = float(np.max(np.abs(gl)))
        if gn <= grad_tol:
            status = ST_CONVERGED
            break
        if it >= max_iter:
            status = ST_MAXITER
            break
        gtp = 0.0
        if S:
            p = two_loop(np.array(S), np.array(Y), g)
            gtp = float(np.dot(g, p))
        if not S or not gtp < 0.0:
            S, Y = [], []
            p = -g * (1.0 / (gn if gn > 1.0 else 1.0))
            gtp = float(np.dot(g, p))
        alpha, ok = 1.0, False
        for _ in range(41):
            xt = x + alpha * p
            lt, glt = lg(xt)
            if math.isfinite(lt) and -lt <= -l + 1e-4 * alpha * gtp:
                ok = True
                break
            alpha *= 0.5
        if not ok:
            if S:
                S, Y = [], []
                continue
            status = ST_STALLED
            break
        sv, yv = xt - x, -glt - g
        if float(np.dot(sv, yv)) > 1e-10 * float(np.linalg.norm(sv)) * float(np.linalg.norm(yv)):
            if len(S) == m:
                S.pop(0)
                Y.pop(0)
            S.append(sv)
            Y.append(yv)
        x, l, gl = xt, lt, glt
        it += 1
        Xs.append(x.copy())
        Gs.append(gl.copy())
    return dict(X=np.array(Xs), G=np.array(Gs), status=status)


def perpendicular_step_fraction(X, G, h, rel_floor=1e-3):
    """Perpendicular step fraction of one trajectory (section "Automatic Geometry Detection",
    Step 1, and the appendix "Rotation Detection"): in coordinates whitened by sqrt(h)
    (h_i = -H_ii > 0, u = sqrt(h) theta), step t from X[t] to X[t+1] has du = sqrt(h) dtheta
    and the gradient of l at X[t] becomes gw = G[t] / sqrt(h); f_perp = |du_perp| / |du| with
    du_perp the part of du perpendicular to gw.  Reading: a step counts only while its whitened
    gradient is at least rel_floor of the trajectory's first (closer to the mode the gradient
    is at the level of the stopping rule's noise and carries no direction).  Returns the f_perp
    of the counted steps."""
    X, G = _f64(X), _f64(G)
    sh = np.sqrt(_f64(h))
    out = []
    g0 = float(np.linalg.norm(G[0] / sh)) if len(G) else 0.0
    for t in range(len(X) - 1):
        gw = G[t] / sh
        if not float(np.linalg.norm(gw)) >= rel_floor * g0 or g0 == 0.0:
            continue
        du = sh * (X[t + 1] - X[t])
        nd = float(np.linalg.norm(du))
        if nd == 0.0:
            continue
        perp = du - (float(np.dot(du, gw)) / float(np.dot(gw, gw))) * gw
        out.append(float(np.linalg.norm(perp)) / nd)
    return np.array(out)


def greendragon_seeds(mode, hdiag):
    """GreenDragon's seeds of a peak (its algorithm summary: 2d samples at
    theta* +- 0.9 w e_i): with the width read from the diagonal curvature, w_i =
    1/sqrt(-H_ii); seed 2i is theta* + 0.9 w_i e_i, seed 2i + 1 theta* - 0.9 w_i e_i."""
    mode, hdiag = _f64(mode), _f64(hdiag)
    d = mode.size
    w = 1.0 / np.sqrt(-hdiag)
    S = np.repeat(mode[None], 2 * d, axis=0)
    for i in range(d):
        S[2 * i, i] = mode[i] + 0.9 * w[i]
        S[2 * i + 1, i] = mode[i] - 0.9 * w[i]
    return S


def trajectory_geometry(f, modes, hdiag, eps, n_iter, m=8, grad_tol=0.0, rel_floor=1e-3):
    """Per mode, the largest perpendicular step fraction over the trajectories of its
    GreenDragon seeds (n_iter L-BFGS steps each, whitening h = -hdiag of the mode); NaN when no
    step counts."""
    modes, hdiag = np.atleast_2d(_f64(modes)), np.atleast_2d(_f64(hdiag))
    out = np.full(modes.shape[0], np.nan)
    for k in range(modes.shape[0]):
        vals = []
        for x0 in greendragon_seeds(modes[k], hdiag[k]):
            tr = lbfgs_user(f, x0, eps, m=m, max_iter=n_iter, grad_tol=grad_tol)
            vals.extend(perpendicular_step_fraction(tr["X"], tr["G"], -hdiag[k], rel_floor))
        if vals:
            out[k] = max(vals)
    return out


def user_mode_evidence_geo(f, modes, lo, hi, eps, rot_tol, n_iter, eps_axis, eps_rot, m=8,
                           grad_tol=0.0, eps_grad=None):
    """Laplace evidence at given modes with the two-step geometry detection of the algorithm
    "BendTheBow Evidence Calculation": Step 1, the perpendicular step fraction of the
    GreenDragon trajectories (trajectory_geometry); f_perp > eps_rot: rotated; f_perp <=
    eps_axis: axis-aligned; otherwise (or with no counted step) inconclusive, and Step 2, the
    probe b, decides (|b| > rot_tol |mean H_ii|: rotated).  Rotated modes take the full FD
    Hessian and its Cholesky log det, the others sum log(-H_ii).  decision [n]: 0 axis-aligned
    by the trajectories, 1 rotated by them, 2 axis-aligned by the probe, 3 rotated by it.
    The trajectories' gradients take the step eps_grad (default eps).  Returns None if some
    mode is not a maximum."""
    modes = np.atleast_2d(_f64(modes))
    n, d = modes.shape
    lv = log_volume(lo, hi)
    r = fd_derivatives(f, modes, eps, full=False)
    if np.any(r["hdiag"] >= 0):
        return None
    fp = trajectory_geometry(f, modes, r["hdiag"], eps if eps_grad is None else eps_grad,
                             n_iter, m=m, grad_tol=grad_tol)
    out = dict(logl=r["l"].copy(), logdet=np.zeros(n), fperp=fp,
               decision=np.zeros(n, dtype=np.int32), mode_log_z=np.zeros(n))
    for k in range(n):
        if fp[k] > eps_rot:
            dec = 1
        elif fp[k] <= eps_axis:
            dec = 0
        else:
            a = float(np.mean(r["hdiag"][k]))
            dec = 3 if abs(r["probe_b"][k]) > rot_tol * abs(a) else 2
        out["decision"][k] = dec
        if dec in (1, 3):
            Hk = fd_derivatives(f, modes[k:k + 1], eps, full=True)["H"][0]
            st, _ = cholesky(-Hk)
            if st:
                return None
            out["logdet"][k] = logdet_spd(-Hk)
        else:
            out["logdet"][k] = pairwise_sum(np.log(-r["hdiag"][k]))
        out["mode_log_z"][k] = mode_log_z(d, out["logl"][k], out["logdet"][k], lv)
    out["log_z"] = logsumexp(np.sort(out["mode_log_z"])[::-1])
    return out
