"""Seeded synthetic evidence problems (inputs only).

This module builds the likelihood parameters and prior boxes that both the
HIP path and the CPU oracle consume.  It holds none of the method's
arithmetic: it draws orthogonal matrices, eigenvalues, mixture weights and
separated means, and nothing here evaluates a likelihood, optimises, or forms
an evidence.

Problem shapes follow the five workloads the method is measured on:

* ``c0``: one correlated Gaussian, peak-zero normalisation, d=4, box +-10.
* ``c1``: K=4 Gaussian mixture (normalised density), d=64, box +-12,
  Mahalanobis separation >= 12.
* ``c2``: multivariate Student-t (nu=30, normalised density), d=256, box +-20.
* ``c3``: 512 independent mixtures with d log-uniform in 8..512, K in 1..4,
  per-problem box of half-width 3*max|mu|.
* ``c4a``: one Gaussian, peak-zero, d=1024, lambda in [1e-3, 1], box +-30.
* ``c4b``: K=8 Gaussian mixture (density), d=1024, separation >= 15, box +-30.

Covariances are Sigma = Q diag(lambda) Q^T with Q Haar-orthogonal (QR of a
Gaussian matrix with the sign fix of Mezzadri, 2007) and lambda log-uniform;
the problem stores the precision P = Q diag(1/lambda) Q^T (symmetrised) and
sum(log lambda) for closed-form checks.  Seeds default to 2601199570 + c.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

SEED_BASE = 2601199570

FAMILY_GAUSS_MIX = 0
FAMILY_STUDENT_T = 1
NORM_PEAK_ZERO = 0
NORM_DENSITY = 1
PREC_FP64 = 0
PREC_MIXED = 1


@dataclasses.dataclass
class Problem:
    """One evidence problem: likelihood family + parameters + uniform box prior."""

    family: int
    norm: int
    d: int
    K: int
    log_w: np.ndarray  # [K] float64
    mu: np.ndarray  # [K, d] float64
    prec: np.ndarray  # [K, d, d] float64, symmetric positive definite
    nu: float
    logl_offset: float
    lo: np.ndarray  # [d]
    hi: np.ndarray  # [d]
    sum_log_lambda: np.ndarray  # [K]: sum_i log(lambda_i) of each covariance
    name: str = ""

    def copy(self) -> "Problem":
        return dataclasses.replace(
            self,
            log_w=self.log_w.copy(),
            mu=self.mu.copy(),
            prec=self.prec.copy(),
            lo=self.lo.copy(),
            hi=self.hi.copy(),
            sum_log_lambda=self.sum_log_lambda.copy(),
        )


@dataclasses.dataclass
class RunConfig:
    """Run parameters of one evidence call (mirrors the C ``sb_config``)."""

    n_rays: int
    n_points: int
    n_starts: int
    m: int = 8
    max_iter: int = 0  # <= 0: default 10*d + 200
    max_modes: int = 64
    precision: int = PREC_FP64
    grad_tol: float = 0.0  # <= 0: default
    dedup_tol: float = 0.0  # <= 0: default 1e-6 * max box width
    seed: int = 0
    dedup_tol_pre: float = 0.0  # <= 0: default 0.25


# ----------------------------------------------------------------- primitives

def haar_orthogonal(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of N(0,1)^{d x d}, columns sign-fixed."""
    z = rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def log_uniform(rng: np.random.Generator, a: float, b: float, size) -> np.ndarray:
    return np.exp(rng.uniform(math.log(a), math.log(b), size))


def random_precision(rng: np.random.Generator, d: int, lam_lo: float, lam_hi: float):
    """Return (P, sum(log lambda)) with Sigma = Q diag(lambda) Q^T, P = Sigma^-1."""
    q = haar_orthogonal(rng, d)
    lam = log_uniform(rng, lam_lo, lam_hi, d)
    p = (q * (1.0 / lam)[None, :]) @ q.T
    p = 0.5 * (p + p.T)
    return p, float(np.sum(np.log(lam)))


def dirichlet_ones(rng: np.random.Generator, k: int) -> np.ndarray:
    e = rng.exponential(1.0, k)
    return e / e.sum()


def _separated_means(rng, K, d, lo, hi, precs, sum_log_lam, log_w, sep, linf_min,
                     max_tries=10000):
    """Draw K means uniform in [lo, hi]^d, rejecting until every pair satisfies:

    * Mahalanobis separation min(D_Pi, D_Pj) >= sep,
    * the other component's density at each mean is < e^-60 of the own one
      (weights and normalisations included),
    * L-infinity distance >= linf_min.
    """
    half_logdet = [-0.5 * s for s in sum_log_lam]  # 0.5*log det P_k
    for _ in range(max_tries):
        mu = rng.uniform(lo, hi, (K, d))
        ok = True
        for i in range(K):
            for j in range(i + 1, K):
                v = mu[i] - mu[j]
                di2 = float(v @ precs[i] @ v)
                dj2 = float(v @ precs[j] @ v)
                if min(di2, dj2) < sep * sep or np.max(np.abs(v)) < linf_min:
                    ok = False
                    break
                # density of component j at mu_i relative to component i at mu_i (and vice versa)
                r_ji = (log_w[j] - log_w[i]) + (half_logdet[j] - half_logdet[i]) - 0.5 * dj2
                r_ij = (log_w[i] - log_w[j]) + (half_logdet[i] - half_logdet[j]) - 0.5 * di2
                if r_ji > -60.0 or r_ij > -60.0:
                    ok = False
                    break
            if not ok:
                break
        if ok:
            return mu
    raise RuntimeError("could not draw separated means")


def gaussian_mixture(rng, d, K, mu_lo, mu_hi, lam_lo, lam_hi, sep, box_half=None,
                     box_from_mu=None, norm=NORM_DENSITY, name="", linf_min=2.5) -> Problem:
    precs, sll = [], []
    for _ in range(K):
        p, s = random_precision(rng, d, lam_lo, lam_hi)
        precs.append(p)
        sll.append(s)
    w = dirichlet_ones(rng, K) if K > 1 else np.ones(1)
    log_w = np.log(w)
    if K > 1:
        mu = _separated_means(rng, K, d, mu_lo, mu_hi, precs, sll, log_w, sep, linf_min)
    else:
        mu = rng.uniform(mu_lo, mu_hi, (1, d))
    if box_from_mu is not None:
        h = box_from_mu * float(np.max(np.abs(mu)))
    else:
        h = box_half
    lo = np.full(d, -h)
    hi = np.full(d, h)
    return Problem(FAMILY_GAUSS_MIX, norm, d, K, log_w, mu, np.stack(precs), 0.0, 0.0,
                   lo, hi, np.array(sll), name)


def hidden_mode_mixture(d: int, seed: int, offset: float = 5.0, box_half: float = 10.0,
                        name: str = "hidden") -> Problem:
    """Two equally weighted Gaussians (density-normalised) in the box +-box_half: a narrow
    component at the box centre (lambda in [0.2, 0.3]) and a wide one (lambda in [6, 12])
    whose mean sits at +offset in the first two coordinates.  The narrow component's peak is
    far higher, so every coarse ray that passes near the centre outranks every point of the
    wide component's basin; its basin is small, so moving a sample a few units from the
    centre puts it in the wide component's basin."""
    rng = np.random.Generator(np.random.PCG64(seed))
    PA, slA = random_precision(rng, d, 0.2, 0.3)
    PB, slB = random_precision(rng, d, 6.0, 12.0)
    mu = np.zeros((2, d))
    mu[1, :min(2, d)] = offset
    return Problem(FAMILY_GAUSS_MIX, NORM_DENSITY, d, 2, np.log(np.array([0.5, 0.5])), mu,
                   np.stack([PA, PB]), 0.0, 0.0, np.full(d, -box_half), np.full(d, box_half),
                   np.array([slA, slB]), name=name)


def student_t(rng, d, nu, mu_lo, mu_hi, lam_lo, lam_hi, box_half, name="") -> Problem:
    p, s = random_precision(rng, d, lam_lo, lam_hi)
    mu = rng.uniform(mu_lo, mu_hi, (1, d))
    return Problem(FAMILY_STUDENT_T, NORM_DENSITY, d, 1, np.zeros(1), mu, p[None], float(nu),
                   0.0, np.full(d, -box_half), np.full(d, box_half), np.array([s]), name)


def nuisance_gaussian(d: int, n_flat: int, n_soft: int, seed: int, box_half: float = 10.0,
                      flat_scale: float = 1e6, soft_scale: float = 30.0,
                      centred: bool = True) -> Problem:
    """Peak-zero Gaussian with degenerate coordinates, for the preprocessing probe.

    Coordinates 0..n_flat-1 have standard deviation flat_scale box half-widths (unconstrained
    by the likelihood), the next n_soft soft_scale half-widths (weakly constrained); the others
    form a dense correlated block with eigenvalues of Sigma log-uniform in [0.05, 1] (squared
    half-widths).  The flagged coordinates are uncorrelated with the block.  The mean is the
    box centre (centred) or uniform in the inner half of the box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    na = d - n_flat - n_soft
    if na < 1 or n_flat < 0 or n_soft < 0:
        raise ValueError("need at least one constrained coordinate")
    p = np.zeros((d, d))
    nf = n_flat + n_soft
    sig = np.concatenate([np.full(n_flat, flat_scale), np.full(n_soft, soft_scale)]) * box_half
    p[np.arange(nf), np.arange(nf)] = 1.0 / sig ** 2
    pa, sa = random_precision(rng, na, 0.05 * box_half ** 2, box_half ** 2)
    p[nf:, nf:] = pa
    mu = np.zeros((1, d)) if centred else rng.uniform(-0.5 * box_half, 0.5 * box_half, (1, d))
    sll = sa + float(np.sum(2.0 * np.log(sig)))
    return Problem(FAMILY_GAUSS_MIX, NORM_PEAK_ZERO, d, 1, np.zeros(1), mu, p[None], 0.0, 0.0,
                   np.full(d, -box_half), np.full(d, box_half), np.array([sll]),
                   f"nuisance_d{d}")


# ------------------------------------------------------------- the workloads

def c3_dimension(u: float) -> int:
    """d = clamp(round(exp(U[ln 8, ln 512])), 8, 512) from a uniform draw u in [0,1)."""
    v = math.exp(math.log(8.0) + u * (math.log(512.0) - math.log(8.0)))
    return int(min(512, max(8, round(v))))


def make_problem(name: str, seed: Optional[int] = None, d: Optional[int] = None,
                 n_problems: Optional[int] = None):
    """Build the named workload's problem(s).  ``d``/``n_problems`` shrink it for tests."""
    idx = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4a": 4, "c4b": 4}[name]
    if seed is None:
        seed = SEED_BASE + idx + (1000 if name == "c4b" else 0)
    rng = np.random.Generator(np.random.PCG64(seed))
    if name == "c0":
        dd = d or 4
        return gaussian_mixture(rng, dd, 1, -5.0, 5.0, 0.1, 1.0, 0.0, box_half=10.0,
                                norm=NORM_PEAK_ZERO, name=name)
    if name == "c1":
        dd = d or 64
        return gaussian_mixture(rng, dd, 4, -8.0, 8.0, 0.05, 1.0, 12.0, box_half=12.0,
                                norm=NORM_DENSITY, name=name)
    if name == "c2":
        dd = d or 256
        return student_t(rng, dd, 30.0, -5.0, 5.0, 0.01, 1.0, 20.0, name=name)
    if name == "c4a":
        dd = d or 1024
        return gaussian_mixture(rng, dd, 1, -8.0, 8.0, 1e-3, 1.0, 0.0, box_half=30.0,
                                norm=NORM_PEAK_ZERO, name=name)
    if name == "c4b":
        dd = d or 1024
        return gaussian_mixture(rng, dd, 8, -8.0, 8.0, 1e-3, 1.0, 15.0, box_half=30.0,
                                norm=NORM_DENSITY, name=name)
    if name == "c3":
        n = n_problems or 512
        out = []
        for pi in range(n):
            dd = d or c3_dimension(float(rng.uniform()))
            K = int(rng.integers(1, 5))
            out.append(gaussian_mixture(rng, dd, K, -8.0, 8.0, 0.05, 1.0, 12.0,
                                        box_from_mu=3.0, norm=NORM_DENSITY,
                                        name=f"c3[{pi}]"))
        return out
    raise KeyError(name)


# rays x points, starts, precision for each workload
RUN_TABLE = {
    "c0": dict(n_rays=256, n_points=32, n_starts=64, precision=PREC_FP64),
    "c1": dict(n_rays=4096, n_points=32, n_starts=4096, precision=PREC_FP64),
    "c2": dict(n_rays=8192, n_points=32, n_starts=8192, precision=PREC_FP64),
    "c3": dict(n_rays=1024, n_points=32, n_starts=1024, precision=PREC_FP64),
    "c4a": dict(n_rays=16384, n_points=32, n_starts=16384, precision=PREC_MIXED),
    "c4b": dict(n_rays=16384, n_points=32, n_starts=16384, precision=PREC_MIXED),
}


def make_run_config(name: str, n_starts: Optional[int] = None, precision: Optional[int] = None,
                    seed: int = 12345, **kw) -> RunConfig:
    t = dict(RUN_TABLE[name])
    if n_starts is not None:
        t["n_rays"] = max(n_starts, t["n_rays"] * n_starts // t["n_starts"])
        t["n_starts"] = n_starts
    if precision is not None:
        t["precision"] = precision
    t.update(kw)
    return RunConfig(seed=seed, **t)


def make_workload(name: str, n_starts: Optional[int] = None, d: Optional[int] = None,
                  precision: Optional[int] = None, seed: Optional[int] = None,
                  n_problems: Optional[int] = None, **kw) -> Tuple[object, RunConfig]:
    prob = make_problem(name, seed=seed, d=d, n_problems=n_problems)
    return prob, make_run_config(name, n_starts=n_starts, precision=precision, **kw)


def random_points(problem: Problem, n: int, seed: int, spread: float = 1.0) -> np.ndarray:
    """n points uniform in the problem's box scaled about its centre by ``spread``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = 0.5 * (problem.lo + problem.hi)
    h = 0.5 * (problem.hi - problem.lo) * spread
    return c + rng.uniform(-1.0, 1.0, (n, problem.d)) * h


def points_near_modes(problem: Problem, n: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """n points at mu_k + scale * N(0, I), cycling over components."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.arange(n) % problem.K
    return problem.mu[k] + scale * rng.standard_normal((n, problem.d))


def random_spd(d: int, seed: int, cond: float = 100.0, batch: int = 1) -> np.ndarray:
    """Batch of SPD matrices with eigenvalues log-uniform in [1, cond]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(batch):
        q = haar_orthogonal(rng, d)
        lam = log_uniform(rng, 1.0, cond, d)
        a = (q * lam[None, :]) @ q.T
        out.append(0.5 * (a + a.T))
    return np.stack(out)


def lbfgs_history(d: int, m: int, cnt: int, seed: int, batch: int = 1):
    """Random L-BFGS histories with positive curvature pairs (s^T y > 0).

    Returns S, Y [batch, m, d] (logical order, oldest first; rows >= cnt are
    zero) and G [batch, d].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    S = np.zeros((batch, m, d))
    Y = np.zeros((batch, m, d))
    for b in range(batch):
        A = random_spd(d, seed + 7 + b, cond=50.0)[0]
        for j in range(cnt):
            s = rng.standard_normal(d)
            S[b, j] = s
            Y[b, j] = A @ s
    G = rng.standard_normal((batch, d))
    return S, Y, G


def as_list(p) -> List[Problem]:
    return p if isinstance(p, list) else [p]
