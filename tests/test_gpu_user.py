"""Generic user log-likelihoods: run-time compiled HIP source, batched evaluation, and the
finite-difference gradient, diagonal and full Hessian and rotation probe, against the oracle's
finite differences of the same function written in numpy and against analytic derivatives.

The two sides evaluate f in different rounding orders (|df| of a few eps_mach |f|), which the
stencils divide by eps (gradient) or eps^2 (Hessian): the tolerances carry those factors.
"""
import numpy as np
import pytest

import oracle as O
from paper_2601_19957_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPSM = 2.220446049250313e-16

GAUSS_SRC = r"""
// -(x - mu)^T P (x - mu) / 2 + c with params = [P (d*d), mu (d), c]
__device__ double gauss(const double *x, int d, const double *p) {
  const double *P = p, *mu = p + d * d;
  double q = 0.0;
  for (int i = 0; i < d; ++i) {
    double r = 0.0;
    for (int j = 0; j < d; ++j) r += P[i * d + j] * (x[j] - mu[j]);
    q += (x[i] - mu[i]) * r;
  }
  return p[d * d + d] - 0.5 * q;
}
"""

ROSEN_SRC = r"""
__device__ double rosen(const double *x, int d, const double *p) {
  double s = 0.0;
  for (int i = 0; i + 1 < d; ++i) {
    const double a = x[i + 1] - x[i] * x[i], b = 1.0 - x[i];
    s += 100.0 * a * a + b * b;
  }
  return -s;
}
"""


@pytest.fixture(scope="module")
def L():
    from paper_2601_19957_amd import _lib

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    _lib.lib()
    return _lib


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def gauss_case(d, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    P, _ = synth.random_precision(rng, d, 0.2, 2.0)
    mu = rng.uniform(-1, 1, d)
    c = 1.5
    f = lambda x: c - 0.5 * (x - mu) @ P @ (x - mu)
    params = np.concatenate([P.ravel(), mu, [c]])
    return P, mu, f, params


@pytest.mark.parametrize("d", [1, 5, 37])
def test_user_gaussian_matches_oracle_and_closed_form(L, d):
    P, mu, f, params = gauss_case(d, 200 + d)
    fn = L.UserLogL(GAUSS_SRC, "gauss")
    X = np.random.default_rng(d).uniform(-2, 2, (7, d))
    pd = dev(params)
    l = fn.logl(dev(X), pd).cpu().numpy()
    fref = np.array([f(x) for x in X])
    fs = np.max(np.abs(fref)) + 1.0
    assert np.max(np.abs(l - fref)) <= 8 * d * EPSM * fs
    eps = 1e-3
    full = d <= 5
    out = fn.fd(dev(X), eps, pd, full=full)
    ref = O.fd_derivatives(f, X, eps, full=full)
    tol_g = 16 * d * EPSM * fs / eps
    tol_h = 32 * d * EPSM * fs / eps ** 2
    g = out["grad"].cpu().numpy()
    hd = out["hdiag"].cpu().numpy()
    assert np.max(np.abs(g - ref["grad"])) <= tol_g
    assert np.max(np.abs(hd - ref["hdiag"])) <= tol_h
    # central differences are exact on quadratics up to that rounding
    assert np.max(np.abs(g + (X - mu) @ P)) <= tol_g
    assert np.max(np.abs(hd + np.diag(P))) <= tol_h
    assert np.max(np.abs(out["probe_b"].cpu().numpy() - ref["probe_b"])) <= 4 * tol_h
    if full:
        H = out["H"].cpu().numpy()
        assert np.max(np.abs(H - ref["H"])) <= tol_h
        assert np.max(np.abs(H + P[None])) <= tol_h


def test_user_rosenbrock_full_hessian(L):
    """A quartic with ragged d: full FD Hessian against the oracle's stencils."""
    d = 9
    fn = L.UserLogL(ROSEN_SRC, "rosen")

    def f(x):
        return -np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1.0 - x[:-1]) ** 2)

    X = np.random.default_rng(5).uniform(-1.2, 1.2, (4, d))
    eps = 1e-4
    out = fn.fd(dev(X), eps, None, full=True)
    ref = O.fd_derivatives(f, X, eps, full=True)
    fs = max(abs(f(x)) for x in X) + 1.0
    assert np.max(np.abs(out["l"].cpu().numpy() - ref["l"])) <= 8 * d * EPSM * fs
    assert np.max(np.abs(out["grad"].cpu().numpy() - ref["grad"])) <= 16 * d * EPSM * fs / eps
    assert np.max(np.abs(out["H"].cpu().numpy() - ref["H"])) <= 32 * d * EPSM * fs / eps ** 2


def test_user_rotation_probe_uniform_correlation(L):
    """H = a0 I + b0 (1 1^T - I): the probe returns b0; axis-aligned: 0."""
    d, a0, b0 = 16, -3.0, 0.25
    Hm = a0 * np.eye(d) + b0 * (np.ones((d, d)) - np.eye(d))
    fn = L.UserLogL(GAUSS_SRC, "gauss")
    X = np.random.default_rng(9).uniform(-1, 1, (3, d))
    out = fn.fd(dev(X), 1e-3, dev(np.concatenate([-Hm.ravel(), np.zeros(d), [0.0]])))
    assert np.max(np.abs(out["probe_b"].cpu().numpy() - b0)) <= 1e-6
    out2 = fn.fd(dev(X), 1e-3, dev(np.concatenate([np.eye(d).ravel(), np.zeros(d), [0.0]])))
    assert np.max(np.abs(out2["probe_b"].cpu().numpy())) <= 1e-6


def test_user_compile_error_is_reported(L):
    with pytest.raises(L.SbError):
        L.UserLogL("__device__ double f(const double *x, int d, const double *p) { return ; }",
                   "f")
    assert "error" in L.last_error()
