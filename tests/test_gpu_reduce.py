"""Eigendecomposition and dimensional reduction at the modes (cyclic Jacobi, FP64) against
the oracle (numpy.linalg.eigh).

Eigenvalues agree to n eps |H| (a backward-stable method on both sides); eigenvectors of
well-separated eigenvalues agree up to sign; V is orthogonal and V diag(lambda) V^T
reproduces H; classes and d_eff match wherever no eigenvalue lies within that tolerance of a
threshold, and the marginal log-evidence within the bound its terms inherit from the
eigenvalue and eigenvector errors.
"""
import numpy as np
import pytest

import oracle as O
from paper_2601_19957_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    from paper_2601_19957_amd import _lib

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    _lib.lib()
    return _lib


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def spectrum_matrix(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    q = synth.haar_orthogonal(rng, n)
    lam = np.exp(rng.uniform(np.log(1e-9), np.log(50.0), n))
    return (q * lam[None, :]) @ q.T


def check(L, Hs, lo, hi, eps_i, eps_n):
    C, n, _ = Hs.shape
    out = L.sb_eig_reduce_dev(dev(Hs), dev(lo), dev(hi), eps_i, eps_n)
    ev = out["eigval"].cpu().numpy()
    V = out["V"].cpu().numpy()
    cls = out["cls"].cpu().numpy()
    lz = out["logz_marginal"].cpu().numpy()
    assert out["sweeps"] <= 40
    for c in range(C):
        ref = O.eig_reduce(Hs[c], lo, hi, eps_i, eps_n)
        scale = float(np.max(np.abs(ref["eigval"])))
        tol = 8.0 * n * 2.2e-16 * scale
        assert np.max(np.abs(ev[c] - ref["eigval"])) <= tol, c
        assert np.max(np.abs(V[c].T @ V[c] - np.eye(n))) <= 1e-12 * max(1, n) ** 0.5
        assert np.max(np.abs((V[c] * ev[c]) @ V[c].T - 0.5 * (Hs[c] + Hs[c].T))) <= 4 * tol
        # eigenvectors of eigenvalues separated from their neighbours by > 1e-6 of the scale
        gap = np.minimum(np.abs(np.diff(ref["eigval"], prepend=np.inf)),
                         np.abs(np.diff(ref["eigval"], append=-np.inf)))
        sep = gap > 1e-6 * scale
        dots = np.abs(np.sum(V[c] * ref["V"], axis=0))
        assert np.all(np.abs(dots[sep] - 1.0) < 1e-6), c
        near = (np.abs(ref["eigval"] - eps_i) <= tol) | (np.abs(ref["eigval"] - eps_n) <= tol)
        assert np.array_equal(cls[c][~near], ref["cls"][~near])
        if not near.any():
            assert out["d_eff"][c] == ref["d_eff"]
            # the marginal's sensitivity: a nuisance term moves by |d lambda| / (2 lambda); a
            # degenerate term by |d width| / width, where width = sum_j |v_j| (hi_j - lo_j) and
            # an eigenvector is determined to ~ n eps |H| / gap (clustered tiny eigenvalues
            # leave their eigenvectors ill-determined, on both sides)
            w = np.abs(ref["V"]).T @ (hi - lo)
            eta = np.minimum(8.0 * n * 2.2e-16 * scale / np.maximum(gap, 1e-300), 2.0)
            dterm = np.where(ref["cls"] == 2, np.sqrt(n) * eta * np.max(hi - lo) / w,
                             np.where(ref["cls"] == 1,
                                      0.5 * tol / np.maximum(ref["eigval"], 1e-300), 0.0))
            bound = 1e-9 * max(1.0, abs(ref["logz_marginal"])) + float(np.sum(dterm))
            assert abs(lz[c] - ref["logz_marginal"]) <= bound, (c, bound)


@pytest.mark.parametrize("n,C", [(1, 2), (2, 3), (7, 2), (33, 3), (64, 1), (200, 2)])
def test_eig_reduce_constructed(L, n, C):
    """Batches of matrices with eigenvalues log-uniform over 1e-9..50 (all three classes);
    odd n exercises the dummy index of the round-robin pairing."""
    Hs = np.stack([spectrum_matrix(n, 100 * n + c) for c in range(C)])
    lo = -np.linspace(1.0, 4.0, n)
    hi = np.linspace(2.0, 6.0, n)
    check(L, Hs, lo, hi, 1.0, 1e-4)


def test_eig_reduce_mode_hessians(L):
    """The exact Hessians H_k = -grad^2 l at the modes of a mixture (sb_hessian_dev at the
    means), all informative: d_eff = d, marginal 0."""
    rng = np.random.Generator(np.random.PCG64(81))
    prob = synth.gaussian_mixture(rng, 48, 3, -8.0, 8.0, 0.05, 1.0, 12.0, box_half=12.0,
                                  norm=synth.NORM_DENSITY, linf_min=1.0)
    m = L.DeviceModel(prob)
    H = L.sb_hessian_dev(m, dev(prob.mu))
    Hs = H.cpu().numpy()
    check(L, Hs, prob.lo, prob.hi, 0.01, 1e-6)
    out = L.sb_eig_reduce_dev(H, dev(prob.lo), dev(prob.hi), 0.01, 1e-6)
    assert out["d_eff"] == [48, 48, 48]


def test_eig_reduce_d1024(L):
    """The d = 1024 Gaussian's Hessian at its mode (its precision), one matrix."""
    prob = synth.make_problem("c4a")
    check(L, prob.prec.copy(), prob.lo, prob.hi, 10.0, 1.5)


def test_eig_reduce_rejects_bad_thresholds(L):
    H = dev(np.eye(3)[None])
    lo, hi = dev(-np.ones(3)), dev(np.ones(3))
    with pytest.raises(L.SbError):
        L.sb_eig_reduce_dev(H, lo, hi, 1e-3, 1.0)


def test_eig_reduce_reports_the_sweep_cap(L, monkeypatch):
    """The convergence test runs after the last allowed sweep too: a dense matrix capped at one
    sweep is still above 4 n eps |A|_F and comes back SB_E_NOCONV (outputs written); with the
    default cap it converges; a diagonal matrix needs no sweep even with a cap of 0."""
    rng = np.random.default_rng(7)
    A = rng.normal(size=(16, 16))
    H = dev((A @ A.T + 16 * np.eye(16))[None])
    lo, hi = dev(-np.ones(16)), dev(np.ones(16))
    monkeypatch.setenv("SB_JACOBI_MAX_SWEEPS", "1")
    with pytest.raises(L.SbError) as ei:
        L.sb_eig_reduce_dev(H, lo, hi, 1e-3, 1e-6)
    assert ei.value.status == L.E_NOCONV and "after 1 sweeps" in str(ei.value)
    monkeypatch.setenv("SB_JACOBI_MAX_SWEEPS", "0")
    out = L.sb_eig_reduce_dev(dev(np.diag(np.arange(1.0, 17.0))[None]), lo, hi, 1e-3, 1e-6)
    assert out["sweeps"] == 0
    monkeypatch.delenv("SB_JACOBI_MAX_SWEEPS")
    out = L.sb_eig_reduce_dev(H, lo, hi, 1e-3, 1e-6)
    assert 1 < out["sweeps"] < 40
