"""Preprocessing probe (dimensional pathology detection) on the GPU against the oracle.

Sensitivities are differences of FP64 log-likelihoods at the 2d + 1 probe points, which the
two sides sum in different orders: relative agreement ~1e-12 of the l values, so s agrees to
1e-9 relative (plus an absolute floor of 1e-9 |l|).  Classes are integers decided by comparing
s with thresholds from the same s: they must match wherever s_i is not within that tolerance
of a threshold.  The marginal log-evidence is a sum of logarithms of these quantities.
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


def mixture(d, K, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.gaussian_mixture(rng, d, K, -8.0, 8.0, 0.05, 1.0, 12.0 if K > 1 else 0.0,
                                  box_half=12.0, norm=synth.NORM_DENSITY, linf_min=1.0)


def t_problem(d, seed, nu):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.student_t(rng, d, nu, -5.0, 5.0, 0.01, 1.0, 20.0)


CASES = {
    "nuisance_d37": lambda: synth.nuisance_gaussian(37, 3, 4, seed=61, centred=False),
    "nuisance_d300": lambda: synth.nuisance_gaussian(300, 20, 9, seed=62),
    "mix_d64_K3": lambda: mixture(64, 3, 63),
    "t_d70": lambda: t_problem(70, 64, 4.0),
    "d1": lambda: mixture(1, 1, 65),
    "c4a": lambda: synth.make_problem("c4a"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_precheck_matches_oracle(L, name):
    prob = CASES[name]()
    ref = O.precheck(prob)
    assert ref["status"] == 0
    m = L.DeviceModel(prob)
    out = L.sb_precheck_dev(m)
    s = out["s"].cpu().numpy()
    cls = out["cls"].cpu().numpy()
    lz = float(out["logz_marginal"].cpu().numpy()[0])
    # |l| scale of the probe values, for the absolute floor
    X = np.vstack([0.5 * (prob.lo + prob.hi)])
    l0 = abs(float(O.logl(prob, X, grad=False)[0]))
    tol = 1e-9 * np.abs(ref["s"]) + 1e-9 * max(1.0, l0)
    assert np.all(np.abs(s - ref["s"]) <= tol), float(np.max(np.abs(s - ref["s"]) / tol))
    med, mx = np.median(ref["s"]), np.max(ref["s"])
    near = (np.abs(ref["s"] - 1e-6 * med) <= 2 * tol) | (np.abs(ref["s"] - 1e-3 * mx) <= 2 * tol)
    assert np.array_equal(cls[~near], ref["cls"][~near])
    assert out["n_flat"] == int((cls == 1).sum()) and out["n_soft"] == int((cls == 2).sum())
    if not near.any():
        assert abs(lz - ref["logz_marginal"]) <= 1e-9 * max(1.0, abs(ref["logz_marginal"]))


def test_precheck_flags_the_constructed_coordinates(L):
    """Ragged d (not a multiple of any tile), flat and soft coordinates spread through the
    index range by a permutation of the constructed problem."""
    base = synth.nuisance_gaussian(133, 7, 5, seed=66)
    perm = np.random.default_rng(67).permutation(133)
    prob = synth.Problem(**{**vars(base), "mu": base.mu[:, perm],
                            "prec": base.prec[:, perm][:, :, perm]})
    out = L.sb_precheck_dev(L.DeviceModel(prob))
    cls = out["cls"].cpu().numpy()
    want = np.zeros(133, dtype=np.int32)
    want[:7] = 1
    want[7:12] = 2
    assert np.array_equal(cls, want[perm])
    D = 0.5 * (prob.hi - prob.lo)
    sig = 1.0 / np.sqrt(np.diag(prob.prec[0]))
    ref = float(np.sum(np.log(2 * D[want[perm] == 1])) +
                np.sum(0.5 * np.log(2 * np.pi) + np.log(sig[want[perm] == 2])))
    assert abs(float(out["logz_marginal"].cpu().numpy()[0]) - ref) <= 1e-10 * abs(ref)


def test_precheck_non_finite_probe_is_an_error(L):
    """A box so wide that l overflows to -inf at the probe points: SB_E_INVAL, as the oracle."""
    prob = mixture(6, 1, 68)
    prob = synth.Problem(**{**vars(prob), "lo": np.full(6, -1e300), "hi": np.full(6, 1e300)})
    assert O.precheck(prob)["status"] == -1
    with pytest.raises(L.SbError):
        L.sb_precheck_dev(L.DeviceModel(prob))
