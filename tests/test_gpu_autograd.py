"""The autograd Function over the hand-written gradient and HVP kernels:
first and second derivatives against the oracle's analytic ones and against
central differences of the GPU's own l."""
import numpy as np
import pytest

import oracle as O
from paper_2601_19957_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    from paper_2601_19957_amd import _lib, autograd

    assert torch.cuda.is_available()
    return _lib, autograd


def problems():
    rng = np.random.Generator(np.random.PCG64(3))
    mix = synth.gaussian_mixture(rng, 12, 3, -8, 8, 0.05, 1.0, 12.0, box_half=12.0,
                                 norm=synth.NORM_DENSITY, linf_min=1.0)
    t = synth.student_t(np.random.Generator(np.random.PCG64(4)), 10, 5.0, -5, 5, 0.05, 1.0, 20.0)
    return {"mix": mix, "t": t}


@pytest.mark.parametrize("name", ["mix", "t"])
def test_backward_matches_oracle_gradient(mods, name):
    L, A = mods
    prob = problems()[name]
    m = L.DeviceModel(prob)
    Xn = synth.points_near_modes(prob, 7, 2, scale=0.5)
    X = torch.tensor(Xn, device="cuda", requires_grad=True)
    w = torch.linspace(0.5, 2.0, 7, device="cuda", dtype=torch.float64)
    (A.logl(m, X) * w).sum().backward()
    _, go = O.logl(prob, Xn)
    err = float(np.max(np.abs(X.grad.cpu().numpy() - w.cpu().numpy()[:, None] * go)))
    assert err <= 1e-11 * max(1.0, float(np.abs(go).max())), err


@pytest.mark.parametrize("name", ["mix", "t"])
def test_double_backward_is_oracle_hvp(mods, name):
    L, A = mods
    prob = problems()[name]
    m = L.DeviceModel(prob)
    Xn = synth.points_near_modes(prob, 5, 3, scale=0.4)
    V = np.random.default_rng(9).standard_normal(Xn.shape)
    X = torch.tensor(Xn, device="cuda", requires_grad=True)
    (g,) = torch.autograd.grad(A.logl(m, X).sum(), X, create_graph=True)
    (hv,) = torch.autograd.grad((g * torch.tensor(V, device="cuda")).sum(), X)
    ref = O.hvp(prob, Xn, V)
    err = float(np.max(np.abs(hv.cpu().numpy() - ref)))
    assert err <= 1e-11 * max(1.0, float(np.abs(ref).max())), err


def test_functional_hvp_and_gradcheck(mods):
    L, A = mods
    prob = problems()["mix"]
    m = L.DeviceModel(prob)
    x = torch.tensor(synth.points_near_modes(prob, 1, 5, scale=0.3), device="cuda")
    v = torch.ones_like(x)
    f = lambda z: A.logl(m, z).sum()
    _, hv = torch.autograd.functional.hvp(f, x, v)
    ref = O.hvp(prob, x.cpu().numpy(), v.cpu().numpy())
    assert float(np.max(np.abs(hv.cpu().numpy() - ref))) <= 1e-10 * float(np.abs(ref).max())
    xs = torch.tensor(synth.points_near_modes(prob, 2, 6, scale=0.3), device="cuda",
                      requires_grad=True)
    assert torch.autograd.gradcheck(lambda z: A.logl(m, z), (xs,), eps=1e-6, atol=1e-5)
    assert torch.autograd.gradgradcheck(lambda z: A.logl(m, z), (xs,), eps=1e-6, atol=1e-4)


def test_float32_path(mods):
    L, A = mods
    prob = problems()["mix"]
    m = L.DeviceModel(prob, low_precision=True)
    Xn = synth.points_near_modes(prob, 4, 7, scale=0.3)
    X = torch.tensor(Xn, device="cuda", dtype=torch.float32, requires_grad=True)
    A.logl(m, X).sum().backward()
    _, go = O.logl(prob, Xn)
    err = float(np.max(np.abs(X.grad.double().cpu().numpy() - go)))
    assert err <= 1e-4 * max(1.0, float(np.abs(go).max())), err
