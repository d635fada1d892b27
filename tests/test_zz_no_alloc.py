"""The allocation-free logL + gradient entry point (sb_logl_grad_noalloc_dev) against the
workspace one (sb_logl_grad_dev) through the C ABI: two calls in a row, the second with a
smaller input, each equal to the workspace entry point's result to the FP64 / FP32 bar of
the logL + gradient parity tests; sizes beyond the static scratch are rejected."""
import numpy as np
import pytest

from paper_2601_19957_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    from paper_2601_19957_amd import _lib

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    _lib.lib()
    return _lib


def _mixture(d, K, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.gaussian_mixture(rng, d, K, -8.0, 8.0, 0.05, 1.0, 12.0 if K > 1 else 0.0,
                                  box_half=12.0, norm=synth.NORM_DENSITY, linf_min=1.0)


@pytest.mark.parametrize("dtype", ["f64", "f32", "split"])
@pytest.mark.parametrize("d,K", [(64, 4), (256, 1)])
def test_noalloc_matches_workspace_entry(L, dtype, d, K):
    prob = _mixture(d, K, 1300 + d + K)
    low = dtype != "f64"
    m = L.DeviceModel(prob, low_precision=low)
    dt = {"f64": L.DTYPE_F64, "f32": L.DTYPE_F32, "split": L.DTYPE_F32_SPLIT}[dtype]
    tol = 1e-12 if dtype == "f64" else 1e-5
    for B in (2000, 333):  # the second call smaller: the scratch keeps the first call's data
        Xh = synth.points_near_modes(prob, B, 77 + B, scale=1.0)
        X = torch.as_tensor(Xh, device="cuda")
        if low:
            X = X.float()
        l_ref, g_ref = L.sb_logl_grad_dev(m, X, dtype=dt)
        l = torch.full_like(l_ref, float("nan"))
        g = torch.full_like(g_ref, float("nan"))
        L.sb_logl_grad_noalloc_dev(m, X, l, g, dtype=dt)
        torch.cuda.synchronize()
        lr, gr = l_ref.double().cpu().numpy(), g_ref.double().cpu().numpy()
        la, ga = l.double().cpu().numpy(), g.double().cpu().numpy()
        assert np.all(np.isfinite(la)) and np.all(np.isfinite(ga))
        el = float(np.max(np.abs(la - lr) / np.maximum(1.0, np.abs(lr))))
        eg = float(np.max(np.abs(ga - gr)) / max(1.0, float(np.max(np.abs(gr)))))
        assert el <= tol and eg <= tol, (B, el, eg)
        # l only
        l2 = torch.full_like(l_ref, float("nan"))
        L.sb_logl_grad_noalloc_dev(m, X, l2, None, dtype=dt)
        torch.cuda.synchronize()
        e2 = float(np.max(np.abs(l2.double().cpu().numpy() - lr) / np.maximum(1.0, np.abs(lr))))
        assert e2 <= tol


def test_noalloc_rejects_sizes_beyond_the_scratch(L):
    import ctypes as C

    prob = _mixture(1024, 8, 1400)
    m = L.DeviceModel(prob)
    B = 4096  # 4096 x 8 x 1024 FP64 rows of Y: 256 MiB, beyond 32 MiB
    X = torch.zeros((B, 1024), dtype=torch.float64, device="cuda")
    l = torch.empty(B, dtype=torch.float64, device="cuda")
    mv = m.view(L.DTYPE_F64)
    st = L.lib().sb_logl_grad_noalloc_dev(C.byref(mv), B, X.data_ptr(), l.data_ptr(), None,
                                          L.DTYPE_F64, None)
    assert st == L.E_NOMEM and "static" in L.last_error()
