"""The split-BF16 contraction (dtype F32_SPLIT) and its operand copies.

FP32 data v is carried as hi = bf16(v) plus lo = bf16(v - hi); each product
is formed as hi*hi + hi*lo + lo*hi with FP32 accumulation.  Per product the
dropped lo*lo and the two representation remainders are each below about
2^-16 of |x y|, so every output obeys |Y - Y_exact| <= 2^-14 sum_j |P_nj
delta_j| (this also absorbs the FP32 rounding of delta and of the d-term
sums).  A missing cross term would exceed that bound by ~2^6.
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


def gaussian(d, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = synth.gaussian_mixture(rng, d, 1, -8.0, 8.0, 1e-3, 1.0, 0.0, box_half=30.0,
                               norm=synth.NORM_PEAK_ZERO)
    p.mu = p.mu.astype(np.float32).astype(np.float64)  # the GPU's FP32 mean, exactly
    return p


@pytest.mark.parametrize("d,B", [(8, 5), (64, 300), (200, 129), (1024, 260)])
def test_split_contraction_within_bound(L, d, B):
    prob = gaussian(d, 900 + d)
    X = synth.random_points(prob, B, 901, spread=0.7).astype(np.float32).astype(np.float64)
    m = L.DeviceModel(prob, low_precision=True)
    _, g = L.sb_logl_grad_dev(m, torch.as_tensor(X, device="cuda").float(),
                              dtype=L.DTYPE_F32_SPLIT)
    g = g.double().cpu().numpy()
    _, g_ref = O.logl(prob, X)  # K = 1: grad l = -P (x - mu), exactly the contraction
    delta = X - prob.mu[0]
    bound = 2.0 ** -14 * (np.abs(delta) @ np.abs(prob.prec[0]).T) + 1e-30
    ratio = float(np.max(np.abs(g - g_ref) / bound))
    assert ratio <= 1.0, ratio


def test_split_quadform_matches_fp32_kernel(L):
    """Same FP32 data through the FP32 and the split contraction: Y agree to the split bound."""
    prob = synth.make_problem("c1")
    X = torch.as_tensor(synth.points_near_modes(prob, 300, 5, scale=1.0), device="cuda").float()
    m = L.DeviceModel(prob, low_precision=True)
    q32 = L.QuadForm(m, X)
    qs = L.QuadForm(m, X, dtype=L.DTYPE_F32_SPLIT)
    q32()
    qs()
    torch.cuda.synchronize()
    y32, ys = q32.Y.double().cpu().numpy(), qs.Y.double().cpu().numpy()
    delta = X.double().cpu().numpy()[:, None, :] - prob.mu[None, :, :]
    bound = 2.0 ** -13 * np.einsum("bkj,knj->bkn", np.abs(delta), np.abs(prob.prec))
    err = np.abs(ys - y32).reshape(bound.shape)
    assert float(np.max(err / (bound + 1e-30))) <= 1.0


def test_split_copy_bits(L):
    """hi / lo bit patterns against torch's round-to-nearest-even BF16 conversion."""
    rng = np.random.Generator(np.random.PCG64(77))
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.uniform(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 3.0e38, -1e-30, 65504.0]])
    xd = torch.as_tensor(x, device="cuda")
    hi = torch.empty(x.size, dtype=torch.int16, device="cuda")
    lo = torch.empty(x.size, dtype=torch.int16, device="cuda")
    L._check(L.lib().sb_split_bf16_dev(x.size, xd.data_ptr(), hi.data_ptr(), lo.data_ptr(), 0),
             "sb_split_bf16_dev")
    torch.cuda.synchronize()
    t = torch.as_tensor(x.astype(np.float32))
    hi_ref = t.to(torch.bfloat16)
    lo_ref = torch.as_tensor((x - hi_ref.double().numpy()).astype(np.float32)).to(torch.bfloat16)
    assert torch.equal(hi.cpu(), hi_ref.view(torch.int16))
    assert torch.equal(lo.cpu(), lo_ref.view(torch.int16))


@pytest.mark.parametrize("name", ["c1", "t_d256"])
def test_split_logl_grad(L, name):
    if name == "c1":
        prob = synth.make_problem("c1")
    else:
        rng = np.random.Generator(np.random.PCG64(5))
        prob = synth.student_t(rng, 256, 30.0, -5.0, 5.0, 0.01, 1.0, 20.0)
    X = synth.points_near_modes(prob, 200, 13, scale=0.5)
    lo, go = O.logl(prob, X)
    m = L.DeviceModel(prob, low_precision=True)
    l, g = L.sb_logl_grad_dev(m, torch.as_tensor(X, device="cuda").float(),
                              dtype=L.DTYPE_F32_SPLIT)
    l, g = l.double().cpu().numpy(), g.double().cpu().numpy()
    q_scale = np.maximum(1.0, np.abs(lo - O.prep(prob)[1].max()))
    el = float(np.max(np.abs(l - lo) / (q_scale + np.abs(lo))))
    eg = float(np.max(np.abs(g - go) / np.maximum(1.0, np.abs(go).max(axis=1, keepdims=True))))
    assert el < 5e-4 and eg < 5e-4, (el, eg)


TILES = ["128x128x32", "128x128x64", "256x128x32", "128x256x32", "256x256x32",
         "128x128x32x2", "256x256x32x2"]


@pytest.fixture
def forced_tile(request):
    import os

    old = os.environ.get("SB_TILE")
    os.environ["SB_TILE"] = request.param
    yield request.param
    if old is None:
        os.environ.pop("SB_TILE", None)
    else:
        os.environ["SB_TILE"] = old


@pytest.mark.parametrize("forced_tile", TILES, indirect=True)
@pytest.mark.parametrize("d,B", [(200, 300), (1024, 129)])
def test_split_every_tile_variant(L, forced_tile, d, B):
    """Each tile variant the autotuner may pick, on ragged row and column tails."""
    prob = gaussian(d, 950 + d)
    X = synth.random_points(prob, B, 951, spread=0.7).astype(np.float32).astype(np.float64)
    m = L.DeviceModel(prob, low_precision=True)
    _, g = L.sb_logl_grad_dev(m, torch.as_tensor(X, device="cuda").float(),
                              dtype=L.DTYPE_F32_SPLIT)
    g = g.double().cpu().numpy()
    _, g_ref = O.logl(prob, X)
    delta = X - prob.mu[0]
    bound = 2.0 ** -14 * (np.abs(delta) @ np.abs(prob.prec[0]).T) + 1e-30
    assert float(np.max(np.abs(g - g_ref) / bound)) <= 1.0


@pytest.mark.parametrize("forced_tile", ["128x128x32", "128x256x32", "256x256x32", "128x128x32x2",
                                         "256x256x32x2"], indirect=True)
@pytest.mark.parametrize("npts", [32, 6, 3])  # 6: rows straddle rays; 3: per-point path
def test_bf16_discovery_every_tile_variant(L, forced_tile, npts):
    """BF16 ray-point contraction per tile variant: the best BF16 sample of each ray lies
    within the BF16 error bound of the ray's FP64 maximum."""
    rng = np.random.Generator(np.random.PCG64(61))
    prob = synth.gaussian_mixture(rng, 96, 2, -8.0, 8.0, 0.05, 1.0, 12.0, box_half=12.0,
                                  norm=synth.NORM_DENSITY, linf_min=1.0)
    R = 96
    m = L.DeviceModel(prob, low_precision=True)
    out = L.sb_discover_dev(m, R, npts, 32, 7, dtype=L.DTYPE_BF16)
    ref = O.discover(prob, R, npts, 32, 7)
    P0o, P1o = O.rays(prob.d, prob.lo, prob.hi, R, 7)
    bj = out["ray_best_j"].cpu().numpy()
    pts = P0o + ((bj + 0.5) / npts)[:, None] * (P1o - P0o)
    lv = O.logl(prob, pts, grad=False)
    gap = ref["ray_best_l"] - lv
    assert float(gap.min()) >= -1e-9
    assert float(np.max(gap / np.maximum(1.0, np.abs(ref["ray_best_l"])))) < 0.05


@pytest.mark.parametrize("d,K,B,tile2", [(64, 4, 300, None), (200, 3, 129, None),
                                         (1024, 8, 260, None), (256, 6, 2000, None),
                                         (256, 6, 2000, "256x256x32x2"),
                                         (1024, 8, 260, "256x256x32x2")])
def test_split_pairs_contraction(L, d, K, B, tile2, monkeypatch):
    """The contraction of listed (row, component) pairs, as the screened mixture bulk runs it:
    every listed pair's Y block and q partial sum to the split bound of the oracle's
    P_k (x - mu_k); unlisted blocks are left untouched.  Rows are listed for one or two
    components each, with uneven list lengths and an empty component; the fourth case spans
    several row tiles per component; the last two take 256 x 256 tiles (SB_TILE2)."""
    if tile2:
        monkeypatch.setenv("SB_TILE2", tile2)
    import ctypes as C

    rng = np.random.Generator(np.random.PCG64(950 + d))
    prob = synth.gaussian_mixture(rng, d, K, -8.0, 8.0, 1e-3, 1.0, 0.0, box_half=30.0,
                                  norm=synth.NORM_DENSITY, linf_min=0.5)
    prob.mu = prob.mu.astype(np.float32).astype(np.float64)
    X = synth.random_points(prob, B, 951, spread=0.7).astype(np.float32).astype(np.float64)
    lists = [[] for _ in range(K)]
    for r in range(B):
        lists[r % (K - 1)].append(r)  # component K - 1 gets no rows
        if r % 3 == 0:
            lists[(r + 1) % (K - 1)].append(r)
    cnt = np.array([len(v) for v in lists], dtype=np.int32)
    rows = np.zeros((K, B), dtype=np.int32)
    for k in range(K):
        rows[k, :cnt[k]] = lists[k]
    m = L.DeviceModel(prob, low_precision=True)
    Xd = torch.as_tensor(X, device="cuda").float()
    ntn_max = (d + 63) // 64
    Y = torch.full((B, K * d), float("nan"), dtype=torch.float32, device="cuda")
    qp = torch.zeros((B, K, ntn_max), dtype=torch.float32, device="cuda")
    mv = m.view(L.DTYPE_F32_SPLIT)
    nt = C.c_int32()
    g = torch.as_tensor(cnt, device="cuda")
    rw = torch.as_tensor(rows, device="cuda")
    st = L.lib().sb_quadform_pairs_dev(C.byref(mv), B, Xd.data_ptr(), g.data_ptr(),
                                       rw.data_ptr(), B, Y.data_ptr(), qp.data_ptr(),
                                       C.byref(nt), None)
    assert st == 0, L.last_error()
    torch.cuda.synchronize()
    Yh = Y.double().cpu().numpy().reshape(B, K, d)
    ntn = nt.value  # q partials are [B][K][ntn] with the launch's tile count
    qh = qp.double().cpu().numpy().reshape(-1)[:B * K * ntn].reshape(B, K, ntn)
    listed = np.zeros((B, K), dtype=bool)
    for k in range(K):
        listed[rows[k, :cnt[k]], k] = True
    for b in range(B):
        for k in range(K):
            if not listed[b, k]:
                assert np.all(np.isnan(Yh[b, k]))
                continue
            delta = X[b] - prob.mu[k]
            y_ref = prob.prec[k] @ delta
            bound = 2.0 ** -14 * (np.abs(prob.prec[k]) @ np.abs(delta)) + 1e-30
            assert float(np.max(np.abs(Yh[b, k] - y_ref) / bound)) <= 1.0, (b, k)
            q_ref = float(delta @ y_ref)
            qb = 2.0 ** -13 * float(np.abs(delta) @ np.abs(prob.prec[k]) @ np.abs(delta)) + 1e-30
            assert abs(float(qh[b, k].sum()) - q_ref) <= qb, (b, k)

