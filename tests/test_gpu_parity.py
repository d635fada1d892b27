"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Step by step on identical seeded inputs (l, grad, HVP, Hessian, Cholesky,
rays, discovery, two-loop, L-BFGS, dedup, combine), then the whole path per
workload.  FP64 tolerances follow from rounding-order differences of O(d)
sums (~d * 2^-53 relative); the mixed path is held to |d log Z| <= 1e-6.
"""
import math

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


def small_mixture(d, K, seed, box=12.0, norm=synth.NORM_DENSITY):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.gaussian_mixture(rng, d, K, -8.0, 8.0, 0.05, 1.0, 12.0 if K > 1 else 0.0,
                                  box_half=box, norm=norm, linf_min=1.0)


def t_problem(d, seed, nu=30.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.student_t(rng, d, nu, -5.0, 5.0, 0.01, 1.0, 20.0)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def rel(a, ref, floor=1.0, axis=None):
    """max |a - ref| / max(floor, |ref|) (row-wise scale when axis=1), as a float."""
    a, ref = np.asarray(a, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    if axis is None:
        sc = np.maximum(floor, np.abs(ref))
    else:
        sc = np.maximum(floor, np.abs(ref).max(axis=axis, keepdims=True))
    return float(np.max(np.abs(a - ref) / sc)) if a.size else 0.0


def absmax(a):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64)))) if np.size(a) else 0.0


PROBLEMS = {
    "c0": lambda: synth.make_problem("c0"),
    "mix_d37_K3": lambda: small_mixture(37, 3, 3),
    "mix_d200_K2": lambda: small_mixture(200, 2, 4),
    "c1": lambda: synth.make_problem("c1"),
    "t_d256": lambda: t_problem(256, 5),
    "t_d70": lambda: t_problem(70, 6, nu=4.0),
}


# ------------------------------------------------------------------ prep / A1

@pytest.mark.parametrize("name", list(PROBLEMS))
def test_prep_constants(L, name):
    prob = PROBLEMS[name]()
    st, beta, ld = O.prep(prob)
    m = L.DeviceModel(prob)
    assert np.allclose(m.beta.cpu().numpy(), beta, rtol=1e-12, atol=1e-10)
    assert np.allclose(m.logdet_prec.cpu().numpy(), ld, rtol=1e-12, atol=1e-10)


def test_prep_rejects_indefinite_and_asymmetric(L):
    prob = small_mixture(20, 2, 9)
    bad = prob.copy()
    bad.prec[1] = -bad.prec[1]
    with pytest.raises(L.SbError) as e:
        L.DeviceModel(bad)
    assert e.value.status == L.E_NOTPD
    asym = prob.copy()
    asym.prec[0, 2, 5] += 1e-6
    with pytest.raises(L.SbError) as e:
        L.DeviceModel(asym)
    assert e.value.status == L.E_NOTPD


# ---------------------------------------------------------- logl + grad / A3

@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("B", [1, 131, 300])
def test_logl_grad_fp64(L, name, B):
    prob = PROBLEMS[name]()
    X = np.concatenate([synth.points_near_modes(prob, (B + 1) // 2, 11, scale=0.8),
                        synth.random_points(prob, B // 2, 12, spread=0.9)])[:B]
    lo, go = O.logl(prob, X)
    m = L.DeviceModel(prob)
    l, g = L.sb_logl_grad_dev(m, dev(X))
    l, g = l.cpu().numpy(), g.cpu().numpy()
    el, eg = rel(l, lo), rel(g, go, axis=1)
    assert el < 1e-11 and eg < 1e-11, (el, eg)


FP64_TILES = ["64x64x16", "128x64x16", "64x128x16", "128x128x16", "64x64x32", "128x64x32",
              "64x128x32", "32x64x32"]


@pytest.mark.parametrize("tile", FP64_TILES)
@pytest.mark.parametrize("make", [lambda: small_mixture(200, 3, 31), lambda: small_mixture(37, 3, 32),
                                  lambda: t_problem(70, 33)], ids=["mix_d200_K3", "mix_d37_K3",
                                                                   "t_d70"])
def test_logl_grad_fp64_every_tile(L, tile, make, monkeypatch):
    """Each FP64 tile the autotuner may pick (BM x BN x k-tile; SB_TILE forces it) on ragged
    row and column tails: d = 200 (16-byte rows, 7 of 13 32-wide k-tiles whole), d = 37 (odd:
    the element-wise kernel), a Student-t at d = 70, 131 rows; l and the gradient equal the
    oracle's to 1e-11.  (d <= 128 problems would take the fused launch: SB_FUSED=0 keeps the
    tiled contraction.)"""
    monkeypatch.setenv("SB_TILE", tile)
    monkeypatch.setenv("SB_FUSED", "0")
    prob = make()
    X = synth.random_points(prob, 131, 34, spread=0.9)
    lo, go = O.logl(prob, X)
    m = L.DeviceModel(prob)
    l, g = (t.cpu().numpy() for t in L.sb_logl_grad_dev(m, dev(X)))
    el, eg = rel(l, lo), rel(g, go, axis=1)
    assert el < 1e-11 and eg < 1e-11, (el, eg)


@pytest.mark.parametrize("make", [lambda: small_mixture(96, 4, 21), lambda: t_problem(5, 22),
                                  lambda: small_mixture(1, 1, 23), lambda: t_problem(128, 24),
                                  lambda: small_mixture(40, 3, 26), lambda: small_mixture(64, 5, 27)],
                         ids=["mix_d96_K4", "t_d5", "gauss_d1", "t_d128", "mix_d40_K3",
                              "mix_d64_K5"])
def test_logl_grad_fp64_fused_equals_two_launch(L, make, monkeypatch):
    """Small FP64 problems take the fused launch (contraction and row epilogue in one kernel,
    d <= 128 and K * round_up(d, 32) <= 384: the first case sits at the second edge, the
    fourth at the first); 1 to 6 16-column output blocks per wave (t_d5 / gauss_d1 1, t_d128 2,
    mix_d40_K3 3, mix_d64_K5 5, mix_d96_K4 6), element-wise P loads where d is not a multiple of
    8 (t_d5, gauss_d1) and whole-run loads with lanes past d zeroed at d = 40; on a ragged last row
    tile its l equals the two-launch path's (SB_FUSED=0) to a few ulps of the O(d) sums, and l
    and the gradient equal the oracle's to 1e-11.  The two paths' gradients agree only as
    closely as their responsibilities: r_k = exp(a_k - lse) moves by r_k |dq_k| / 2, and q
    of a few 1e4 at these points carries ~1e-12 of summation-order rounding."""
    prob = make()
    B = 16 * 7 + 3
    X = synth.random_points(prob, B, 25, spread=0.9)
    m = L.DeviceModel(prob)
    l1, g1 = (t.cpu().numpy() for t in L.sb_logl_grad_dev(m, dev(X)))
    monkeypatch.setenv("SB_FUSED", "0")
    l2, g2 = (t.cpu().numpy() for t in L.sb_logl_grad_dev(m, dev(X)))
    lo, go = O.logl(prob, X)
    assert rel(l1, l2) < 1e-13 and rel(g1, g2, axis=1) < 1e-11
    assert rel(l1, lo) < 1e-11 and rel(g1, go, axis=1) < 1e-11


@pytest.mark.parametrize("name", ["mix_d37_K3", "c1", "t_d256"])
def test_logl_grad_fp32(L, name):
    prob = PROBLEMS[name]()
    X = synth.points_near_modes(prob, 200, 13, scale=0.5)
    lo, go = O.logl(prob, X)
    m = L.DeviceModel(prob, low_precision=True)
    l, g = L.sb_logl_grad_dev(m, dev(X).float())
    l, g = l.double().cpu().numpy(), g.double().cpu().numpy()
    # FP32 rounding of delta, P and the O(d) sums: ~ d * 2^-24 relative to |q|, |P delta|
    q_scale = np.maximum(1.0, np.abs(lo - O.prep(prob)[1].max()))
    el = float(np.max(np.abs(l - lo) / (q_scale + np.abs(lo))))
    eg = rel(g, go, axis=1)
    assert el < 5e-5 and eg < 5e-5, (el, eg)


FP32_TILES = ["64x64x16", "128x64x16", "64x128x16", "128x128x16", "64x64x32", "128x64x32",
              "64x128x32", "128x128x32"]


@pytest.mark.parametrize("tile", FP32_TILES)
@pytest.mark.parametrize("name", ["mix_d37_K3", "t_d256"])
def test_logl_grad_fp32_every_tile(L, tile, name, monkeypatch):
    """Each FP32 matrix-core tile (SB_TILE forces it; 16- and 32-wide k-tiles) against the
    oracle to the FP32 bound of test_logl_grad_fp32, on d = 37 (odd: the element-wise kernel)
    and a Student-t at d = 256, 131 rows (a ragged last row tile)."""
    monkeypatch.setenv("SB_TILE", tile)
    prob = PROBLEMS[name]()
    X = synth.points_near_modes(prob, 131, 14, scale=0.5)
    lo, go = O.logl(prob, X)
    m = L.DeviceModel(prob, low_precision=True)
    l, g = L.sb_logl_grad_dev(m, dev(X).float(), dtype=L.DTYPE_F32)
    l, g = l.double().cpu().numpy(), g.double().cpu().numpy()
    q_scale = np.maximum(1.0, np.abs(lo - O.prep(prob)[1].max()))
    el = float(np.max(np.abs(l - lo) / (q_scale + np.abs(lo))))
    eg = rel(g, go, axis=1)
    assert el < 5e-5 and eg < 5e-5, (el, eg)


def test_gradient_central_differences_on_gpu(L):
    """The hand-written backward against central differences of the GPU's own l (h = 1e-6)."""
    prob = synth.make_problem("c1")
    m = L.DeviceModel(prob)
    x = synth.points_near_modes(prob, 1, 21, scale=0.3)[0]
    _, g = L.sb_logl_grad_dev(m, dev(x[None]))
    g = g.cpu().numpy()[0]
    h = 1e-6
    E = np.eye(prob.d) * h
    lp = L.sb_logl_grad_dev(m, dev(x[None] + E), grad=False).cpu().numpy()
    lm = L.sb_logl_grad_dev(m, dev(x[None] - E), grad=False).cpu().numpy()
    fd = (lp - lm) / (2 * h)
    e = absmax(fd - g) / max(1.0, absmax(g))
    assert e <= 1e-6, e


# --------------------------------------------------------------- HVP / A3'

@pytest.mark.parametrize("name", ["c0", "mix_d37_K3", "c1", "t_d256", "t_d70"])
def test_hvp(L, name):
    prob = PROBLEMS[name]()
    X = synth.points_near_modes(prob, 40, 31, scale=0.6)
    V = np.random.default_rng(32).standard_normal(X.shape)
    ref = O.hvp(prob, X, V)
    m = L.DeviceModel(prob)
    hv = L.sb_hvp_dev(m, dev(X), dev(V)).cpu().numpy()
    e = rel(hv, ref, axis=1)
    assert e < 1e-11, e


# ---------------------------------------------------------- Hessian / A8

@pytest.mark.parametrize("name", ["c0", "mix_d37_K3", "mix_d200_K2", "t_d256"])
def test_hessian_assembly(L, name):
    prob = PROBLEMS[name]()
    X = synth.points_near_modes(prob, 3, 41, scale=0.2)
    m = L.DeviceModel(prob)
    H = L.sb_hessian_dev(m, dev(X)).cpu().numpy()
    for c in range(3):
        ref = O.neg_hessian(prob, X[c])
        e = absmax(H[c] - ref) / absmax(ref)
        assert e <= 1e-12, e
        assert np.array_equal(H[c], H[c].T)


def test_hessian_equals_hvp_columns(L):
    prob = small_mixture(24, 3, 8)
    m = L.DeviceModel(prob)
    x = synth.points_near_modes(prob, 1, 5, scale=0.4)
    H = L.sb_hessian_dev(m, dev(x)).cpu().numpy()[0]
    X = np.repeat(x, prob.d, axis=0)
    HV = L.sb_hvp_dev(m, dev(X), dev(np.eye(prob.d))).cpu().numpy()
    e = absmax(-HV.T - H) / absmax(H)
    assert e <= 1e-12, e


# ---------------------------------------------------------- Cholesky / A9

@pytest.mark.parametrize("n", [1, 5, 64, 65, 200, 1024])
def test_cholesky_logdet(L, n):
    A = synth.random_spd(n, 100 + n, cond=1e3, batch=3)
    Lf, ld, info = L.sb_cholesky_logdet_dev(dev(A))
    Lf, ld, info = Lf.cpu().numpy(), ld.cpu().numpy(), info.cpu().numpy()
    for c in range(3):
        st, Lo = O.cholesky(A[c])
        assert info[c] == 0 and st == 0
        e = absmax(Lf[c] - Lo) / absmax(Lo)
        assert e <= 1e-12, e
        e2 = abs(ld[c] - O.logdet_spd(A[c])) / max(1.0, abs(ld[c]))
        assert e2 <= 1e-12, e2
    b = np.random.default_rng(n).standard_normal((3, n))
    x = L.sb_cholesky_solve_dev(torch.as_tensor(Lf, device="cuda"), dev(b)).cpu().numpy()
    for c in range(3):
        ref = O.chol_solve(O.cholesky(A[c])[1], b[c])
        e = rel(x[c], ref, floor=1e-2)
        assert e <= 1e-10, e


def test_cholesky_failure_column(L):
    A = synth.random_spd(70, 3, cond=10.0, batch=2)
    A[1, 66, 66] = -5.0  # pivot 67 fails
    st, _ = O.cholesky(A[1])
    _, ld, info = L.sb_cholesky_logdet_dev(dev(A))
    info = info.cpu().numpy()
    assert info[0] == 0 and info[1] == st == 67
    assert math.isnan(float(ld[1]))


# -------------------------------------------------------------- rays / A2

@pytest.mark.parametrize("d", [4, 7, 300])
def test_rays_match_oracle(L, d):
    prob = small_mixture(d, 1, 50 + d, box=9.0)
    R = 64
    P0o, P1o = O.rays(d, prob.lo, prob.hi, R, 777)
    m = L.DeviceModel(prob)
    out = L.sb_discover_dev(m, R, 8, 8, 777)
    P0, P1 = out["P0"].cpu().numpy(), out["P1"].cpu().numpy()
    assert np.array_equal(P0[0::4], P0o[0::4]) and np.array_equal(P1[0::4], P1o[0::4])
    assert np.array_equal(P0[1::4], P0o[1::4]) and np.array_equal(P1[1::4], P1o[1::4])
    assert np.array_equal(P0[2::4], P0o[2::4]) and np.array_equal(P1[2::4], P1o[2::4])
    # sunburst: Box-Muller uses the device's log/cos (a few ulp from the host libm)
    e0, e1 = absmax(P0[3::4] - P0o[3::4]), absmax(P1[3::4] - P1o[3::4])
    assert e0 <= 1e-13 and e1 <= 1e-11, (e0, e1)


@pytest.mark.parametrize("name", ["c0", "mix_d37_K3", "t_d70"])
def test_discovery_fp64(L, name):
    prob = PROBLEMS[name]()
    R, npts, ns = 256, 32, 64
    ref = O.discover(prob, R, npts, ns, 4242)
    m = L.DeviceModel(prob)
    out = L.sb_discover_dev(m, R, npts, ns, 4242)
    bl = out["ray_best_l"].cpu().numpy()
    e = rel(bl, ref["ray_best_l"])
    assert e < 1e-11, e
    # argmax is unique where the best two samples of a ray differ clearly: compare the
    # chosen sample's value instead of its index (equal values are both correct)
    P0o, P1o = O.rays(prob.d, prob.lo, prob.hi, R, 4242)
    bj = out["ray_best_j"].cpu().numpy()
    t = (bj + 0.5) / npts
    pts = P0o + t[:, None] * (P1o - P0o)
    lv = O.logl(prob, pts, grad=False)
    e = rel(lv, ref["ray_best_l"])
    assert e < 1e-11, e
    # the chosen rays carry the n_starts largest maxima, in order
    sr = out["start_ray"].cpu().numpy()
    assert np.all(np.diff(ref["ray_best_l"][sr]) <= 1e-9 * np.abs(ref["ray_best_l"][sr[:-1]]))
    assert set(sr) == set(ref["start_ray"]) or np.sort(ref["ray_best_l"])[-ns] == \
        np.sort(ref["ray_best_l"])[-ns - 1]
    X0 = out["X0"].cpu().numpy()
    e = absmax(X0 - pts[sr]) / absmax(pts)
    assert e <= 1e-12, e


def test_discovery_top_n_ties(L):
    """A likelihood flat to FP64 precision (P = 1e-300 I): every ray's maximum is the same
    value, so the top-n rule (l descending, ties to the lower ray index) keeps rays 0..n-1.
    R is not a multiple of the ranking blocks."""
    d, R, npts, ns = 4, 333, 8, 100
    prob = synth.Problem(family=synth.FAMILY_GAUSS_MIX, norm=synth.NORM_DENSITY, d=d, K=1,
                         log_w=np.zeros(1), mu=np.zeros((1, d)),
                         prec=(1e-300 * np.eye(d))[None], nu=0.0, logl_offset=0.0,
                         lo=-np.ones(d), hi=np.ones(d), sum_log_lambda=np.array([d * 690.8]))
    ref = O.discover(prob, R, npts, ns, 5)
    assert np.all(ref["ray_best_l"] == ref["ray_best_l"][0])
    m = L.DeviceModel(prob)
    out = L.sb_discover_dev(m, R, npts, ns, 5)
    sr = out["start_ray"].cpu().numpy()
    assert np.array_equal(sr, np.arange(ns)) and np.array_equal(ref["start_ray"], np.arange(ns))


def test_discovery_bf16_ranks(L):
    """BF16 scores only rank the samples: the best BF16 sample of a ray must be
    within the BF16 error bound of the ray's true maximum (parity of values unpinned)."""
    prob = small_mixture(128, 2, 60, box=12.0)
    R, npts = 128, 32
    m = L.DeviceModel(prob, low_precision=True)
    out = L.sb_discover_dev(m, R, npts, 32, 99, dtype=L.DTYPE_BF16)
    ref = O.discover(prob, R, npts, 32, 99)
    P0o, P1o = O.rays(prob.d, prob.lo, prob.hi, R, 99)
    bj = out["ray_best_j"].cpu().numpy()
    pts = P0o + ((bj + 0.5) / npts)[:, None] * (P1o - P0o)
    lv = O.logl(prob, pts, grad=False)
    gap = ref["ray_best_l"] - lv
    assert float(gap.min()) >= -1e-9, float(gap.min())
    # |dq| <~ 2^-7 |delta|^T |P| |delta| per component; compare with the scale of q
    e = float(np.max(gap / np.maximum(1.0, np.abs(ref["ray_best_l"]))))
    assert e < 0.05, e


# ------------------------------------------------------------ two-loop / A4

@pytest.mark.parametrize("d", [4, 64, 100, 256, 700, 1024, 2047, 4096])
def test_two_loop_direction(L, d):
    B, m = 6, 8
    cnts = [0, 1, 3, 5, 8, 8]
    S = np.zeros((B, m, d))
    Y = np.zeros((B, m, d))
    G = np.zeros((B, d))
    for b in range(B):
        s_, y_, g_ = synth.lbfgs_history(d, m, cnts[b], seed=70 + b)
        S[b], Y[b], G[b] = s_[0], y_[0], g_[0]
    P = L.sb_lbfgs_direction_dev(dev(S), dev(Y), dev(G), dev(np.array(cnts, dtype=np.int32)))
    P = P.cpu().numpy()
    for b in range(B):
        ref = O.two_loop(S[b, :cnts[b]], Y[b, :cnts[b]], G[b]) if cnts[b] else -G[b]
        e = absmax(P[b] - ref) / absmax(ref)
        assert e <= 1e-12, (b, e)


@pytest.mark.parametrize("m", [16, 32])
@pytest.mark.parametrize("d", [4, 100, 1024, 4096])
def test_two_loop_direction_long_memory(L, d, m):
    """Memories beyond the register-resident 8 pairs: the history is read from memory in
    each loop of the recursion; same direction as the oracle's two-loop in FP64, and in
    FP32 within its rounding (inputs rounded to FP32 for both sides)."""
    B = 6
    cnts = [0, 1, 9, m - 1, m, m]
    S = np.zeros((B, m, d))
    Y = np.zeros((B, m, d))
    G = np.zeros((B, d))
    for b in range(B):
        s_, y_, g_ = synth.lbfgs_history(d, m, cnts[b], seed=170 + b)
        S[b], Y[b], G[b] = s_[0], y_[0], g_[0]
    cnt = dev(np.array(cnts, dtype=np.int32))
    P = L.sb_lbfgs_direction_dev(dev(S), dev(Y), dev(G), cnt).cpu().numpy()
    S32, Y32, G32 = (a.astype(np.float32).astype(np.float64) for a in (S, Y, G))
    P32 = L.sb_lbfgs_direction_dev(dev(S).float(), dev(Y).float(), dev(G).float(),
                                   cnt).cpu().numpy()
    for b in range(B):
        c = cnts[b]
        ref = O.two_loop(S[b, :c], Y[b, :c], G[b]) if c else -G[b]
        e = absmax(P[b] - ref) / absmax(ref)
        assert e <= 1e-12, (b, e)
        ref32 = O.two_loop(S32[b, :c], Y32[b, :c], G32[b]) if c else -G32[b]
        e32 = absmax(P32[b] - ref32) / absmax(ref32)
        assert e32 <= 1e-3, (b, e32)


# -------------------------------------------------------------- L-BFGS / A4-A5

@pytest.mark.parametrize("name", ["c0", "mix_d37_K3", "t_d70"])
def test_lbfgs_reaches_oracle_points(L, name):
    """Same start points, FP64: every start converges to the point the oracle's
    optimiser reaches (the paths may differ in the last bits)."""
    prob = PROBLEMS[name]()
    X0 = synth.points_near_modes(prob, 48, 81, scale=1.0)
    m = L.DeviceModel(prob)
    out = L.sb_lbfgs_dev(m, dev(X0), m=8, grad_tol=1e-10)
    st = out["status"].cpu().numpy()
    x = out["x"].cpu().numpy()
    assert int((st != L.ST_CONVERGED).sum()) == 0, np.unique(st).tolist()
    op = O.OracleProblem(prob)
    for s in range(0, 48, 5):
        r = O.lbfgs(prob, X0[s], m=8, grad_tol=1e-10, op=op)
        assert r["status"] == O.ST_CONVERGED
        e = absmax(x[s] - r["x"])
        assert e < 1e-8, (s, e)
    eg = absmax(out["grad"].cpu().numpy())
    assert eg <= 1e-10, eg


@pytest.mark.parametrize("name,m,scale,max_iter", [("mix_d37_K3", 8, 2.0, 20),
                                                    ("t_d70", 8, 2.0, 15),
                                                    ("t_d70", 1, 8.0, 30),
                                                    ("mix_d37_K3", 16, 2.0, 30),
                                                    ("t_d70", 16, 2.0, 40),
                                                    ("t_d70", 32, 2.0, 45),
                                                    ("mix_d200_K2", 32, 2.0, 45)])
def test_lbfgs_path_matches_oracle(L, name, m, scale, max_iter):
    """FP64, the same starts stopped after max_iter accepted steps, past the point where the
    history ring is full: the GPU points equal the oracle's up to rounding order, so the
    two-loop sees the oracle's history (ring order, the evicted pair dropped, a pair the
    curvature test keeps out leaving the oldest one in place; the m = 1 case from far starts
    on the heavy-tailed t meets that test's failure with the ring full; m = 16 and 32 run
    the step whose history is read from memory in each loop of the recursion).  The oracle's own
    paths move by at most ~1.2e-10 relative under 1e-15 perturbations of the starts in these
    cases (far starts with m = 16 on the nu = 4 t move by 3e-8, so none are used here)."""
    prob = PROBLEMS[name]()
    X0 = synth.points_near_modes(prob, 16, 91, scale=scale)
    md = L.DeviceModel(prob)
    out = L.sb_lbfgs_dev(md, dev(X0), m=m, max_iter=max_iter, grad_tol=1e-14)
    x = out["x"].cpu().numpy()
    st = out["status"].cpu().numpy()
    op = O.OracleProblem(prob)
    for s in range(16):
        r = O.lbfgs(prob, X0[s], m=m, max_iter=max_iter, grad_tol=1e-14, op=op)
        assert r["status"] == O.ST_MAXITER and st[s] == L.ST_MAXITER, (s, r["status"], st[s])
        e = absmax(x[s] - r["x"]) / max(1.0, absmax(r["x"]))
        assert e < 1e-8, (s, e)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_lbfgs_timed_matches_untimed(L, dtype):
    """The timed variant runs the same loop: identical results, and one duration per step."""
    prob = PROBLEMS["mix_d200_K2"]()
    X0 = synth.points_near_modes(prob, 64, 83, scale=1.0)
    md = L.DeviceModel(prob, low_precision=(dtype == "f32"))
    Xd = dev(X0) if dtype == "f64" else dev(X0).float()
    a = L.sb_lbfgs_dev(md, Xd, m=8, max_iter=40)
    b = L.sb_lbfgs_timed_dev(md, Xd, m=8, max_iter=40, n_timed=24)
    for k in ("x", "logl", "grad", "status", "iters"):
        assert torch.equal(a[k], b[k]), k
    assert a["n_evals"] == b["n_evals"]
    ran = b["step_rows"] > 0  # steps after the last one report 0
    assert int(b["step_rows"][0]) == 64 and int(ran.sum()) >= 8
    assert np.all(b["step_us"][ran] > 0) and np.all(b["step_rows"] <= 64)
    # the first step only chooses directions; counts stay within the active starts
    assert b["step_full"][0] == 0 and b["step_back"][0] == 0
    assert np.all(b["step_full"] + b["step_back"] <= b["step_rows"])
    # per-launch algorithmic bytes: -1 for the first step; where every active start accepted
    # with a full ring or halved, the (2m + 6) d and 3 d counts
    nb, es, d = b["step_bytes"], (8 if dtype == "f64" else 4), prob.d
    assert nb[0] == -1 and np.all((nb == -1) | (nb > 0) | ~ran)
    whole = ran & (b["step_full"] + b["step_back"] == b["step_rows"]) & (nb > 0)
    assert whole.any()
    ref = ((2 * 8 + 6) * b["step_full"] + 3 * b["step_back"]) * d * es
    assert np.array_equal(nb[whole], ref[whole].astype(np.float64))


@pytest.mark.parametrize("d,seed", [(200, 4), (300, 8), (520, 7)])
def test_lbfgs_bf16_history(L, d, seed):
    """FP32 L-BFGS with the history ring in BF16 (dtype F32_H16): timed and untimed runs are
    bit-identical; from points near the modes of a K = 2 mixture every start ends within the
    FP32 bulk's reach of the oracle's mode (1e-2 in L-inf, well inside the basin: the modes
    are 12 Mahalanobis units apart; the polish's job from there), as the FP32 ring does; each
    launch's byte count uses 2-byte ring vectors; m > 8 is refused.  d = 200: four values per
    thread; d = 300 (not a multiple of 8) and 520 (ragged last chunk): eight per thread, the
    element-wise ring access and the whole-chunk loads beside it."""
    prob = small_mixture(d, 2, seed)
    X0 = synth.points_near_modes(prob, 64, 84, scale=1.0)
    md = L.DeviceModel(prob, low_precision=True)
    Xd = dev(X0).float()
    a = L.sb_lbfgs_dev(md, Xd, m=8, max_iter=400, hist_bf16=True)
    b = L.sb_lbfgs_timed_dev(md, Xd, m=8, max_iter=400, n_timed=24, hist_bf16=True)
    for k in ("x", "logl", "grad", "status", "iters"):
        assert torch.equal(a[k], b[k]), k
    ref = O.reference_modes(prob)
    modes = ref.modes[:ref.n_modes]
    f = L.sb_lbfgs_dev(md, Xd, m=8, max_iter=400)
    for r in (a, f):
        x = r["x"].double().cpu().numpy()
        dist = np.abs(x[:, None, :] - modes[None, :, :]).max(axis=2).min(axis=1)
        assert float(dist.max()) < 1e-2, float(dist.max())
    ran = b["step_rows"] > 0
    nb, d = b["step_bytes"], prob.d
    whole = ran & (b["step_full"] + b["step_back"] == b["step_rows"]) & (nb > 0)
    assert whole.any()
    ref_b = ((2 * 8 * 2 + 6 * 4) * b["step_full"] + 3 * 4 * b["step_back"]) * d
    assert np.array_equal(nb[whole], ref_b[whole].astype(np.float64))
    with pytest.raises(L.SbError) as e:
        L.sb_lbfgs_dev(md, Xd, m=9, max_iter=10, hist_bf16=True)
    assert e.value.status == L.E_UNSUPPORTED

# -------------------------------------------------------------- dedup / A7

def test_dedup_handmade(L):
    X = np.array([[0.0, 0.0], [0.05, 0.0], [1.0, 1.0], [1.02, 0.99], [0.0, 0.09], [5.0, 5.0]])
    l = np.array([1.0, 3.0, 2.0, 2.0, 0.5, -1.0])
    rep_of, reps = L.sb_dedup_dev(dev(X), dev(l), 0.1)
    assert list(reps.cpu().numpy()) == [1, 2, 5]
    assert list(rep_of.cpu().numpy()) == [1, 1, 2, 2, 1, 5]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dedup_matches_oracle(L, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (500, 6))
    l = np.round(rng.standard_normal(500), 1)
    valid = rng.uniform(size=500) > 0.1
    ro, rs = O.dedup(X, l, 0.3, valid=valid)
    rep_of, reps = L.sb_dedup_dev(dev(X), dev(l), 0.3, valid=dev(valid))
    assert np.array_equal(rep_of.cpu().numpy(), ro)
    assert np.array_equal(reps.cpu().numpy(), rs)


# ------------------------------------------------------------ combine / A10

def test_combine(L):
    rng = np.random.default_rng(4)
    d, n = 9, 6
    lo, hi = -np.ones(d) * 3, np.ones(d) * 4
    logl = rng.normal(size=n) * 5
    logl[4] = logl[1]
    logdet = rng.normal(size=n)
    logdet[4] = logdet[1]
    modes = rng.normal(size=(n, d))
    order, mlz, lz = L.sb_combine_dev(dev(lo), dev(hi), dev(logl), dev(logdet), dev(modes))
    lv = O.log_volume(lo, hi)
    ref = np.array([O.mode_log_z(d, logl[i], logdet[i], lv) for i in range(n)])
    o = order.cpu().numpy()
    e = absmax(mlz.cpu().numpy() - ref[o])
    assert e <= 1e-12, e
    assert np.all(np.diff(ref[o]) <= 0)
    # the tie (modes 1 and 4) is broken lexicographically
    i1, i4 = list(o).index(1), list(o).index(4)
    assert (i1 < i4) == (tuple(modes[1]) < tuple(modes[4]))
    assert abs(float(lz) - O.logsumexp(ref[o])) < 1e-12


# ------------------------------------------------------------ whole path

def _compare(r, ref, tol_logz, tol_modes=1e-8):
    assert r.status == 0, (r.status, r.n_modes)
    assert ref.status == 0
    assert r.n_modes == ref.n_modes, (r.n_modes, ref.n_modes, r.n_reps_pre)
    dz = abs(r.log_z - ref.log_z)
    dm = absmax(r.modes - ref.modes)
    dk = absmax(r.mode_log_z - ref.mode_log_z)
    dh = absmax(r.log_det_h - ref.log_det_h)
    assert dz <= tol_logz and dm <= tol_modes and dk <= tol_logz and dh <= max(tol_logz, 1e-9), \
        (dz, dm, dk, dh)


@pytest.mark.parametrize("name,ns,prec", [
    ("c0", None, 0), ("c0", None, 1), ("c1", 512, 0), ("c1", 512, 1), ("c2", 256, 0),
])
def test_evidence_matches_oracle(L, name, ns, prec):
    prob, cfg = synth.make_workload(name, n_starts=ns, precision=prec)
    r = L.sb_evidence(prob, cfg)
    ref = O.evidence(prob, synth.make_run_config(name, n_starts=ns, precision=0))
    _compare(r, ref, 1e-9 if prec == 0 else 1e-6)


@pytest.mark.parametrize("m,prec", [(16, 0), (32, 0), (32, 1)])
def test_evidence_long_memory(L, m, prec):
    """The whole path with L-BFGS memories beyond the register-resident 8 pairs (c1's
    mixture, 512 starts): the same mode set and log Z as the oracle run with that memory."""
    prob, cfg = synth.make_workload("c1", n_starts=512, precision=prec)
    cfg.m = m
    r = L.sb_evidence(prob, cfg)
    rc = synth.make_run_config("c1", n_starts=512, precision=0)
    rc.m = m
    ref = O.evidence(prob, rc)
    _compare(r, ref, 1e-9 if prec == 0 else 1e-6)


def _same_result(a, b):
    assert a.status == b.status == 0
    assert a.log_z == b.log_z and a.n_modes == b.n_modes
    assert np.array_equal(a.modes, b.modes) and np.array_equal(a.mode_log_z, b.mode_log_z)
    assert np.array_equal(a.log_det_h, b.log_det_h)
    assert a.n_grad_evals == b.n_grad_evals and a.iterations == b.iterations


@pytest.mark.parametrize("prec", [0, 1])
def test_exec_context_graphs(L, prec):
    """sb_evidence_exec_dev runs the L-BFGS iteration blocks as the context's HIP graphs:
    results bitwise equal to sb_evidence_dev (blocks launched directly, nothing allocated) on
    a stream and on the null stream, and to the host entry point.  A repeated call captures
    nothing; another problem on the same context captures its own block once, and the first
    problem's graph is still found afterwards."""
    p1, c1 = synth.make_workload("c1", n_starts=256, precision=prec)
    p2, c2 = synth.make_workload("c0", precision=prec)
    ex = L.ExecContext()
    stream = torch.cuda.Stream()
    r1 = L.EvidenceRunner(p1, c1, exec=ex)
    r2 = L.EvidenceRunner(p2, c2, exec=ex)
    plain = L.EvidenceRunner(p1, c1)
    with torch.cuda.stream(stream):
        a = r1.run(stream)
        s1 = ex.stats()
        b = r1.run(stream)
        s2 = ex.stats()
        c = r2.run(stream)
        s3 = ex.stats()
        e = r1.run(stream)
        s4 = ex.stats()
        f = plain.run(stream)
    torch.cuda.synchronize()
    g = plain.run()  # the null stream
    h = L.sb_evidence(p1, c1)
    assert s1["captured"] == 1 and s1["instantiated"] == 1 and s1["launched"] >= 1, s1
    assert s2["captured"] == 1 and s2["instantiated"] == 1 and s2["launched"] > s1["launched"]
    assert s3["captured"] == 2, s3
    assert s4["captured"] == 2 and s4["launched"] > s3["launched"], s4
    assert c.status == 0 and c.n_modes == 1
    for r in (b, e, f, g, h):
        _same_result(a, r)
    assert a.seconds[2] > 0 and a.seconds[7] > 0  # phase times with a context
    assert f.seconds[2] == 0 and f.seconds[7] > 0  # only the total without one
    ex.close()


def test_evidence_dev_rejects_bad_box_on_device(L):
    """The allocation-free entry point checks the box on the device."""
    prob, cfg = synth.make_workload("c0")
    prob.lo = prob.lo.copy()
    prob.lo[2] = prob.hi[2]
    r = L.EvidenceRunner(prob, cfg).run()
    assert r.status == L.E_INVAL and math.isnan(r.log_z)


@pytest.mark.parametrize("name,d", [("c0", 64), ("c1", 64)])
def test_evidence_mixed_split_paths(L, name, d):
    """Mixed precision at d = 64 (split contraction): a single Gaussian (gradient written by
    the contraction) and a mixture (two-stage bulk) against the FP64 oracle."""
    prob, cfg = synth.make_workload(name, n_starts=256, d=d, precision=1)
    r = L.sb_evidence(prob, cfg)
    ref = O.evidence(prob, synth.make_run_config(name, n_starts=256, precision=0))
    _compare(r, ref, 1e-6)


def _close_mixture(a):
    """d = 64, K = 4, means uniform in [-a, a]^64: at a = 0.8 the closest pair is only
    ~12 Mahalanobis units apart, so many bulk rows weigh several components."""
    rng = np.random.Generator(np.random.PCG64(4242))
    return synth.gaussian_mixture(rng, 64, 4, -a, a, 0.05, 1.0, 0.0, box_half=12.0,
                                  norm=synth.NORM_DENSITY, linf_min=0.5)


MIX_PATHS = {"one_stage": {"SB_MIX_TWO_STAGE": "0"},
             "two_stage": {"SB_MIX_TWO_STAGE": "1", "SB_MIX_SCREEN": "0"},
             "screened": {"SB_MIX_TWO_STAGE": "1", "SB_MIX_SCREEN": "1"}}


def _run_path(L, prob, cfg, path):
    import os

    old = {k: os.environ.get(k) for k in ("SB_MIX_TWO_STAGE", "SB_MIX_SCREEN")}
    os.environ.update(MIX_PATHS[path])
    try:
        return L.sb_evidence(prob, cfg)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("which", ["c1", "close"])
def test_mixture_bulk_paths(L, which):
    """The three mixed-precision mixture bulks (one stage over every component; two stages;
    screened by bounds carried from each row's reference point) against the FP64 oracle.
    The screen only drops components whose weight is below e^-120, so the screened bulk
    follows the one-stage bulk's trajectory (the same split Y and q) up to rounding: equal
    L-BFGS work within 2%."""
    if which == "c1":
        prob = synth.make_problem("c1")
    else:
        prob = _close_mixture(0.8)
    cfg = synth.make_run_config("c1", n_starts=256, precision=1)
    ref = O.evidence(prob, synth.make_run_config("c1", n_starts=256, precision=0))
    rs = {p: _run_path(L, prob, cfg, p) for p in MIX_PATHS}
    for p, r in rs.items():
        _compare(r, ref, 1e-6)
    e1, es = rs["one_stage"].n_grad_evals, rs["screened"].n_grad_evals
    assert abs(es - e1) <= 0.02 * e1, (e1, es, rs["two_stage"].n_grad_evals)


@pytest.mark.parametrize("d,K,seed", [(520, 3, 11), (1032, 2, 12)])
def test_screened_bulk_wide(L, d, K, seed):
    """The screened mixture bulk where the screen holds a row in registers (d = 520: three
    16-byte chunks per lane) and where it streams the row (d = 1032, beyond four chunks),
    against the one-stage bulk and the closed form of a normalised, well-separated mixture
    (log Z = -log V up to the box's truncation): every component found by both, the same
    modes, log Z within 1e-6 of the closed form, equal L-BFGS work within 2%."""
    prob = small_mixture(d, K, seed)
    cfg = synth.make_run_config("c4b", n_starts=512, precision=1)
    rs = {p: _run_path(L, prob, cfg, p) for p in ("one_stage", "screened")}
    logv = float(np.sum(np.log(prob.hi - prob.lo)))
    for p, r in rs.items():
        assert r.status == 0 and r.n_modes == K, (p, r.status, r.n_modes)
        assert abs(r.log_z + logv) <= 1e-6, (p, r.log_z, -logv)
    a = rs["one_stage"].modes[np.lexsort(rs["one_stage"].modes.T[::-1])]
    b = rs["screened"].modes[np.lexsort(rs["screened"].modes.T[::-1])]
    assert absmax(a - b) <= 1e-8
    e1, es = rs["one_stage"].n_grad_evals, rs["screened"].n_grad_evals
    assert abs(es - e1) <= 0.02 * e1, (e1, es)


@pytest.mark.parametrize("prec", [0, 1])  # 1: mixed (component lists built with atomics)
def test_evidence_device_entry_and_determinism(L, prec):
    prob, cfg = synth.make_workload("c1", n_starts=256, precision=prec)
    run = L.EvidenceRunner(prob, cfg)
    a = run.run()
    b = run.run()
    assert a.status == 0
    assert a.log_z == b.log_z and np.array_equal(a.modes, b.modes)
    h = L.sb_evidence(prob, cfg)
    assert h.log_z == a.log_z


def test_evidence_statuses(L):
    prob, cfg = synth.make_workload("c1", n_starts=128)
    cfg.max_modes = 2
    r = L.sb_evidence(prob, cfg)
    assert r.status == L.E_CAPACITY and r.n_modes == 4 and math.isnan(r.log_z)
    p0, c0 = synth.make_workload("c0")
    p0.mu = p0.mu + 25.0
    r0 = L.sb_evidence(p0, c0)
    assert r0.status == L.E_NOMODE and r0.log_z == -math.inf
    p1, c1 = synth.make_workload("c0")
    p1.prec[0] = -p1.prec[0]
    assert L.sb_evidence(p1, c1).status == L.E_NOTPD


# ------------------------------------------------------------- edge cases

def test_empty_inputs(L):
    """Empty batches are valid calls that write nothing: l + grad of 0 rows, dedup of 0
    candidates, Cholesky of 0 matrices."""
    prob = PROBLEMS["mix_d37_K3"]()
    m = L.DeviceModel(prob)
    l, g = L.sb_logl_grad_dev(m, torch.empty((0, prob.d), dtype=torch.float64, device="cuda"))
    assert l.numel() == 0 and g.shape == (0, prob.d)
    rep_of, reps = L.sb_dedup_dev(torch.empty((0, 3), dtype=torch.float64, device="cuda"),
                                  torch.empty(0, dtype=torch.float64, device="cuda"), 0.1)
    assert rep_of.numel() == 0 and reps.numel() == 0
    Lf, ld, info = L.sb_cholesky_logdet_dev(torch.empty((0, 5, 5), dtype=torch.float64,
                                                        device="cuda"))
    assert ld.numel() == 0


def test_logl_grad_largest_supported_dimension(L):
    """d = 4096 (the largest the L-BFGS step supports) with a ragged batch: l and grad
    against the oracle."""
    rng = np.random.Generator(np.random.PCG64(4096))
    d = 4096
    # dense SPD precision, cheap to build at this size: diagonal plus two rank-one terms
    lam = np.exp(rng.uniform(np.log(0.1), 0.0, d))
    u, v = rng.standard_normal(d) / 64.0, rng.standard_normal(d) / 64.0
    P = np.diag(1.0 / lam) + np.outer(u, u) + np.outer(v, v)
    mu = rng.uniform(-1, 1, (1, d))
    prob = synth.Problem(synth.FAMILY_GAUSS_MIX, synth.NORM_PEAK_ZERO, d, 1, np.zeros(1), mu,
                         P[None], 0.0, 0.0, np.full(d, -5.0), np.full(d, 5.0), np.zeros(1))
    X = mu + 0.5 * rng.standard_normal((3, d))
    lo, go = O.logl(prob, X)
    l, g = L.sb_logl_grad_dev(L.DeviceModel(prob), dev(X))
    assert rel(l.cpu().numpy(), lo) < 1e-10
    assert rel(g.cpu().numpy(), go, axis=1) < 1e-10
