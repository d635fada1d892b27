"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a closed form,
a library routine computing the same quantity by another method, brute-force
quadrature, a textbook identity, or an invariant of the evidence.
"""
import math
import os

import numpy as np
import pytest
import scipy.special as sps
import scipy.stats as st

from paper_2601_19957_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LOG2PI = math.log(2.0 * math.pi)


def small_mixture(d=6, K=3, seed=5, sep=12.0, box=12.0, norm=synth.NORM_DENSITY):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.gaussian_mixture(rng, d, K, -8.0, 8.0, 0.05, 1.0, sep, box_half=box, norm=norm)


def small_t(d=6, nu=5.0, seed=9, box=20.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.student_t(rng, d, nu, -5.0, 5.0, 0.05, 1.0, box)


# ------------------------------------------------------------------ RNG

def test_philox_known_answers(oracle_lib):
    O = oracle_lib
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox4x32_10(v[:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_uniform_range_and_moments(oracle_lib):
    O = oracle_lib
    u = np.array([O.rng_uniform(77, 0, r, s, i) for r in range(64) for s in range(2)
                  for i in range(32)])
    assert np.all(u >= 0.0) and np.all(u < 1.0)
    assert abs(u.mean() - 0.5) < 0.03
    assert abs(u.var() - 1.0 / 12.0) < 0.01
    # uniform index i and the words of block i//2 are the same Philox output
    w = O.philox4x32_10([5, 3, 1, 0], [77, 0])
    a, b = int(w[2]), int(w[3])
    expect = ((a >> 5) * 67108864.0 + (b >> 6)) / 9007199254740992.0
    assert O.rng_uniform(77, 0, 5, 1, 7) == expect


# ------------------------------------------------------------------ rays

def test_ray_geometries(oracle_lib):
    O = oracle_lib
    d = 7
    lo = np.linspace(-3.0, -1.0, d)
    hi = np.linspace(2.0, 5.0, d)
    P0, P1 = O.rays(d, lo, hi, 400, 2024)
    c = 0.5 * (lo + hi)
    on = lambda x: np.isclose(x, lo) | np.isclose(x, hi)
    for r in range(400):
        p, q = P0[r], P1[r]
        g = r % 4
        if g == 0:  # vertex to vertex
            assert on(p).all() and on(q).all()
        elif g == 1:  # vertex to the midpoint of an edge
            assert on(p).all()
            mid = np.isclose(q, c)
            assert mid.sum() == 1 and (on(q) | mid).all()
        elif g == 2:  # wall to wall along one axis
            ax = np.flatnonzero(np.isclose(p, lo) & np.isclose(q, hi))
            assert ax.size >= 1
            assert np.all((p >= lo) & (p <= hi) & (q >= lo) & (q <= hi))
        else:  # sunburst: from the centre to the boundary
            assert np.allclose(p, c)
            assert np.all(q >= lo - 1e-12) and np.all(q <= hi + 1e-12)
            assert (np.isclose(q, lo, atol=1e-12) | np.isclose(q, hi, atol=1e-12)).any()
    # sunburst directions are isotropic: the mean direction is near 0
    dirs = P1[3::4] - P0[3::4]
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    assert np.linalg.norm(dirs.mean(0)) < 0.25


def test_discovery_orders_and_argmax(oracle_lib):
    O = oracle_lib
    prob, cfg = synth.make_workload("c0")
    res = O.discover(prob, cfg.n_rays, cfg.n_points, cfg.n_starts, cfg.seed)
    bl, sr = res["ray_best_l"], res["start_ray"]
    # starts are the rays with the largest maxima, in descending order
    assert np.all(np.diff(bl[sr]) <= 0)
    assert bl[sr].min() >= np.sort(bl)[-cfg.n_starts]
    # each start is the best sample of its ray: no sample of the ray is higher
    P0, P1 = O.rays(prob.d, prob.lo, prob.hi, cfg.n_rays, cfg.seed)
    t = (np.arange(cfg.n_points) + 0.5) / cfg.n_points
    for s in range(0, cfg.n_starts, 7):
        r = sr[s]
        pts = P0[r] + t[:, None] * (P1[r] - P0[r])
        # independent evaluation of the peak-zero Gaussian: -1/2 (x-mu)^T P (x-mu)
        dl = pts - prob.mu[0]
        lv = -0.5 * np.einsum("ij,jk,ik->i", dl, prob.prec[0], dl)
        assert np.argmax(lv) == res["ray_best_j"][r]
        assert np.allclose(res["X0"][s], pts[res["ray_best_j"][r]])


# ------------------------------------------------------- family functions

def test_logl_matches_scipy_mixture(oracle_lib):
    O = oracle_lib
    prob = small_mixture()
    X = synth.random_points(prob, 50, 1, spread=0.8)
    l, _ = O.logl(prob, X)
    comp = np.stack([st.multivariate_normal(prob.mu[k], np.linalg.inv(prob.prec[k])).logpdf(X)
                     for k in range(prob.K)], axis=1)
    ref = sps.logsumexp(comp + prob.log_w[None, :], axis=1)
    assert np.max(np.abs(l - ref)) < 1e-9 * max(1.0, np.abs(ref).max())


def test_logl_matches_scipy_student_t(oracle_lib):
    O = oracle_lib
    prob = small_t()
    X = synth.random_points(prob, 40, 2, spread=0.5)
    l, _ = O.logl(prob, X)
    ref = st.multivariate_t(prob.mu[0], np.linalg.inv(prob.prec[0]), df=prob.nu).logpdf(X)
    assert np.max(np.abs(l - ref)) < 1e-10 * max(1.0, np.abs(ref).max())


def test_peak_zero_gaussian_and_offset(oracle_lib):
    O = oracle_lib
    prob = small_mixture(K=1, norm=synth.NORM_PEAK_ZERO)
    prob.logl_offset = 2.5
    l, g = O.logl(prob, prob.mu)
    assert l[0] == 2.5 and np.all(g == 0.0)


@pytest.mark.parametrize("fam", ["mix", "t"])
def test_gradient_central_differences(oracle_lib, fam):
    O = oracle_lib
    prob = small_mixture(d=8, K=3) if fam == "mix" else small_t(d=8)
    X = synth.points_near_modes(prob, 6, 3, scale=0.7)
    _, G = O.logl(prob, X)
    h = 1e-6
    for b in range(X.shape[0]):
        fd = np.zeros(prob.d)
        for i in range(prob.d):
            e = np.zeros(prob.d)
            e[i] = h
            fd[i] = (O.logl(prob, X[b] + e, grad=False)[0] - O.logl(prob, X[b] - e, grad=False)[0]) / (2 * h)
        assert np.max(np.abs(fd - G[b])) <= 1e-6 * max(1.0, np.abs(G[b]).max())


@pytest.mark.parametrize("fam", ["mix", "t"])
def test_hessian_and_hvp_against_gradient_differences(oracle_lib, fam):
    O = oracle_lib
    prob = small_mixture(d=6, K=3) if fam == "mix" else small_t(d=6)
    x = synth.points_near_modes(prob, 1, 4, scale=0.5)[0]
    H = O.neg_hessian(prob, x)
    h = 1e-5
    fd = np.zeros((prob.d, prob.d))
    for j in range(prob.d):
        e = np.zeros(prob.d)
        e[j] = h
        gp = O.logl(prob, x + e)[1][0]
        gm = O.logl(prob, x - e)[1][0]
        fd[:, j] = -(gp - gm) / (2 * h)
    assert np.linalg.norm(H - fd) <= 1e-6 * np.linalg.norm(H)
    V = np.random.default_rng(1).standard_normal((3, prob.d))
    HV = O.hvp(prob, np.repeat(x[None], 3, 0), V)
    assert np.allclose(HV, -(V @ fd.T), rtol=1e-5, atol=1e-6 * np.abs(H).max())


def test_student_t_hessian_at_mode_closed_form(oracle_lib):
    O = oracle_lib
    prob = small_t(d=5, nu=7.0)
    H = O.neg_hessian(prob, prob.mu[0])
    assert np.allclose(H, (prob.nu + prob.d) / prob.nu * prob.prec[0], rtol=1e-13, atol=0)


# ---------------------------------------------------------- linear algebra

def test_cholesky_logdet_against_numpy(oracle_lib):
    O = oracle_lib
    for d in (1, 3, 17, 64):
        A = synth.random_spd(d, 100 + d, cond=1e3)[0]
        stt, L = O.cholesky(A)
        assert stt == 0
        assert np.allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
        ld = O.logdet_spd(A)
        assert abs(ld - np.linalg.slogdet(A)[1]) <= 1e-12 * max(1, abs(ld)) + 1e-12
        assert abs(ld - np.sum(np.log(np.linalg.eigvalsh(A)))) <= 1e-11 * max(1, abs(ld))
        b = np.arange(d, dtype=float) + 1
        assert np.allclose(O.chol_solve(L, b), np.linalg.solve(A, b), rtol=1e-10)


def test_cholesky_rejects_indefinite(oracle_lib):
    O = oracle_lib
    A = np.diag([2.0, 1.0, -1.0, 3.0])
    stt, _ = O.cholesky(A)
    assert stt == 3  # third pivot fails


# ------------------------------------------------------------ reductions

def test_pairwise_sum_and_logsumexp(oracle_lib):
    O = oracle_lib
    x = np.random.default_rng(3).standard_normal(1001) * 1e3
    assert abs(O.pairwise_sum(x) - math.fsum(x)) < 1e-9
    assert O.pairwise_sum(np.array([])) == 0.0
    v = np.array([-1.0, 2.0, 0.5, -np.inf])
    assert abs(O.logsumexp(v) - sps.logsumexp(v)) < 1e-15
    assert O.logsumexp(np.array([-np.inf, -np.inf])) == -np.inf
    assert O.logsumexp(np.array([])) == -np.inf
    assert abs(O.logsumexp(np.array([5.0, 5.0, 5.0])) - (5.0 + math.log(3))) < 1e-15
    assert O.logsumexp(np.array([0.0, -2000.0])) == 0.0
    assert abs(O.logsumexp(np.array([1e4, 1e4 - 1.0])) - (1e4 + math.log1p(math.exp(-1)))) < 1e-11


# --------------------------------------------------------------- L-BFGS

def dense_lbfgs_direction(S, Y, g):
    """-H g with H from the BFGS inverse update applied to H0 = gamma I, oldest pair first
    (Nocedal & Wright, Numerical Optimization, eq. 6.17 / 7.19)."""
    d = g.size
    s, y = S[-1], Y[-1]
    H = (s @ y) / (y @ y) * np.eye(d)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        V = np.eye(d) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return -H @ g


def test_two_loop_equals_dense_bfgs_matrix(oracle_lib):
    O = oracle_lib
    for cnt in (1, 3, 8):
        S, Y, G = synth.lbfgs_history(9, 8, cnt, seed=40 + cnt)
        p = O.two_loop(S[0, :cnt], Y[0, :cnt], G[0])
        ref = dense_lbfgs_direction(S[0, :cnt], Y[0, :cnt], G[0])
        assert np.allclose(p, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_two_loop_secant_equation(oracle_lib):
    O = oracle_lib
    S, Y, _ = synth.lbfgs_history(12, 8, 5, seed=3)
    p = O.two_loop(S[0, :5], Y[0, :5], Y[0, 4])
    assert np.allclose(p, -S[0, 4], rtol=1e-12, atol=1e-13)


def test_two_loop_quadratic_termination(oracle_lib):
    """With memory >= d and exact line searches, L-BFGS on a strictly convex
    quadratic reaches the minimiser within d steps (conjugate directions)."""
    O = oracle_lib
    d = 6
    A = synth.random_spd(d, 11, cond=30.0)[0]
    b = np.arange(1.0, d + 1.0)
    x = np.zeros(d)
    S, Y = [], []
    g = A @ x - b
    for it in range(d):
        p = -g if not S else O.two_loop(np.array(S), np.array(Y), g)
        a = -(g @ p) / (p @ A @ p)
        xn = x + a * p
        gn = A @ xn - b
        S.append(xn - x)
        Y.append(gn - g)
        x, g = xn, gn
    assert np.linalg.norm(g) <= 1e-10 * np.linalg.norm(b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10)


def test_lbfgs_reaches_gaussian_mode(oracle_lib):
    O = oracle_lib
    prob = small_mixture(d=10, K=1, norm=synth.NORM_PEAK_ZERO)
    r = O.lbfgs(prob, prob.mu[0] + 3.0, m=8, grad_tol=1e-10)
    assert r["status"] == O.ST_CONVERGED
    assert np.max(np.abs(r["x"] - prob.mu[0])) < 1e-8
    assert np.max(np.abs(r["grad"])) <= 1e-10


def test_newton_single_step_exact_for_gaussian(oracle_lib):
    O = oracle_lib
    prob = small_mixture(d=9, K=1, norm=synth.NORM_PEAK_ZERO)
    st_, x, steps = O.newton(prob, prob.mu[0] + np.linspace(-4, 4, 9), max_steps=1)
    assert st_ == 0 and steps == 1
    assert np.max(np.abs(x - prob.mu[0])) < 1e-12


# ---------------------------------------------------------------- dedup

def check_leader_clustering(X, l, tau, rep_of, reps):
    """Properties that characterise the greedy leader clustering uniquely."""
    order = sorted(range(len(l)), key=lambda i: (-l[i], i))
    pos = {c: t for t, c in enumerate(order)}
    dist = lambda a, b: np.max(np.abs(X[a] - X[b]))
    # representatives appear in visiting order, each founded by itself
    assert list(reps) == sorted(reps, key=lambda c: pos[c])
    for r in reps:
        assert rep_of[r] == r
    for c in range(len(l)):
        r = rep_of[c]
        # c joined the first representative (in creation order) that is within tau
        # and was created before c was visited
        earlier = [q for q in reps if pos[q] < pos[c] or q == c]
        within = [q for q in earlier if q != c and dist(c, q) <= tau]
        if r == c:
            assert not within
        else:
            assert within and within[0] == r


def test_dedup_handmade(oracle_lib):
    O = oracle_lib
    X = np.array([[0.0, 0.0], [0.05, 0.0], [1.0, 1.0], [1.02, 0.99], [0.0, 0.09], [5.0, 5.0]])
    l = np.array([1.0, 3.0, 2.0, 2.0, 0.5, -1.0])
    rep_of, reps = O.dedup(X, l, 0.1)
    # l order: 1 (3.0), 2 (2.0), 3 (2.0), 0 (1.0), 4 (0.5), 5 (-1)
    assert list(reps) == [1, 2, 5]
    # point 4 is within 0.1 of point 1 in L-infinity (|0.05| in x, |0.09| in y)
    assert list(rep_of) == [1, 1, 2, 2, 1, 5]
    check_leader_clustering(X, l, 0.1, rep_of, reps)


def test_dedup_random_sets_properties(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(8)
    for trial in range(20):
        X = rng.uniform(0, 1, (40, 3))
        l = np.round(rng.standard_normal(40), 1)  # many ties
        rep_of, reps = O.dedup(X, l, 0.25)
        check_leader_clustering(X, l, 0.25, rep_of, reps)


def test_dedup_excludes_invalid(oracle_lib):
    O = oracle_lib
    X = np.zeros((3, 2))
    rep_of, reps = O.dedup(X, np.array([1.0, 2.0, 3.0]), 0.1, valid=[1, 1, 0])
    assert list(reps) == [1] and list(rep_of) == [1, 1, -1]


# ------------------------------------------------------ evidence closed forms

def gaussian_closed_form(prob):
    """Peak-zero Gaussian: integral of exp(l) over R^d = (2 pi)^(d/2) det(Sigma)^(1/2)."""
    d = prob.d
    return 0.5 * d * LOG2PI + 0.5 * prob.sum_log_lambda[0] - float(np.sum(np.log(prob.hi - prob.lo)))


def test_c0_closed_form(oracle_lib):
    O = oracle_lib
    prob, cfg = synth.make_workload("c0")
    r = O.evidence(prob, cfg)
    assert r.status == 0 and r.n_modes == 1
    assert abs(r.log_z - gaussian_closed_form(prob)) < 1e-10
    assert np.max(np.abs(r.modes[0] - prob.mu[0])) < 1e-8
    assert abs(r.log_det_h[0] + prob.sum_log_lambda[0]) < 1e-10


def test_c1_mixture_closed_form(oracle_lib):
    O = oracle_lib
    prob, cfg = synth.make_workload("c1", n_starts=128)
    r = O.evidence(prob, cfg)
    logv = 64 * math.log(24.0)
    assert r.status == 0 and r.n_modes == 4
    assert abs(r.log_z + logv) < 1e-9
    # each mode: log Z_k = log w_k - log V, log det H_k = log det P_k = -sum log lambda_k
    order = [int(np.argmin(np.abs(prob.mu - m).max(1))) for m in r.modes]
    assert sorted(order) == [0, 1, 2, 3]
    for i, k in enumerate(order):
        assert np.max(np.abs(r.modes[i] - prob.mu[k])) < 1e-8
        assert abs(r.mode_log_z[i] - (prob.log_w[k] - logv)) < 1e-9
        assert abs(r.log_det_h[i] + prob.sum_log_lambda[k]) < 1e-9


def test_c2_student_t_laplace_closed_form(oracle_lib):
    O = oracle_lib
    prob, cfg = synth.make_workload("c2", n_starts=16)
    r = O.evidence(prob, cfg)
    nu, d = 30.0, 256
    expect = (math.lgamma(143) - math.lgamma(15) + 128 * math.log(2.0 / 286.0) - 256 * math.log(40.0))
    assert r.status == 0 and r.n_modes == 1
    assert abs(r.log_z - expect) < 1e-9
    assert abs(expect - (-1039.663593014300)) < 1e-9


def test_c4a_closed_form_reduced_dimension(oracle_lib):
    O = oracle_lib
    prob, cfg = synth.make_workload("c4a", d=128, n_starts=8)
    r = O.evidence(prob, cfg)
    assert r.status == 0 and r.n_modes == 1
    assert abs(r.log_z - gaussian_closed_form(prob)) < 1e-9


def test_student_t_laplace_gap_matches_paper(oracle_lib):
    """The Laplace gap of a normalised Student-t (box truncation aside) against the
    errors the paper prints for nu = 3 (35% at 2D, a factor 10^12 at 64D)."""
    O = oracle_lib
    rows = [l.split() for l in open(os.path.join(GOLDEN, "student_t_laplace_error.txt"))
            if l.strip() and not l.startswith("#")]
    for nu_s, d_s, err_s, kind in rows:
        nu, d, err = float(nu_s), int(d_s), float(err_s)
        rng = np.random.Generator(np.random.PCG64(d))
        prob = synth.student_t(rng, d, nu, -1.0, 1.0, 0.5, 1.0, 50.0)
        cfg = synth.RunConfig(n_rays=32, n_points=16, n_starts=8, seed=1)
        r = O.evidence(prob, cfg)
        gap = r.log_z + float(np.sum(np.log(prob.hi - prob.lo)))  # log(Z_L / Z_true)
        if kind == "rel":
            assert 0.5 * err < abs(math.exp(gap) - 1.0) < 1.5 * err
        else:
            assert math.log10(err) <= -gap / math.log(10) < math.log10(err) + 1


def test_quadrature_d1_exact_erf(oracle_lib):
    O = oracle_lib
    prob = synth.Problem(0, synth.NORM_PEAK_ZERO, 1, 1, np.zeros(1), np.array([[0.7]]),
                         np.array([[4.0]]), 0.0, 0.0, np.array([-5.0]), np.array([6.0]),
                         np.array([math.log(0.25)]))
    cfg = synth.RunConfig(n_rays=8, n_points=16, n_starts=4, seed=3)
    r = O.evidence(prob, cfg)
    s = 1.0 / math.sqrt(4.0)
    mass = math.sqrt(2 * math.pi) * s * 0.5 * (math.erf((6.0 - 0.7) / (s * math.sqrt(2)))
                                               - math.erf((-5.0 - 0.7) / (s * math.sqrt(2))))
    assert abs(r.log_z - (math.log(mass) - math.log(11.0))) < 1e-10


def test_quadrature_d2_mixture(oracle_lib):
    O = oracle_lib
    rng = np.random.Generator(np.random.PCG64(21))
    prob = synth.gaussian_mixture(rng, 2, 2, -4.0, 4.0, 0.1, 0.4, 12.0, box_half=10.0,
                                  norm=synth.NORM_DENSITY, linf_min=1.0)
    cfg = synth.RunConfig(n_rays=64, n_points=32, n_starts=32, seed=5)
    r = O.evidence(prob, cfg)
    assert r.n_modes == 2
    # composite Gauss-Legendre (400 panels x 8 nodes per axis) of the mixture density
    xg, wg = np.polynomial.legendre.leggauss(8)
    edges = np.linspace(-10, 10, 401)
    a, b = edges[:-1, None], edges[1:, None]
    nodes = (0.5 * (b - a) * xg[None] + 0.5 * (a + b)).ravel()
    weights = (0.5 * (b - a) * wg[None]).ravel()
    XX, YY = np.meshgrid(nodes, nodes, indexing="ij")
    pts = np.stack([XX.ravel(), YY.ravel()], 1)
    dens = sum(math.exp(prob.log_w[k]) *
               st.multivariate_normal(prob.mu[k], np.linalg.inv(prob.prec[k])).pdf(pts)
               for k in range(2))
    integral = float(np.sum(dens * np.outer(weights, weights).ravel()))
    truth = math.log(integral) - math.log(400.0)
    assert abs(r.log_z - truth) < 1e-10


# --------------------------------------------------------------- invariants

def _run(O, prob, cfg):
    r = O.evidence(prob, cfg)
    assert r.status == 0
    return r


def test_invariant_offset_and_permutation(oracle_lib):
    O = oracle_lib
    prob = small_mixture(d=5, K=3, seed=13)
    cfg = synth.RunConfig(n_rays=96, n_points=32, n_starts=96, seed=7)
    base = _run(O, prob, cfg)
    assert base.n_modes == 3
    p2 = prob.copy()
    p2.logl_offset = 4.25
    r2 = _run(O, p2, cfg)
    assert abs(r2.log_z - (base.log_z + 4.25)) < 1e-10
    assert np.allclose(r2.modes, base.modes, atol=1e-10)
    perm = [2, 0, 1]
    p3 = prob.copy()
    p3.log_w, p3.mu, p3.prec = prob.log_w[perm], prob.mu[perm], prob.prec[perm]
    r3 = _run(O, p3, cfg)
    assert abs(r3.log_z - base.log_z) < 1e-10
    assert np.allclose(r3.modes, base.modes, atol=1e-9)


def test_invariant_translation_scaling_box(oracle_lib):
    O = oracle_lib
    prob = small_mixture(d=4, K=2, seed=17)
    cfg = synth.RunConfig(n_rays=64, n_points=32, n_starts=64, seed=9)
    base = _run(O, prob, cfg)
    t = np.array([1.5, -2.0, 0.25, 3.0])
    pt = prob.copy()
    pt.mu, pt.lo, pt.hi = prob.mu + t, prob.lo + t, prob.hi + t
    rt = _run(O, pt, cfg)
    assert abs(rt.log_z - base.log_z) < 1e-10
    assert np.allclose(rt.modes, base.modes + t, atol=1e-9)
    s = 2.0
    ps = prob.copy()
    ps.mu, ps.lo, ps.hi, ps.prec = prob.mu * s, prob.lo * s, prob.hi * s, prob.prec / s ** 2
    rs = _run(O, ps, cfg)
    assert abs(rs.log_z - (base.log_z - prob.d * math.log(s))) < 1e-10
    pb = prob.copy()
    pb.hi = prob.hi + 3.0
    rb = _run(O, pb, cfg)
    dv = float(np.sum(np.log(pb.hi - pb.lo)) - np.sum(np.log(prob.hi - prob.lo)))
    assert abs(rb.log_z - (base.log_z - dv)) < 1e-10


def test_modes_equal_reference_set(oracle_lib):
    O = oracle_lib
    prob, cfg = synth.make_workload("c1", n_starts=64)
    r = O.evidence(prob, cfg)
    ref = O.reference_modes(prob)
    assert ref.n_modes == r.n_modes == 4
    assert np.max(np.abs(ref.modes - r.modes)) < 1e-8
    assert abs(ref.log_z - r.log_z) < 1e-9


# ------------------------------------------------------------- status codes

def test_status_capacity_and_nomode(oracle_lib):
    O = oracle_lib
    prob, cfg = synth.make_workload("c1", n_starts=64)
    cfg.max_modes = 2
    r = O.evidence(prob, cfg)
    assert r.status == O.E_CAPACITY and r.n_modes == 4 and math.isnan(r.log_z)
    p0, c0 = synth.make_workload("c0")
    p0.mu = p0.mu + 25.0  # mode outside the box: rejected by the inside-box filter
    r0 = O.evidence(p0, c0)
    assert r0.status == O.E_NOMODE and r0.log_z == -math.inf


def test_validation(oracle_lib):
    O = oracle_lib
    prob, cfg = synth.make_workload("c0")

    def status(mod):
        p = prob.copy()
        c = synth.RunConfig(**vars(cfg))
        mod(p, c)
        return O.evidence(p, c).status

    assert status(lambda p, c: None) == 0
    assert status(lambda p, c: setattr(c, "m", 0)) == O.E_INVAL
    assert status(lambda p, c: setattr(c, "m", 33)) == O.E_INVAL
    assert status(lambda p, c: setattr(c, "max_modes", 0)) == O.E_INVAL
    assert status(lambda p, c: setattr(c, "n_starts", c.n_rays + 1)) == O.E_INVAL
    assert status(lambda p, c: p.lo.__setitem__(0, 20.0)) == O.E_INVAL
    assert status(lambda p, c: p.hi.__setitem__(1, np.inf)) == O.E_INVAL
    assert status(lambda p, c: p.mu.__setitem__((0, 0), np.nan)) == O.E_INVAL

    def asym(p, c):
        p.prec[0, 0, 1] += 1e-3

    assert status(asym) == O.E_NOTPD

    def indef(p, c):
        p.prec[0] = -p.prec[0]

    assert status(indef) == O.E_NOTPD
    t = small_t(d=4)
    t2 = t.copy()
    t2.nu = 0.0
    c = synth.RunConfig(n_rays=8, n_points=4, n_starts=4)
    assert O.evidence(t2, c).status == O.E_INVAL
    t3 = t.copy()
    t3.K = 2
    t3.mu = np.concatenate([t.mu, t.mu])
    t3.prec = np.concatenate([t.prec, t.prec])
    t3.log_w = np.zeros(2)
    assert O.evidence(t3, c).status == O.E_UNSUPPORTED


# ------------------------------------------------------------ preprocessing

def probe_points(lo, hi):
    """The 2d + 1 probe points of the preprocessing: centre, then + and - half-width per axis."""
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
    X = [c.copy()]
    for i in range(c.size):
        for sgn in (1.0, -1.0):
            x = c.copy()
            x[i] = c[i] + sgn * h[i]
            X.append(x)
    return np.array(X)


def test_precheck_gaussian_sensitivity_closed_form(oracle_lib):
    """For a Gaussian l = const - (x - mu)^T P (x - mu) / 2 the probe differences are
    l(c +- D e_i) - l(c) = -(+-D g_i + D^2 P_ii / 2), g = P (c - mu): s_i in closed form."""
    O = oracle_lib
    for norm, seed in ((synth.NORM_PEAK_ZERO, 3), (synth.NORM_DENSITY, 4)):
        rng = np.random.Generator(np.random.PCG64(seed))
        prob = synth.gaussian_mixture(rng, 9, 1, -4.0, 4.0, 0.1, 1.0, 0.0, box_half=7.0,
                                      norm=norm)
        r = O.precheck(prob)
        assert r["status"] == 0
        P, mu = prob.prec[0], prob.mu[0]
        c, D = 0.5 * (prob.lo + prob.hi), 0.5 * (prob.hi - prob.lo)
        g = P @ (c - mu)
        ref = np.abs(D * g + 0.5 * D ** 2 * np.diag(P)) + np.abs(-D * g + 0.5 * D ** 2 * np.diag(P))
        assert np.allclose(r["s"], ref, rtol=1e-11, atol=0)


def test_precheck_sensitivity_against_scipy(oracle_lib):
    """s from library log-densities at the 2d + 1 probe points (mixture and Student-t)."""
    O = oracle_lib
    for prob in (small_mixture(d=5, K=3, seed=21), small_t(d=6, nu=4.0, seed=22)):
        X = probe_points(prob.lo, prob.hi)
        if prob.family == synth.FAMILY_STUDENT_T:
            cov = np.linalg.inv(prob.prec[0])
            l = st.multivariate_t(prob.mu[0], cov, df=prob.nu).logpdf(X)
        else:
            comp = [lw + st.multivariate_normal(m, np.linalg.inv(P)).logpdf(X)
                    for lw, m, P in zip(prob.log_w, prob.mu, prob.prec)]
            l = sps.logsumexp(np.array(comp), axis=0)
        ref = np.abs(l[1::2] - l[0]) + np.abs(l[2::2] - l[0])
        r = O.precheck(prob)
        assert np.allclose(r["s"], ref, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("d,n_flat,n_soft", [(12, 2, 3), (13, 1, 1), (40, 5, 4)])
def test_precheck_classes_and_marginal_closed_form(oracle_lib, d, n_flat, n_soft):
    """Centred Gaussian with unconstrained and weakly constrained coordinates: s_i = D^2 P_ii,
    so the classes are the constructed ones and the soft width estimate D / sqrt(s_i) is exactly
    1 / sqrt(P_ii); the marginal is sum_flat log(b - a) + sum_soft (log 2 pi / 2 + log sigma_i).
    The classes also follow numpy's median and maximum of the same s."""
    O = oracle_lib
    prob = synth.nuisance_gaussian(d, n_flat, n_soft, seed=30 + d)
    r = O.precheck(prob)
    assert r["status"] == 0
    D = 0.5 * (prob.hi - prob.lo)
    Pd = np.diag(prob.prec[0])
    assert np.allclose(r["s"], D ** 2 * Pd, rtol=1e-12)
    want = np.zeros(d, dtype=np.int32)
    want[:n_flat] = 1
    want[n_flat:n_flat + n_soft] = 2
    assert np.array_equal(r["cls"], want)
    s = r["s"]
    by_np = np.where(s < 1e-6 * np.median(s), 1, np.where(s < 1e-3 * np.max(s), 2, 0))
    assert np.array_equal(r["cls"], by_np)
    sig = 1.0 / np.sqrt(Pd)
    ref = float(np.sum(np.log(2.0 * D[:n_flat])) +
                np.sum(0.5 * LOG2PI + np.log(sig[n_flat:n_flat + n_soft])))
    assert abs(r["logz_marginal"] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_precheck_flat_term_is_the_prior_range_integral(oracle_lib):
    """A coordinate the likelihood does not constrain contributes the integral of its (constant)
    likelihood factor over the prior range: for a Gaussian factor of width 1e6 D the exact
    truncated integral sigma sqrt(2 pi) erf(D / (sigma sqrt 2)) equals b - a to 1e-12, which
    fixes the flat term as log(b - a) (the half-width D would be off by log 2)."""
    O = oracle_lib
    prob = synth.nuisance_gaussian(8, 1, 0, seed=41)
    r = O.precheck(prob)
    D = 0.5 * (prob.hi[0] - prob.lo[0])
    sig = 1.0 / math.sqrt(prob.prec[0][0, 0])
    exact = math.log(sig * math.sqrt(2 * math.pi) * math.erf(D / (sig * math.sqrt(2.0))))
    assert r["cls"][0] == 1 and abs(r["logz_marginal"] - exact) < 1e-11


def test_precheck_invariants_and_validation(oracle_lib):
    """A constant added to l changes nothing; scaling P by c scales s by c (classes kept);
    a median of an even count is the mean of the middle two; a bad box is rejected."""
    O = oracle_lib
    prob = synth.nuisance_gaussian(10, 2, 2, seed=50, centred=False)
    r = O.precheck(prob)
    p2 = synth.Problem(**{**vars(prob), "logl_offset": 123.25})
    r2 = O.precheck(p2)
    assert np.allclose(r2["s"], r["s"], rtol=1e-9, atol=1e-9)
    assert np.array_equal(r2["cls"], r["cls"])
    p3 = synth.Problem(**{**vars(prob), "prec": 4.0 * prob.prec})
    r3 = O.precheck(p3)
    assert np.allclose(r3["s"], 4.0 * r["s"], rtol=1e-11)
    assert np.array_equal(r3["cls"], r["cls"])
    # even d = 4 with s = D^2 P_ii = [1.2e-6, 1, 2, 3]: the mean median 1.5 flags the first
    # coordinate (1.2e-6 < 1.5e-6), the lower middle value 1 would not
    P = np.diag([1.2e-6, 1.0, 2.0, 3.0])[None]
    p4 = synth.Problem(synth.FAMILY_GAUSS_MIX, synth.NORM_PEAK_ZERO, 4, 1, np.zeros(1),
                       np.zeros((1, 4)), P, 0.0, 0.0, -np.ones(4), np.ones(4), np.zeros(1))
    r4 = O.precheck(p4)
    assert list(r4["cls"]) == [1, 0, 0, 0]
    p5 = synth.Problem(**{**vars(p4), "lo": np.array([-1.0, 1.0, -1.0, -1.0])})
    assert O.precheck(p5)["status"] == -1


# ------------------------------------------------- reduction at the modes

def constructed_spectrum(n, seed, lam):
    q = synth.haar_orthogonal(np.random.Generator(np.random.PCG64(seed)), n)
    return (q * lam[None, :]) @ q.T, q


def test_eig_reduce_constructed_spectrum(oracle_lib):
    """H = Q diag(lam) Q^T with known lam spread over the three classes: eigenvalues, classes,
    d_eff, nuisance terms 1/2 log(2 pi / lam) and degenerate extents sum_j |Q_ji| (b_j - a_j)
    in closed form from (lam, Q)."""
    O = oracle_lib
    n = 24
    lam = np.concatenate([np.geomspace(50.0, 2.0, 10), np.geomspace(0.5, 0.02, 8),
                          np.geomspace(1e-5, 1e-8, 6)])
    H, q = constructed_spectrum(n, 71, lam)
    lo, hi = -np.linspace(1.0, 3.0, n), np.linspace(2.0, 5.0, n)
    r = O.eig_reduce(H, lo, hi, eps_inform=1.0, eps_nuisance=1e-3)
    assert np.allclose(r["eigval"], lam, rtol=1e-9, atol=1e-13 * lam[0])
    want = np.array([0] * 10 + [1] * 8 + [2] * 6)
    assert np.array_equal(r["cls"], want) and r["d_eff"] == 10
    ext = np.abs(q).T @ (hi - lo)
    ref = float(np.sum(0.5 * np.log(2 * np.pi / lam[10:18])) + np.sum(np.log(ext[18:])))
    assert abs(r["logz_marginal"] - ref) <= 1e-9 * abs(ref)
    # eigenvectors: each column equals the constructed one up to sign (distinct eigenvalues)
    dots = np.abs(np.sum(r["V"] * q, axis=0))
    assert np.all(np.abs(dots[:18] - 1.0) < 1e-8)


def test_eig_reduce_axis_aligned_and_invariants(oracle_lib):
    """A diagonal H: the degenerate term of coordinate i is log(b_i - a_i), the flat term of the
    preprocessing probe; a symmetric permutation of H and the box changes nothing."""
    O = oracle_lib
    lam = np.array([3.0, 1e-9, 0.2, 7.0, 1e-10, 0.05])
    lo, hi = -np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0]), np.array([2.0, 2.0, 1.0, 1.0, 3.0, 9.0])
    r = O.eig_reduce(np.diag(lam), lo, hi, eps_inform=1.0, eps_nuisance=1e-6)
    ref = (np.log(hi[1] - lo[1]) + np.log(hi[4] - lo[4]) +
           0.5 * np.log(2 * np.pi / 0.2) + 0.5 * np.log(2 * np.pi / 0.05))
    assert abs(r["logz_marginal"] - ref) < 1e-13 and r["d_eff"] == 2
    perm = np.array([4, 0, 5, 2, 1, 3])
    r2 = O.eig_reduce(np.diag(lam)[perm][:, perm], lo[perm], hi[perm], 1.0, 1e-6)
    assert np.allclose(r2["eigval"], r["eigval"], rtol=1e-15)
    assert abs(r2["logz_marginal"] - r["logz_marginal"]) < 1e-13


def _gauss_from_spectrum(mu, P, box=20.0):
    d = mu.size
    P = 0.5 * (P + P.T)
    lam = np.linalg.eigvalsh(P)
    return synth.Problem(synth.FAMILY_GAUSS_MIX, synth.NORM_DENSITY, d, 1, np.zeros(1), mu[None],
                         P[None], 0.0, 0.0, np.full(d, -box), np.full(d, box),
                         np.array([-np.log(lam).sum()]), "spectrum")


def test_reduced_logl_closed_form(oracle_lib):
    """The reduced likelihood of a Gaussian with P = Q diag(lam) Q^T (lam descending) at its
    mode theta* = mu, along the first r columns of Q: l_red(phi) = (1/2) sum log lam -
    (d/2) log 2 pi - (1/2) sum_{i<r} lam_i phi_i^2 and its gradient -lam_i phi_i, in closed
    form from (lam, Q); a displacement read as V^T phi, or another column set, fails both."""
    O = oracle_lib
    d, r = 9, 4
    lam = np.array([40.0, 20.0, 9.0, 5.0, 1.0, 0.5, 0.1, 0.01, 0.001])
    P, q = constructed_spectrum(d, 73, lam)
    mu = np.linspace(-1.0, 1.0, d)
    prob = _gauss_from_spectrum(mu, P)
    phi = np.random.Generator(np.random.PCG64(74)).normal(size=(5, r))
    l, g = O.reduced_logl(prob, mu, q, r, phi)
    ref = 0.5 * np.log(lam).sum() - 0.5 * d * np.log(2 * np.pi) - 0.5 * (phi ** 2 @ lam[:r])
    assert np.max(np.abs(l - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(g - (-lam[:r] * phi))) <= 1e-11


def test_reduced_logl_gradient_central_differences(oracle_lib):
    """Away from a mode, on a two-component mixture with a Haar-random V: the gradient in phi
    is the central difference of l_red (the chain rule V_inform^T grad l)."""
    O = oracle_lib
    rng = np.random.Generator(np.random.PCG64(75))
    prob = synth.gaussian_mixture(rng, 6, 2, -3.0, 3.0, 0.2, 2.0, 4.0, box_half=12.0)
    V = synth.haar_orthogonal(rng, 6)
    th = rng.uniform(-1.0, 1.0, 6)
    phi = rng.normal(size=(3, 3))
    _, g = O.reduced_logl(prob, th, V, 3, phi)
    h = 1e-6
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        lp, _ = O.reduced_logl(prob, th, V, 3, phi + e)
        lm, _ = O.reduced_logl(prob, th, V, 3, phi - e)
        assert np.allclose((lp - lm) / (2 * h), g[:, i], rtol=1e-6, atol=1e-7)


def test_reduced_bounds_hand_values(oracle_lib):
    """Bounds in the reduced space: axis directions give lo - theta* and hi - theta* (a negated
    axis the negated, swapped pair); a 45-degree direction in [-1, 1]^2 from (1/2, 0) leaves
    through x = 1 at t = sqrt(2)/2 and through y = -1 at t = -sqrt(2); a zero component puts
    no bound."""
    O = oracle_lib
    lo, hi = np.array([-1.0, -1.0]), np.array([1.0, 1.0])
    th = np.array([0.5, 0.0])
    c = 1.0 / np.sqrt(2.0)
    V = np.array([[c, 0.0, 1.0], [c, -1.0, 0.0]])
    plo, phi = O.reduced_bounds(th, V, 3, lo, hi)
    assert np.allclose(plo, [-np.sqrt(2.0), -1.0, -1.5], atol=1e-15)
    assert np.allclose(phi, [np.sqrt(2.0) / 2.0, 1.0, 0.5], atol=1e-15)


# ------------------------------------------- generic likelihoods: FD derivatives

def test_fd_exact_for_quadratics(oracle_lib):
    """Central differences have no truncation error on a quadratic: gradient -P(x - mu),
    diagonal and full Hessian -P, up to rounding of order eps_mach |f| / eps^2."""
    O = oracle_lib
    rng = np.random.Generator(np.random.PCG64(90))
    d = 5
    P, _ = synth.random_precision(rng, d, 0.2, 2.0)
    mu = rng.uniform(-1, 1, d)
    f = lambda x: 3.0 - 0.5 * (x - mu) @ P @ (x - mu)
    X = rng.uniform(-2, 2, (3, d))
    eps = 1e-3
    r = O.fd_derivatives(f, X, eps, full=True)
    fmax = max(abs(f(x)) for x in X) + 10.0
    tol_g = 4 * 2.2e-16 * fmax / eps
    tol_h = 16 * 2.2e-16 * fmax / eps ** 2
    assert np.allclose(r["l"], [f(x) for x in X], rtol=0, atol=1e-15 * fmax)
    assert np.max(np.abs(r["grad"] + (X - mu) @ P)) <= tol_g
    assert np.max(np.abs(r["hdiag"] + np.diag(P))) <= tol_h
    assert np.max(np.abs(r["H"] + P[None])) <= tol_h


def test_fd_truncation_error_bound_rosenbrock(oracle_lib):
    """A non-quadratic (negative Rosenbrock): the central-difference errors are the leading
    Taylor terms, eps^2/6 f''' for the gradient, eps^2/12 f'''' for the diagonal: checked
    against the analytic derivatives with those terms bounded by the known fourth and third
    derivatives of the quartic."""
    O = oracle_lib

    def f(x):
        return -np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1.0 - x[:-1]) ** 2)

    def grad(x):
        g = np.zeros_like(x)
        g[:-1] += 400.0 * x[:-1] * (x[1:] - x[:-1] ** 2) + 2.0 * (1.0 - x[:-1])
        g[1:] += -200.0 * (x[1:] - x[:-1] ** 2)
        return g

    def hess(x):
        d = x.size
        H = np.zeros((d, d))
        for i in range(d - 1):
            H[i, i] += -(1200.0 * x[i] ** 2 - 400.0 * x[i + 1] + 2.0)
            H[i + 1, i + 1] += -200.0
            H[i, i + 1] += 400.0 * x[i]
            H[i + 1, i] += 400.0 * x[i]
        return H

    X = np.array([[0.3, -0.2, 0.5, 1.1], [1.0, 1.0, 1.0, 1.0]])
    eps = 1e-4
    r = O.fd_derivatives(f, X, eps, full=True)
    for b, x in enumerate(X):
        # |f'''| <= 2400 |x_i| + ..., |f''''| = 2400 along x_i: truncation <= eps^2 * 2400 * 3
        trunc = eps ** 2 * 2400.0 * (3.0 + np.max(np.abs(x)))
        rnd = 16 * 2.2e-16 * (abs(f(x)) + 1.0) / eps ** 2
        assert np.max(np.abs(r["grad"][b] - grad(x))) <= trunc
        assert np.max(np.abs(r["hdiag"][b] - np.diag(hess(x)))) <= trunc + rnd
        assert np.max(np.abs(r["H"][b] - hess(x))) <= trunc + rnd


def test_fd_rotation_probe(oracle_lib):
    """For a quadratic with H = a0 I + b0 (1 1^T - I) (uniform correlation b0) the probe returns
    b0 exactly (up to rounding): v^T H v = a0 + (d - 1) b0 and mean H_ii = a0; an axis-aligned
    quadratic gives 0."""
    O = oracle_lib
    d, a0, b0 = 6, -3.0, 0.4
    Hm = a0 * np.eye(d) + b0 * (np.ones((d, d)) - np.eye(d))
    f = lambda x: 0.5 * x @ Hm @ x
    X = np.array([[0.1, -0.3, 0.2, 0.0, 0.5, -0.1]])
    r = O.fd_derivatives(f, X, 1e-3)
    assert abs(r["probe_b"][0] - b0) <= 1e-8
    f2 = lambda x: 0.5 * x @ np.diag(np.arange(1.0, d + 1)) @ x
    assert abs(O.fd_derivatives(f2, X, 1e-3)["probe_b"][0]) <= 1e-8


def test_user_mode_evidence_gaussians_closed_form(oracle_lib):
    """Laplace with FD curvature is exact for Gaussians (central differences are exact on
    quadratics): a correlated Gaussian takes the full-Hessian branch, an axis-aligned one the
    diagonal branch, both give the closed form (d/2) log 2 pi + (1/2) sum log lambda - log V;
    a normalised two-component mixture at its means gives -log V to the e^-60 overlap."""
    O = oracle_lib
    d = 6
    rng = np.random.Generator(np.random.PCG64(95))
    P, sll = synth.random_precision(rng, d, 0.1, 1.0)
    mu = rng.uniform(-2, 2, d)
    lo, hi = np.full(d, -10.0), np.full(d, 10.0)
    ref = 0.5 * d * LOG2PI + 0.5 * sll - d * math.log(20.0)
    f = lambda x: -0.5 * (x - mu) @ P @ (x - mu)
    r = O.user_mode_evidence(f, mu[None], lo, hi, 1e-3, 1e-3)
    assert r["full"][0] and abs(r["log_z"] - ref) < 1e-7
    lam = np.exp(rng.uniform(np.log(0.1), 0.0, d))
    f2 = lambda x: -0.5 * np.sum((x - mu) ** 2 / lam)
    r2 = O.user_mode_evidence(f2, mu[None], lo, hi, 1e-3, 1e-3)
    ref2 = 0.5 * d * LOG2PI + 0.5 * np.sum(np.log(lam)) - d * math.log(20.0)
    assert not r2["full"][0] and abs(r2["log_z"] - ref2) < 1e-7
    prob = small_mixture(d=d, K=2, seed=96, box=12.0)
    op = O.OracleProblem(prob)
    fm = lambda x: float(O.logl(prob, x[None], grad=False, op=op)[0])
    r3 = O.user_mode_evidence(fm, prob.mu, prob.lo, prob.hi, 1e-3, 1e-3)
    assert abs(r3["log_z"] + O.log_volume(prob.lo, prob.hi)) < 1e-6


# ---------------------------------------------------------------- ChiSao moves (section
# "ChiSao Exploration": stick detection, Hands Like Clouds, anti-convergence)

def test_chisao_stick_special_cases(oracle_lib):
    """Both conditions at their boundaries: l = l_max + log 0.1 sticks (>=), one ulp below
    does not; |g|_inf equal to the tolerance does not (<); non-finite l or g never sticks and
    a non-finite l does not set l_max."""
    O = oracle_lib
    t = -math.log(10.0)
    l = np.array([0.0, t, np.nextafter(t, -np.inf), 0.0, -5.0, np.inf, np.nan, 0.0])
    G = np.zeros((8, 3))
    G[3, 1] = -1e-6          # |g|_inf == tol: not below
    G[7, 2] = np.nan
    assert O.chisao_stick(l, G, 1e-6).tolist() == [1, 1, 0, 0, 0, 0, 0, 0]
    G[3, 1] = -np.nextafter(1e-6, 0.0)
    assert O.chisao_stick(l, G, 1e-6)[3] == 1
    # l_max from the finite values only; none finite: nothing sticks
    assert O.chisao_stick(np.array([np.nan, -np.inf]), np.zeros((2, 2)), 1.0).tolist() == [0, 0]
    assert O.chisao_stick(np.array([-1.0, -3.0]), np.zeros((2, 2)), 1.0).tolist() == [1, 1]
    assert O.chisao_stick(np.array([-1.0, -3.4]), np.zeros((2, 2)), 1.0).tolist() == [1, 0]


def _isotropic_or_dense(seed, d, dense):
    rng = np.random.Generator(np.random.PCG64(seed))
    prob = synth.gaussian_mixture(rng, d, 1, -1.0, 1.0, 0.5, 2.0, 0.0, box_half=1e6,
                                  norm=synth.NORM_PEAK_ZERO)
    if not dense:
        prob.prec = np.eye(d)[None] * 1.7
    return prob


@pytest.mark.parametrize("dense", [False, True])
def test_chisao_anticonverge_closed_form(oracle_lib, dense):
    """On a Gaussian l = -(x - mu)^T P (x - mu)/2 the momentum descent is linear: in an
    eigenvector basis of P (eigenvalue p) the offset e and velocity v evolve by the 2 x 2
    matrix [[1 + a p, m], [a p, m]] from (e0, 0); its n-th power from the eigenvalues of
    that matrix gives the end point.  Stuck samples keep their coordinates bit for bit."""
    O = oracle_lib
    d, a, m, n = 6, 0.05, 0.9, 7
    prob = _isotropic_or_dense(31 + dense, d, dense)
    rng = np.random.Generator(np.random.PCG64(5))
    X = prob.mu[0] + rng.normal(size=(4, d))
    stuck = np.array([0, 1, 0, 0], dtype=np.uint8)
    out = O.chisao_explore(prob, X, stuck, np.zeros((0, 1, 4, d)), 0.0, 0.0, n, a, m)
    w, Q = np.linalg.eigh(prob.prec[0])
    for b in range(4):
        if stuck[b]:
            assert np.array_equal(out[b], X[b])
            continue
        e0 = Q.T @ (X[b] - prob.mu[0])
        e = np.empty(d)
        for i, p in enumerate(w):
            M = np.array([[1.0 + a * p, m], [a * p, m]])
            lam, U = np.linalg.eig(M)
            Mn = (U @ np.diag(lam ** n) @ np.linalg.inv(U)).real
            e[i] = (Mn @ np.array([e0[i], 0.0]))[0]
        assert np.allclose(out[b], prob.mu[0] + Q @ e, rtol=1e-11, atol=1e-11)


def test_chisao_clouds_closed_form_and_invariants(oracle_lib):
    """Antithetic perturbations (z, -z) make the smoothed gradient of a Gaussian exactly
    -P (x - mu), so n steps of size a give e_n = (I - a P)^n e_0 (per eigenvalue p:
    (1 - a p)^n).  K identical perturbations equal one; sigma = 0 equals plain gradient
    ascent whatever Z holds; a step that overshoots the box ends on its faces."""
    O = oracle_lib
    d, a, n = 5, 0.2, 4
    prob = _isotropic_or_dense(41, d, True)
    rng = np.random.Generator(np.random.PCG64(6))
    X = prob.mu[0] + rng.normal(size=(3, d))
    z = rng.normal(size=(n, 1, 3, d))
    Z = np.concatenate([z, -z], axis=1)
    out = O.chisao_explore(prob, X, np.zeros(3, np.uint8), Z, 0.7, a, 0, 0.0, 0.9)
    w, Q = np.linalg.eigh(prob.prec[0])
    for b in range(3):
        e = (1.0 - a * w) ** n * (Q.T @ (X[b] - prob.mu[0]))
        assert np.allclose(out[b], prob.mu[0] + Q @ e, rtol=1e-11, atol=1e-11)
    one = O.chisao_explore(prob, X, np.zeros(3, np.uint8), z, 0.3, a, 0, 0.0, 0.9)
    three = O.chisao_explore(prob, X, np.zeros(3, np.uint8), np.repeat(z, 3, axis=1), 0.3, a,
                             0, 0.0, 0.9)
    assert np.allclose(one, three, rtol=1e-13, atol=1e-13)
    flat = O.chisao_explore(prob, X, np.zeros(3, np.uint8), Z * 0.0, 0.0, a, 0, 0.0, 0.9)
    assert np.allclose(flat, out, rtol=1e-11, atol=1e-11)
    # overshoot: a tiny box around mu and a huge step
    prob.lo = prob.mu[0] - 0.5
    prob.hi = prob.mu[0] + 0.5
    Xs = prob.mu[0] + np.array([[0.3, -0.3, 0.1, -0.1, 0.2]])
    big = O.chisao_explore(prob, Xs, np.zeros(1, np.uint8), np.zeros((1, 1, 1, d)), 0.0, 1e3,
                           0, 0.0, 0.9)
    g = -prob.prec[0] @ (Xs[0] - prob.mu[0])
    ref = np.where(g > 0, prob.hi, np.where(g < 0, prob.lo, Xs[0]))
    assert np.array_equal(big[0], ref)


def test_chisao_reseed_ray_closed_form(oracle_lib):
    """On a Gaussian peak-zero l the best sample of a ray is the sample nearest (in the
    P-metric) to the ray's maximiser t* = u^T P (mu - x) / u^T P u: the ray's l is a parabola
    in t.  The exit point lies on a face of the box and the samples inside it; u = 0 keeps
    x; a ray along one axis ends at that axis's face."""
    O = oracle_lib
    d, n = 7, 32
    prob = _isotropic_or_dense(51, d, True)
    prob.lo = np.full(d, -3.0)
    prob.hi = np.full(d, 4.0)
    rng = np.random.Generator(np.random.PCG64(52))
    X = rng.uniform(-2.5, 3.5, (6, d))
    U = rng.normal(size=(6, d))
    U[4] = 0.0
    U[5] = 0.0
    U[5, 2] = -0.5
    out, best = O.chisao_reseed(prob, X, U, n)
    P, mu = prob.prec[0], prob.mu[0]
    for b in range(4):
        x, u = X[b], U[b]
        te = np.min(np.where(u > 0, (prob.hi - x) / u, (prob.lo - x) / u))
        end = x + te * u
        assert np.min(np.minimum(np.abs(end - prob.lo), np.abs(end - prob.hi))) < 1e-12
        ts = (np.arange(n) + 0.5) / n * te
        tstar = float(u @ P @ (mu - x)) / float(u @ P @ u)
        curv = float(u @ P @ u)
        val = -0.5 * curv * (ts - tstar) ** 2  # l along the ray up to a constant
        j = int(np.argmax(val))
        assert np.allclose(out[b], x + ts[j] * u, rtol=0, atol=1e-12)
        assert np.all(out[b] >= prob.lo - 1e-12) and np.all(out[b] <= prob.hi + 1e-12)
    assert np.array_equal(out[4], X[4])
    assert np.allclose(out[5][[0, 1, 3, 4, 5, 6]], X[5][[0, 1, 3, 4, 5, 6]], rtol=0, atol=0)
    te5 = (prob.lo[2] - X[5, 2]) / -0.5
    assert np.any(np.isclose(out[5][2], X[5, 2] - 0.5 * (np.arange(n) + 0.5) / n * te5,
                             rtol=0, atol=1e-12))


def test_chisao_orthonormal_properties(oracle_lib):
    """The rows are orthonormal, the draws are recovered as G = R' Q with R' lower triangular
    and a positive diagonal (R' = R^T), and the first row is the first draw normalised."""
    O = oracle_lib
    rng = np.random.Generator(np.random.PCG64(53))
    for n, d in ((1, 1), (3, 3), (5, 9), (16, 40)):
        G = rng.normal(size=(2, n, d))
        Q = O.chisao_orthonormal(G)
        for c in range(2):
            assert np.allclose(Q[c] @ Q[c].T, np.eye(n), atol=1e-13)
            Rt = G[c] @ Q[c].T
            assert np.allclose(np.triu(Rt, 1), 0.0, atol=1e-12)
            assert np.all(np.diag(Rt) > 0)
            assert np.allclose(Q[c, 0], G[c, 0] / np.linalg.norm(G[c, 0]), atol=1e-14)
    G = rng.normal(size=(1, 4, 6))
    G[0, 2] = 2.0 * G[0, 0] - G[0, 1]
    Q = O.chisao_orthonormal(G)
    assert np.all(np.isfinite(Q[0, :2])) and np.all(np.isnan(Q[0, 2:]))


# --------------------------------------------------- ChiSao cycle, refinement pass

def test_chisao_normals_are_standard_normal(oracle_lib):
    """The cycle's draws (Box-Muller on the pinned Philox uniforms) are N(0, 1): mean,
    variance and a Kolmogorov-Smirnov test on 250000 draws (a sample of 20000 is too small to
    tell a mild distortion from noise), and draws of two streams are uncorrelated."""
    O = oracle_lib
    z = np.array([O.chisao_normal(5, 0, r, O.CHISAO_STREAM0 + 4, i)
                  for r in range(500) for i in range(500)])
    assert abs(float(z.mean())) < 4.0 / math.sqrt(z.size)
    assert abs(float(z.var()) - 1.0) < 0.01
    assert st.kstest(z, "norm").pvalue > 1e-3
    w = np.array([O.chisao_normal(5, 0, r, O.CHISAO_STREAM0 + 2, i)
                  for r in range(100) for i in range(200)])
    assert abs(float(np.corrcoef(z[:w.size], w)[0, 1])) < 4.0 / math.sqrt(w.size)


def _hidden(d=8, seed=11):
    return synth.hidden_mode_mixture(d, seed)


def test_chisao_cycle_finds_what_one_phase_provably_misses(oracle_lib):
    """A narrow high component at the centre and a wide low one off-centre.  Every start of the
    coarse pass has l above the wide component's mode value, so a monotone optimiser (Armijo
    L-BFGS never lowers l) cannot reach that mode from any start: one convergence phase finds
    only the narrow mode.  The oscillation cycle (reseeding, smoothing, momentum descent) finds
    both, and its result equals the reference set (Newton from each mean) to 1e-8 / 1e-9."""
    O = oracle_lib
    prob = _hidden()
    cfg = synth.RunConfig(n_rays=256, n_points=32, n_starts=16, seed=77)
    ref = O.reference_modes(prob)
    assert ref.status == 0 and ref.n_modes == 2
    l_wide = float(np.min(ref.mode_logl))
    disc = O.discover(prob, cfg.n_rays, cfg.n_points, cfg.n_starts, cfg.seed)
    l0 = O.logl(prob, disc["X0"], grad=False)
    assert float(np.min(l0)) > l_wide + 1.0
    one = O.evidence(prob, cfg)
    assert one.status == 0 and one.n_modes == 1
    prm = O.ChiSaoParams(n_osc=3, n_anti=10, alpha_anti=0.05)
    cyc = O.evidence_chisao(prob, cfg, prm)
    assert cyc.status == 0 and cyc.n_modes == 2, cyc.cycle
    assert float(np.max(np.abs(cyc.modes - ref.modes))) <= 1e-8
    assert abs(cyc.log_z - ref.log_z) <= 1e-9
    assert float(np.max(np.abs(cyc.mode_log_z - ref.mode_log_z))) <= 1e-9
    assert cyc.cycle[0]["reseed"] == 2  # every start converged to one peak: Golden Rooster


def test_chisao_cycle_single_oscillation_is_the_single_phase(oracle_lib):
    """n_osc = 1 without refinement: the coarse pass, one convergence phase and the same tail,
    so the mode set and log Z equal the single-phase path's (starts agree to rounding of the
    ray points)."""
    O = oracle_lib
    for name, ns in (("c0", None), ("c1", 128)):
        prob, cfg = synth.make_workload(name, n_starts=ns)
        a = O.evidence(prob, cfg)
        b = O.evidence_chisao(prob, cfg, O.ChiSaoParams(n_osc=1))
        assert a.status == b.status == 0 and a.n_modes == b.n_modes
        assert abs(a.log_z - b.log_z) <= 1e-12
        assert float(np.max(np.abs(a.modes - b.modes))) <= 1e-10
        assert b.cycle[0]["reseed"] == 0


def test_chisao_cycle_golden_rooster_disables_itself(oracle_lib):
    """One Gaussian: every sample converges to its mode, the duplicates are lost and Golden
    Rooster refills them; the next oscillation finds no new peak, so Golden Rooster is off
    and the lost slots stay empty; the result is the closed form."""
    O = oracle_lib
    prob, cfg = synth.make_workload("c0")
    cfg.n_starts = 16
    cyc = O.evidence_chisao(prob, cfg, O.ChiSaoParams(n_osc=3, n_anti=6, alpha_anti=0.05))
    kinds = [c["reseed"] for c in cyc.cycle]
    assert kinds == [2, 0, 0], cyc.cycle
    assert [c["golden_rooster"] for c in cyc.cycle] == [True, False, False]
    assert cyc.cycle[1]["found"] == 1 and cyc.cycle[2]["lost"] == 0
    ref = O.reference_modes(prob)
    assert cyc.n_modes == 1 and abs(cyc.log_z - ref.log_z) <= 1e-10


@pytest.mark.parametrize("n_far,kind", [(6, 1), (5, 1), (4, 2)])
def test_chisao_cycle_reseed_rule_boundary(oracle_lib, n_far, kind):
    """Ten samples start at the mode (they converge at once, stick, and nine are lost) and
    n_far start far away (one L-BFGS step leaves them unconverged): with at least five
    unconverged samples Repulse Monkey reseeds, with fewer Golden Rooster."""
    O = oracle_lib
    prob, _ = synth.make_workload("c0")
    mode = O.reference_modes(prob).modes[0]
    far = mode + np.array([6.0, -5.0, 4.0, -3.0])
    X0 = np.array([mode] * 10 + [far * (1.0 - 0.05 * j) for j in range(n_far)])
    prm = O.ChiSaoParams(n_osc=2, n_conv=1, n_anti=2, alpha_anti=0.01)
    cyc = O.chisao_cycle(prob, X0, prm, grad_tol=1e-10, dedup_tol=0.25, seed=3)
    c0 = cyc["log"][0]
    assert c0["lost"] == 9 and c0["peaks"] == 1 and c0["reseed"] == kind, c0
    assert c0["converged"] == 10


def test_refine_rays_closed_forms(oracle_lib):
    """Refinement pass: on a flat likelihood the refined points are the uniform quantiles
    (i + 1/2)/n_ref of the whole ray; on a Gaussian the ray's l is a parabola in t and the best
    refined point lies closer to its maximiser than half a coarse spacing, shrinking as n_ref
    grows; with n_ref = 0 the best point is the coarse argmax of the discovery pass."""
    O = oracle_lib
    prob, cfg = synth.make_workload("c0")
    R = 16
    P0, P1 = O.rays(prob.d, prob.lo, prob.hi, R, 9)
    flat = prob.copy()
    flat.prec = flat.prec * 0.0 + np.eye(prob.d)[None] * 1e-300
    rf = O.refine_rays(flat, P0, P1, 8, 10, 10.0)
    assert np.allclose(rf["t_refined"], ((np.arange(10) + 0.5) / 10)[None], atol=1e-15)
    n_pts = 8
    errs = []
    for n_ref in (0, 8, 64):
        rf = O.refine_rays(prob, P0, P1, n_pts, n_ref, 10.0)
        e = 0.0
        for r in range(R):
            D = P1[r] - P0[r]
            a = O.logl(prob, P0[r][None], grad=False)[0]
            # t* maximises the parabola l(P0 + t D): from the gradient at P0 and the curvature
            _, g = O.logl(prob, P0[r][None])
            curv = -float(D @ prob.prec[0] @ D)
            tstar = min(1.0, max(0.0, -float(g[0] @ D) / curv))
            e = max(e, abs(rf["best_t"][r] - tstar))
        errs.append(e)
    assert errs[0] <= 0.5 / n_pts + 1e-12
    assert errs[1] < errs[0] and errs[2] < errs[1]
    d0 = O.discover(prob, R, n_pts, R, 9)
    rf0 = O.refine_rays(prob, P0, P1, n_pts, 0, 10.0)
    assert np.allclose(rf0["best_l"], d0["ray_best_l"], rtol=1e-13, atol=1e-12)
    assert np.allclose(rf0["best_t"], (d0["ray_best_j"] + 0.5) / n_pts, atol=0)


def test_chisao_whole_path_with_refinement_equals_reference(oracle_lib):
    """The coarse and refinement passes feeding the cycle on c1's mixture (fewer starts):
    the mode set and log Z equal the reference set's (the refinement changes only where the
    starts sit)."""
    O = oracle_lib
    prob, cfg = synth.make_workload("c1", n_starts=64)
    ref = O.reference_modes(prob)
    for n_osc in (1, 2):
        r = O.evidence_chisao(prob, cfg, O.ChiSaoParams(n_osc=n_osc, n_anti=4, alpha_anti=0.01),
                              n_ref=8)
        assert r.status == 0 and r.n_modes == ref.n_modes == prob.K
        assert float(np.max(np.abs(r.modes - ref.modes))) <= 1e-8
        assert abs(r.log_z - ref.log_z) <= 1e-9


@pytest.mark.parametrize("n,d", [(4, 6), (16, 16), (24, 64)])
def test_chisao_orthonormal_dependence_threshold(oracle_lib, n, d):
    """A draw whose component outside the earlier rows' span has relative size delta is
    dependent (it and the later rows NaN) when delta <= 8 n eps, independent above: exact
    combinations and delta = 0.5 x threshold give NaN, delta = 2 x threshold and 1e3 x give
    finite orthonormal rows (rounding of the projections, ~n eps, is far from either side)."""
    O = oracle_lib
    thr = 8.0 * n * np.finfo(np.float64).eps
    rng = np.random.Generator(np.random.PCG64(100 + n))
    k = n // 2
    base = rng.normal(size=(n, d))
    Qs, _ = np.linalg.qr(base[:k].T, mode="complete")
    v = Qs[:, k]  # unit vector orthogonal to the first k rows
    comb = rng.normal(size=k) @ base[:k]
    for delta, dependent in ((0.0, True), (0.5 * thr, True), (2.0 * thr, False),
                             (1e3 * thr, False)):
        G = base.copy()
        # |comb + t v| = |g|, t = delta |g|:  t^2 (1 - delta^2) = delta^2 |comb|^2
        t = delta * np.linalg.norm(comb) / math.sqrt(1.0 - delta * delta)
        G[k] = comb + t * v
        Q = O.chisao_orthonormal(G[None])[0]
        assert np.all(np.isfinite(Q[:k]))
        if dependent:
            assert np.all(np.isnan(Q[k:])), delta
        else:
            assert np.all(np.isfinite(Q[k:])), delta
            assert np.allclose(Q @ Q.T, np.eye(n), atol=1e-10)


# ------------------------------------------- trajectory-based rotation detection

def _quad(H, mu):
    def f(x):
        dlt = x - mu
        return -0.5 * float(dlt @ H @ dlt)
    return f


def _quad_logz(H, lo, hi):
    d = H.shape[0]
    return 0.5 * d * math.log(2 * math.pi) - 0.5 * float(np.linalg.slogdet(H)[1]) \
        - float(np.sum(np.log(hi - lo)))


def test_perpendicular_fraction_axis_aligned_is_zero(oracle_lib):
    """Axis-aligned anisotropic quadratic: from the axis seeds every L-BFGS step stays on its
    axis, so in whitened coordinates steps and gradients are parallel: f_perp = 0 to
    rounding, the mode is classed axis-aligned without the probe, log Z is the closed form."""
    O = oracle_lib
    d = 6
    h = synth.log_uniform(np.random.Generator(np.random.PCG64(3)), 0.1, 10.0, d)
    H = np.diag(h)
    mu = np.linspace(-1.0, 1.0, d)
    f = _quad(H, mu)
    lo, hi = np.full(d, -10.0), np.full(d, 10.0)
    fp = O.trajectory_geometry(f, mu[None], -h[None], 1e-4, 12)
    assert fp[0] <= 1e-8, fp
    r = O.user_mode_evidence_geo(f, mu[None], lo, hi, 1e-4, 1e-3, 12, 1e-4, 1e-2)
    assert r["decision"][0] == 0
    assert abs(r["log_z"] - _quad_logz(H, lo, hi)) <= 1e-6


def test_perpendicular_fraction_first_step_closed_form(oracle_lib):
    """From the seed mu + delta e_i the first step follows the gradient -delta H[:, i], so its
    fraction is |D^1/2 c - proj| / |D^1/2 c| with c = H[:, i], D = diag(H), projected on
    D^-1/2 c: equal to the trajectory's first recorded step for every seed."""
    O = oracle_lib
    d = 5
    rng = np.random.Generator(np.random.PCG64(8))
    P, _ = synth.random_precision(rng, d, 0.2, 2.0)
    mu = rng.normal(size=d)
    f = _quad(P, mu)
    hd = np.diag(P)
    seeds = O.greendragon_seeds(mu, -hd)
    for j, x0 in enumerate(seeds):
        tr = O.lbfgs_user(f, x0, 1e-4, max_iter=1)
        got = O.perpendicular_step_fraction(tr["X"], tr["G"], hd)[0]
        c = P[:, j // 2]
        du = np.sqrt(hd) * c
        gw = c / np.sqrt(hd)
        want = np.linalg.norm(du - (du @ gw) / (gw @ gw) * gw) / np.linalg.norm(du)
        assert abs(got - want) <= 1e-8, (j, got, want)


def test_rotated_gaussian_with_zero_offdiagonal_sum_needs_the_trajectories(oracle_lib):
    """A rotated Gaussian whose off-diagonal entries sum to zero: the probe sees b = 0 (it only
    measures the uniform part of the correlation), so the probe alone takes the diagonal
    Laplace and misses log Z; the trajectories see the rotation, the full Hessian is taken and
    log Z is the closed form."""
    O = oracle_lib
    d = 6
    rng = np.random.Generator(np.random.PCG64(21))
    P, _ = synth.random_precision(rng, d, 0.3, 1.0)
    off = P - np.diag(np.diag(P))
    c = float(off.sum()) / (d * (d - 1))
    H = P - c * (np.ones((d, d)) - np.eye(d))
    assert abs(float((H - np.diag(np.diag(H))).sum())) < 1e-12
    assert np.all(np.linalg.eigvalsh(H) > 0)
    mu = rng.normal(size=d)
    f = _quad(H, mu)
    lo, hi = np.full(d, -10.0), np.full(d, 10.0)
    exact = _quad_logz(H, lo, hi)
    probe = O.fd_derivatives(f, mu[None], 1e-4)
    assert abs(probe["probe_b"][0]) <= 1e-6 * abs(float(np.mean(probe["hdiag"][0])))
    old = O.user_mode_evidence(f, mu[None], lo, hi, 1e-4, 1e-3)
    assert abs(old["log_z"] - exact) > 0.05
    new = O.user_mode_evidence_geo(f, mu[None], lo, hi, 1e-4, 1e-3, 12, 1e-4, 1e-2)
    assert new["decision"][0] == 1 and new["fperp"][0] > 0.05
    assert abs(new["log_z"] - exact) <= 1e-6


def test_uniform_correlation_detected_by_both_steps(oracle_lib):
    """H = a I + b 1 1^T (uniformly correlated): the trajectories and the probe both see it."""
    O = oracle_lib
    d = 5
    H = 1.0 * np.eye(d) + 0.3 * np.ones((d, d))
    mu = np.zeros(d)
    f = _quad(H, mu)
    lo, hi = np.full(d, -8.0), np.full(d, 8.0)
    r = O.user_mode_evidence_geo(f, mu[None], lo, hi, 1e-4, 1e-3, 12, 1e-4, 1e-2)
    assert r["decision"][0] == 1
    pr = O.fd_derivatives(f, mu[None], 1e-4)
    assert abs(pr["probe_b"][0] + 0.3) <= 1e-6  # b of the Hessian of l, -0.3 off the diagonal
    assert abs(r["log_z"] - _quad_logz(H, lo, hi)) <= 1e-6
