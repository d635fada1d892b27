"""Batched evidence of many independent problems of uneven dimension
(sb_evidence_batch) against the oracle, problem by problem.

Problem j of a batch draws its rays with Philox counter word 3 = j, so its
oracle run passes problem=j.  FP64 batches are held to the single-problem
bar (|d log Z| <= 1e-9, modes 1e-8); mixed-precision batches to 1e-6.
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


def absmax(a):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64)))) if np.size(a) else 0.0


def c3_member(d, K, seed):
    """One problem of the uneven-batch recipe: K separated Gaussians (density
    normalised, Dirichlet weights), box half-width 3 max |mu|."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.gaussian_mixture(rng, d, K, -8.0, 8.0, 0.05, 1.0, 12.0, box_from_mu=3.0,
                                  norm=synth.NORM_DENSITY)


def mixed_batch():
    """Uneven dimensions (ragged and multiples of 8), K = 1..4, both families,
    both normalisations."""
    probs = []
    for i, (d, K) in enumerate([(1, 1), (8, 2), (13, 3), (24, 4), (37, 2), (64, 1), (100, 2)]):
        probs.append(c3_member(d, K, 7000 + i))
    rng = np.random.Generator(np.random.PCG64(7100))
    probs.append(synth.student_t(rng, 20, 30.0, -5.0, 5.0, 0.01, 1.0, 20.0))
    probs.append(synth.make_problem("c0"))
    return probs


def cfg_for(j, precision=0, n_starts=128, **kw):
    return synth.RunConfig(n_rays=2 * n_starts, n_points=32, n_starts=n_starts,
                           precision=precision, seed=4242 + 17 * j, **kw)


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


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_oracle(L, precision):
    probs = mixed_batch()
    cfgs = [cfg_for(j, precision) for j in range(len(probs))]
    res = L.sb_evidence_batch(probs, cfgs)
    for j, (p, r) in enumerate(zip(probs, res)):
        ref = O.evidence(p, cfg_for(j, 0), problem=j)
        print(f"problem {j} d={p.d} K={p.K}: dlogZ={abs(r.log_z - ref.log_z):.3e}", flush=True)
        _compare(r, ref, 1e-9 if precision == 0 else 1e-6)


def test_batch_long_memory(L):
    """A batch whose starts keep 24 history pairs (read from memory in the recursion)."""
    probs = mixed_batch()[:5]
    cfgs = [cfg_for(j, 0, m=24) for j in range(len(probs))]
    res = L.sb_evidence_batch(probs, cfgs)
    for j, (p, r) in enumerate(zip(probs, res)):
        ref = O.evidence(p, cfg_for(j, 0, m=24), problem=j)
        _compare(r, ref, 1e-9)


def test_batch_of_one_matches_single(L):
    prob, cfg = synth.make_workload("c1", n_starts=256)
    [rb] = L.sb_evidence_batch([prob], [cfg])
    rs = L.sb_evidence(prob, cfg)
    assert rb.status == 0 and rs.status == 0
    assert rb.n_modes == rs.n_modes
    assert abs(rb.log_z - rs.log_z) <= 1e-9
    assert absmax(rb.modes - rs.modes) <= 1e-8


def test_batch_per_problem_statuses(L):
    """A capacity overflow and a problem without modes do not disturb the others."""
    good = c3_member(16, 3, 7200)
    over, _ = synth.make_workload("c1", n_starts=128)
    none = synth.make_problem("c0")
    none.mu = none.mu + 25.0  # the peak leaves the box: no mode passes the filters
    probs = [good, over, none]
    cfgs = [cfg_for(j) for j in range(3)]
    cfgs[1].max_modes = 2
    res = L.sb_evidence_batch(probs, cfgs)
    assert res[1].status == L.E_CAPACITY and math.isnan(res[1].log_z)
    assert res[2].status == L.E_NOMODE and res[2].log_z == -math.inf
    _compare(res[0], O.evidence(good, cfg_for(0), problem=0), 1e-9)


def test_batch_rejects_mixed_precisions(L):
    probs = [c3_member(8, 1, 7300), c3_member(8, 1, 7301)]
    with pytest.raises(L.SbError):
        L.sb_evidence_batch(probs, [cfg_for(0, 0), cfg_for(1, 1)])


def _logsumexp(v):
    v = np.sort(np.asarray(v, dtype=np.float64))[::-1]
    if v.size == 0:
        return -math.inf
    return float(v[0] + math.log(np.sum(np.exp(v - v[0]))))


def test_batch_full_uneven_workload(L):
    """512 problems, d log-uniform in 8..512, K in 1..4, 1024 starts each,
    FP64.  Every problem must find all K modes (a separated mixture has one
    maximum per component inside its box, and discovery that loses one is a
    bug), each equal to one of the oracle's reference modes (Newton from each
    mean) to 1e-8 with its log Z_k to 1e-9, and log Z must equal both the
    logsumexp of the reference values and the closed form -log V of a
    density-normalised separated mixture to 1e-9.  A sample of problems runs
    through the whole oracle path."""
    from concurrent.futures import ThreadPoolExecutor

    probs, cfg = synth.make_workload("c3")
    cfgs = [synth.make_run_config("c3", seed=cfg.seed + j) for j in range(len(probs))]
    res = L.sb_evidence_batch(probs, cfgs)
    print(f"batch done: {len(probs)} problems", flush=True)
    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(O.reference_modes, probs))
    complete, worst_cf = 0, 0.0
    for j, (p, r, ref) in enumerate(zip(probs, res, refs)):
        assert r.status == 0, (j, r.status)
        assert ref.status == 0 and ref.n_modes == p.K, (j, ref.n_modes, p.K)
        assert r.n_modes == p.K, (j, p.d, p.K, r.n_modes, r.n_reps_pre, r.n_candidates)
        picked = []
        for k in range(r.n_modes):
            dist = np.max(np.abs(ref.modes[:ref.n_modes] - r.modes[k]), axis=1)
            i = int(np.argmin(dist))
            assert dist[i] <= 1e-8, (j, k, float(dist[i]))
            assert abs(r.mode_log_z[k] - ref.mode_log_z[i]) <= 1e-9, (j, k)
            picked.append(i)
        assert len(set(picked)) == len(picked), (j, picked)
        assert abs(r.log_z - _logsumexp(ref.mode_log_z[picked])) <= 1e-9, j
        cf = -float(np.sum(np.log(p.hi - p.lo)))
        worst_cf = max(worst_cf, abs(r.log_z - cf))
        assert abs(r.log_z - cf) <= 1e-9, (j, r.log_z, cf)
        complete += 1
    print(f"all modes found in {complete}/{len(probs)} problems; "
          f"max |log Z - closed form|: {worst_cf:.3e}", flush=True)
    order = np.argsort([p.d for p in probs], kind="stable")
    for j in [int(order[0]), int(order[1]), int(order[len(order) // 4])]:
        ref = O.evidence(probs[j], cfgs[j], problem=j)
        _compare(res[j], ref, 1e-9)
