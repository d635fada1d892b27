"""Seeded generator checks: shapes, ranges, SPD, separation, reproducibility."""
import math

import numpy as np

from paper_2601_19957_amd import synth


def test_haar_orthogonal():
    rng = np.random.Generator(np.random.PCG64(1))
    q = synth.haar_orthogonal(rng, 50)
    assert np.max(np.abs(q.T @ q - np.eye(50))) < 1e-13


def test_precision_spectrum():
    rng = np.random.Generator(np.random.PCG64(2))
    p, sll = synth.random_precision(rng, 40, 0.05, 1.0)
    assert np.array_equal(p, p.T)
    ev = np.linalg.eigvalsh(p)
    assert ev.min() >= 1.0 - 1e-9 and ev.max() <= 20.0 + 1e-9
    assert abs(-np.sum(np.log(ev)) - sll) < 1e-9


def test_dirichlet_sums_to_one():
    rng = np.random.Generator(np.random.PCG64(3))
    w = synth.dirichlet_ones(rng, 8)
    assert abs(w.sum() - 1.0) < 1e-15 and np.all(w > 0)


def test_workloads_shapes_and_separation():
    c1 = synth.make_problem("c1")
    assert (c1.d, c1.K) == (64, 4) and abs(np.exp(c1.log_w).sum() - 1) < 1e-14
    for i in range(4):
        for j in range(i + 1, 4):
            v = c1.mu[i] - c1.mu[j]
            assert min(v @ c1.prec[i] @ v, v @ c1.prec[j] @ v) >= 144.0
            assert np.max(np.abs(v)) >= 2.5
    c0 = synth.make_problem("c0")
    assert c0.d == 4 and c0.norm == synth.NORM_PEAK_ZERO and np.all(c0.hi == 10.0)
    c2 = synth.make_problem("c2", d=32)
    assert c2.family == synth.FAMILY_STUDENT_T and c2.nu == 30.0


def test_reproducible():
    a = synth.make_problem("c1", d=16)
    b = synth.make_problem("c1", d=16)
    assert np.array_equal(a.prec, b.prec) and np.array_equal(a.mu, b.mu)


def test_c3_dimensions_and_boxes():
    ps = synth.make_problem("c3", n_problems=20)
    for p in ps:
        assert 8 <= p.d <= 512 and 1 <= p.K <= 4
        h = 3.0 * np.max(np.abs(p.mu))
        assert np.allclose(p.hi, h) and np.allclose(p.lo, -h)
    assert synth.c3_dimension(0.0) == 8 and synth.c3_dimension(0.999999999) == 512
