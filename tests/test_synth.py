"""Checks of the seeded input generators (shared by the oracle and the GPU path)."""
import math

import numpy as np

import synth


def test_splitmix64_counter_form_is_the_sequential_generator():
    """Value i of stream s is the (i+1)-th output of SplitMix64 started at state s
    (Steele, Lea & Flood 2014): compare with a step-by-step Python-int evaluation."""
    mask = (1 << 64) - 1
    for seed in (0, 1, 1234567, 2**63 + 5):
        state, ref = seed, []
        for _ in range(6):
            state = (state + 0x9E3779B97F4A7C15) & mask
            z = state
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
            ref.append(z ^ (z >> 31))
        got = synth.splitmix64(seed, np.arange(6, dtype=np.uint64))
        assert [int(v) for v in got] == ref


def test_uniform_range_and_moments():
    u = synth.uniform(7, 0, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5e-3 and abs(u.var() - 1 / 12) < 2e-3


def test_boundary_points_lie_on_faces():
    for d, lo in [(2, 0), (5, 0), (5, 1)]:
        x = synth.sample_boundary(11, 0, 4000, d, lo)
        on = (x[:, lo:] == 0.0) | (x[:, lo:] == 1.0)
        assert (on.sum(1) == 1).all()
        faces = np.argmax(on, 1) * 2 + x[np.arange(4000), lo + np.argmax(on, 1)].astype(int)
        counts = np.bincount(faces, minlength=2 * (d - lo))
        assert counts.min() > 0.7 * 4000 / (2 * (d - lo))


def test_problem_targets_are_consistent():
    p = synth.poisson5d()
    xi, yi, xb, yb = p.batch(0)
    assert xi.shape == (3000, 5) and xb.shape == (500, 5)
    np.testing.assert_allclose(yi, math.pi ** 2 * np.sin(math.pi * xi).sum(1))
    xi1 = p.batch(1)[0]
    assert not np.array_equal(xi, xi1)          # resampled every step
    h = synth.heat4d()
    xi, yi, xb, yb = h.batch()
    assert xb.shape == (2000, 5) and (xb[:1000, 0] == 0).all() and (yi == 0).all()
    assert synth.poisson100d().theta0().shape == (1325057,)


def test_batch_instances():
    inst = synth.batch_instances()
    assert len(inst) == 64
    assert {p.d for p in inst} <= {2, 5, 10, 20}
    assert all(500 <= p.n_interior <= 4000 and p.n_boundary == -(-p.n_interior // 6) for p in inst)
    assert all(p.widths[1] in (64, 128, 256) for p in inst)
