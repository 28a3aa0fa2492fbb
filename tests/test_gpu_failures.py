"""Failure handling on the device, through the C ABI: every condition is created
from the host (inputs, hyper-parameters, the sweep cap) and every kernel exits
normally; the step must then report the status and leave the parameters, the
momentum and the step counter untouched.  Also the two closed-form pins of the
step on the GPU: the damping of all four factors and the line-search tie rule."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import problem_inputs, rel, to_dev

pytestmark = pytest.mark.gpu


def tiny(kind="poisson"):
    return synth.small_problem(kind, (3, 16, 12, 1), 37, 11, n_init=5 if kind == "heat" else 0,
                               problem_id=71)


def run_one(kp, th, xi, yi, xb, yb, hp, precision):
    from paper_2405_15603_amd import KfacPinn
    tht = to_dev(th, precision)
    dev = [to_dev(a, precision) for a in (xi, yi, xb, yb)]
    info = KfacPinn.decode_info(kp.step(tht, *dev, hp))
    return tht, info, kp.sync()


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16"])
def test_nan_point_reports_nonfinite_and_takes_no_step(precision):
    from paper_2405_15603_amd import HParams, KfacPinn
    from paper_2405_15603_amd import _native as N
    p = tiny()
    th, xi, yi, xb, yb = problem_inputs(p, precision)
    kp = KfacPinn.for_problem(p, precision)
    hp = HParams(lam=1e-3, beta=0.886041, momentum=0.707588)
    tht, info, st = run_one(kp, th, xi, yi, xb, yb, hp, precision)   # one good step
    assert st == 0 and info["status"] == 0 and info["step"] == 1
    theta_before = tht.clone()
    mom_before = kp.get_momentum().clone()
    xi_bad = xi.copy()
    xi_bad[5, 1] = np.nan
    dev = [to_dev(a, precision) for a in (xi_bad, yi, xb, yb)]
    info = KfacPinn.decode_info(kp.step(tht, *dev, hp))
    st = kp.sync()
    assert st == N.KP_ERR_NONFINITE and info["status"] == N.KP_ERR_NONFINITE
    assert info["lr"] == 0.0 and info["step"] == 1
    assert torch.equal(tht, theta_before)
    assert torch.equal(kp.get_momentum(), mom_before)


def test_singular_damped_factor_reports_not_pd():
    """A zero output layer makes every hidden layer's output gradient g exactly 0,
    so with beta = 0 the interior B factors of those layers are exactly zero and,
    with lambda = 0, their damped Cholesky meets a zero pivot."""
    from paper_2405_15603_amd import HParams, KfacPinn
    from paper_2405_15603_amd import _native as N
    p = tiny()
    th, xi, yi, xb, yb = problem_inputs(p, "f64")
    off = synth.layer_offsets(p.widths)
    th = th.copy()
    th[off[-2]:off[-1]] = 0.0
    kp = KfacPinn.for_problem(p, "f64")
    tht, info, st = run_one(kp, th, xi, yi, xb, yb, HParams(lam=0.0, beta=0.0), "f64")
    assert st == N.KP_ERR_NOT_PD and info["status"] == N.KP_ERR_NOT_PD
    assert info["lr"] == 0.0 and info["step"] == 0
    assert torch.equal(tht, to_dev(th, "f64"))
    assert float(kp.get_momentum().abs().max()) == 0.0


def test_sweep_cap_reports_not_converged():
    """One Jacobi sweep from a cold start cannot diagonalise the whitened boundary
    factors of a 2d Poisson net: the step reports KP_ERR_NOT_CONVERGED and takes no
    step; with the default cap the same step converges."""
    from paper_2405_15603_amd import HParams, KfacPinn
    from paper_2405_15603_amd import _native as N
    p = synth.poisson2d()
    th, xi, yi, xb, yb = problem_inputs(p, "f64")
    kp = KfacPinn.for_problem(p, "f64")
    kp.set_max_sweeps(1)
    hp = HParams(lam=1e-3, beta=0.0)
    tht, info, st = run_one(kp, th, xi, yi, xb, yb, hp, "f64")
    assert kp.get_sweeps() and max(kp.get_sweeps()) == 1
    assert st == N.KP_ERR_NOT_CONVERGED and info["status"] == N.KP_ERR_NOT_CONVERGED
    assert info["step"] == 0 and torch.equal(tht, to_dev(th, "f64"))
    kp.set_max_sweeps(20)
    kp.reset_state(True)
    tht, info, st = run_one(kp, th, xi, yi, xb, yb, hp, "f64")
    assert st == 0 and info["status"] == 0 and max(kp.get_sweeps()) < 20
    with pytest.raises(Exception):
        kp.set_max_sweeps(0)


@pytest.mark.parametrize("lam", [1e-3, 0.5])
def test_damping_of_zero_factors(lam):
    """All four factors zero: the damped Kronecker sum is 2 lambda^2 I and the
    preconditioned direction is -g / (2 lambda^2) (the oracle pin on the GPU)."""
    from paper_2405_15603_amd import KfacPinn
    p = tiny("heat")
    kp = KfacPinn.for_problem(p, "f64")
    for l in range(len(p.widths) - 1):
        for t in (0, 1):
            for s in (0, 1):
                n = p.widths[l] + 1 if s == 0 else p.widths[l + 1]
                kp.set_factor(l, t, s, torch.zeros(n, n, dtype=torch.float64))
    kp.invert(lam)
    g = torch.Generator().manual_seed(2)
    grad = torch.randn(kp.D, generator=g, dtype=torch.float64).cuda()
    delta = kp.precondition(grad)
    assert kp.sync() == 0
    assert rel(delta, -grad / (2 * lam * lam)) < 1e-13


@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_line_search_tie_goes_to_the_largest_step(precision):
    """Zero output layer and zero targets: Delta = 0, all candidate losses are 0,
    and the first strict minimum from the largest step is alpha* = 2^0, as on the
    oracle."""
    from paper_2405_15603_amd import HParams, KfacPinn
    p = synth.small_problem("poisson", (3, 7, 5, 1), 13, 6, problem_id=79)
    th = p.theta0().copy()
    off = synth.layer_offsets(p.widths)
    th[off[-2]:off[-1]] = 0.0
    xi, yi, xb, yb = p.batch()
    yi, yb = 0.0 * yi, 0.0 * yb
    kp = KfacPinn.for_problem(p, precision)
    tht, info, st = run_one(kp, th, xi, yi, xb, yb, HParams(lam=1e-3, beta=0.0), precision)
    assert st == 0 and info["status"] == 0
    ls = kp.get_line_search(31).cpu().numpy()
    assert np.all(ls == 0.0)
    _, _, rinfo = oracle.kfac_step(th, p.widths, (xi, yi, xb, yb), oracle.operator_of(p),
                                   oracle.HParams(lam=1e-3, beta=0.0, lr_mode="grid"),
                                   oracle.init_state(p.widths, True))
    assert info["lr"] == rinfo.lr == 1.0
