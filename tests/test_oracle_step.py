"""Pins for the oracle's KFAC step (Section 3.4 and Algorithm 1): the update
direction against a dense solve with the block-diagonal Kronecker-sum curvature,
the grid line search against the closed-form minimiser of a quadratic, momentum,
EMA initialisation, and the non-finite guard."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.kfac import DT


def tiny(kind="poisson", widths=(2, 6, 5, 1), n=12, m=8, seed=0):
    p = synth.small_problem(kind, widths, n, m, n_init=4 if kind == "heat" else 0,
                            problem_id=50 + seed)
    return p, torch.as_tensor(p.theta0()), tuple(torch.as_tensor(a) for a in p.batch())


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_direction_matches_dense_block_solve(kind):
    p, th, data = tiny(kind, widths=(2, 5, 4, 1) if kind == "poisson" else (3, 5, 4, 1))
    op = oracle.operator_of(p)
    hp = oracle.HParams(lam=1e-2, beta=0.0, lr_mode="fixed", lr=1.0)
    st = oracle.init_state(p.widths, True)
    th1, st1, info = oracle.kfac_step(th, p.widths, data, op, hp, st)
    # dense reference: -(A_i (x) B_i + A_b (x) B_b + damping)^-1 g per layer
    gW = oracle.unpack(info.gradient, p.widths)
    ref = []
    for l in range(len(gW)):
        Ai, Bi = oracle.damp(st1.A_int[l], hp.lam), oracle.damp(st1.B_int[l], hp.lam)
        Ab, Bb = oracle.damp(st1.A_bnd[l], hp.lam), oracle.damp(st1.B_bnd[l], hp.lam)
        ref.append(-oracle.kron_sum_solve_dense(Ai, Bi, Ab, Bb, gW[l]))
    torch.testing.assert_close(info.direction, oracle.pack(ref), rtol=1e-9, atol=1e-12)
    torch.testing.assert_close(th1, th + info.direction, rtol=0, atol=1e-15)


def test_ema_and_momentum():
    p, th, data = tiny()
    op = oracle.operator_of(p)
    hp = oracle.HParams(lam=1e-3, beta=0.75, momentum=0.5, lr_mode="fixed", lr=0.25)
    st0 = oracle.init_state(p.widths, True)
    th1, st1, i1 = oracle.kfac_step(th, p.widths, data, op, hp, st0)
    Ws = oracle.unpack(th, p.widths)
    Ai, Bi = oracle.interior_factors(oracle.interior_curvature_inputs(Ws, data[0], data[1], op))
    for l in range(len(Ws)):
        torch.testing.assert_close(st1.A_int[l], 0.75 * torch.eye(Ai[l].shape[0], dtype=DT) + 0.25 * Ai[l])
        torch.testing.assert_close(st1.B_int[l], 0.75 * torch.eye(Bi[l].shape[0], dtype=DT) + 0.25 * Bi[l])
    torch.testing.assert_close(i1.update, 0.25 * i1.direction)       # no momentum at t = 0
    th2, st2, i2 = oracle.kfac_step(th1, p.widths, data, op, hp, st1)
    torch.testing.assert_close(i2.update, 0.25 * (0.5 * i1.update + i2.direction))
    torch.testing.assert_close(th2, th1 + i2.update)


def test_line_search_on_a_quadratic():
    """A single linear layer u = w.x + b has Lap u = 0, so the interior loss is a
    constant and the total loss is exactly quadratic along any direction:
    L(th + a d) = L0 + a g.d + a^2/2 d^T H d with H = (1/M) sum x~ x~^T (x) 1.
    The grid minimiser is then the grid point nearest a* = -g.d / d^T H d."""
    for seed, lam in [(0, 1e-3), (1, 3.0), (2, 40.0), (3, 1e-1)]:
        p, th, data = tiny(widths=(3, 1), seed=seed)
        op = oracle.operator_of(p)
        hp = oracle.HParams(lam=lam, beta=0.0, lr_mode="grid")
        th1, st1, info = oracle.kfac_step(th, p.widths, data, op, hp, oracle.init_state(p.widths, True))
        Xb = data[2]
        Xt = torch.cat([Xb, torch.ones(Xb.shape[0], 1, dtype=DT)], 1)
        H = Xt.T @ Xt / Xb.shape[0]
        dvec = info.direction
        a_star = -(info.gradient @ dvec) / (dvec @ H @ dvec)
        grid = np.array([2.0 ** -k for k in range(31)])
        k_best = int(np.argmin(np.abs(grid - a_star.item())))
        assert info.lr == grid[k_best], (info.lr, a_star)
        # the candidate losses follow the parabola
        L0 = oracle.loss(th, p.widths, *data, op)[0]
        for k, val in enumerate(info.candidate_losses):
            a = 2.0 ** -k
            ref = L0 + a * (info.gradient @ dvec) + 0.5 * a * a * (dvec @ H @ dvec)
            assert abs(val - ref.item()) < 1e-12 * max(1.0, abs(L0))


def test_nonfinite_losses_take_no_step():
    p, th, data = tiny()
    bad = (data[0], data[1].clone(), data[2], data[3])
    bad[1][0] = float("nan")
    st = oracle.init_state(p.widths, True)
    th1, st1, info = oracle.kfac_step(th, p.widths, bad, oracle.operator_of(p),
                                      oracle.HParams(lr_mode="grid"), st)
    assert info.status == 5
    assert torch.equal(th1, th)
    assert st1.step == 0


def test_kfac_descends_on_poisson2d_subset():
    """A few steps on a subset of the 2d Poisson problem decrease the loss."""
    p = synth.poisson2d()
    th = torch.as_tensor(p.theta0())
    xi, yi, xb, yb = (torch.as_tensor(a) for a in p.batch())
    data = (xi[:200], yi[:200], xb[:60], yb[:60])
    widths = [2, 16, 16, 1]
    th = th[:oracle.num_params(widths)].clone()
    op = oracle.operator_of(p)
    hp = oracle.HParams(lam=1e-3, beta=0.886041, momentum=0.707588, lr_mode="grid")
    st = oracle.init_state(widths, True)
    l0 = oracle.loss(th, widths, *data, op)[0]
    for _ in range(5):
        th, st, info = oracle.kfac_step(th, widths, data, op, hp, st)
    assert info.loss_after < 0.5 * l0


@pytest.mark.parametrize("lam", [1e-3, 0.5, 7.0])
def test_damping_closed_forms(lam):
    """Damping adds lambda to each of the four factors (Section 3.4), not to their
    Kronecker sum.  With all four factors zero the damped sum is 2 lambda^2 I, so the
    direction is -g / (2 lambda^2); with scaled identities a_k I, b_k I it is
    (a1+lam)(b1+lam) + (a2+lam)(b2+lam) times I.  Adding lambda to the sum instead
    would give -g / lambda, and damping one term only -g / lambda^2."""
    g = torch.Generator().manual_seed(11)
    V = torch.randn(4, 6, generator=g, dtype=DT)
    Z6, Z4 = torch.zeros(6, 6, dtype=DT), torch.zeros(4, 4, dtype=DT)
    inv = oracle.kron_sum_inverse(oracle.damp(Z6, lam), oracle.damp(Z4, lam),
                                  oracle.damp(Z6, lam), oracle.damp(Z4, lam))
    torch.testing.assert_close(inv.apply(V), V / (2 * lam * lam), rtol=1e-13, atol=0)
    a1, b1, a2, b2 = 0.3, 2.0, 1.5, 0.25
    I6, I4 = torch.eye(6, dtype=DT), torch.eye(4, dtype=DT)
    inv = oracle.kron_sum_inverse(oracle.damp(a1 * I6, lam), oracle.damp(b1 * I4, lam),
                                  oracle.damp(a2 * I6, lam), oracle.damp(b2 * I4, lam))
    c = (a1 + lam) * (b1 + lam) + (a2 + lam) * (b2 + lam)
    torch.testing.assert_close(inv.apply(V), V / c, rtol=1e-13, atol=0)


def zero_output_problem(kind="poisson"):
    """A net whose output layer is zero, with zero targets: u = 0 everywhere, every
    residual and the whole gradient vanish exactly, so Delta = 0 and every
    line-search candidate has the same loss (0)."""
    p = synth.small_problem(kind, (3, 7, 5, 1), 13, 6, n_init=3 if kind == "heat" else 0,
                            problem_id=79)
    th = p.theta0().copy()
    off = synth.layer_offsets(p.widths)
    th[off[-2]:off[-1]] = 0.0
    xi, yi, xb, yb = p.batch()
    return p, th, (xi, 0.0 * yi, xb, 0.0 * yb)


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_line_search_ties_go_to_the_largest_step(kind):
    """Reading G7: scanning from the largest step, the first strict minimum wins.
    With Delta = 0 all 31 candidate losses are equal, so alpha* must be 2^0 (a scan
    that kept the last minimum would return 2^-30)."""
    p, th, data = zero_output_problem(kind)
    op = oracle.operator_of(p)
    hp = oracle.HParams(lam=1e-3, beta=0.0, lr_mode="grid")
    th1, st1, info = oracle.kfac_step(th, p.widths, data, op, hp, oracle.init_state(p.widths, True))
    assert float(info.gradient.abs().max()) == 0.0
    assert len(set(info.candidate_losses)) == 1 and info.candidate_losses[0] == 0.0
    assert info.lr == 1.0 and info.status == 0
