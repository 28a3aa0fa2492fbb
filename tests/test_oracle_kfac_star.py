"""Pins for the KFAC* oracle (Section 3.4, automatic learning rate and momentum):
the Gramian quadratic forms against a dense Gramian assembled from a full
reverse-mode Jacobian; the per-point Jacobian-vector product against the
contraction of the layer slabs (the identity the GPU path evaluates); and, on a
loss that is exactly quadratic in theta, the property that defines the step:
theta + alpha* Delta + mu* delta_{t-1} minimises the loss over that plane."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import kfac_star as ks
from oracle.kfac import DT


def tiny(kind="poisson", widths=(2, 5, 4, 1), n=9, m=7, pid=61):
    p = synth.small_problem(kind, widths, n, m, n_init=3 if kind == "heat" else 0, problem_id=pid)
    data = tuple(torch.as_tensor(a) for a in p.batch())
    return p, torch.as_tensor(p.theta0()), data


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_gramian_forms_match_dense_gramian(kind):
    p, th, data = tiny(kind, widths=(2, 4, 3, 1) if kind == "poisson" else (3, 4, 3, 1))
    op = oracle.operator_of(p)
    f = lambda t: torch.cat(ks.residual_vectors(t, p.widths, *data, op))
    J = torch.autograd.functional.jacobian(f, th)            # (N + M) x D, reverse mode
    N, M = data[0].shape[0], data[2].shape[0]
    w = torch.cat([torch.full((N,), 1.0 / N, dtype=DT), torch.full((M,), 1.0 / M, dtype=DT)])
    G = J.T @ (w[:, None] * J)
    g = torch.Generator().manual_seed(4)
    dirs = [torch.randn(th.numel(), generator=g, dtype=DT) for _ in range(2)]
    Q = ks.gramian_forms(th, p.widths, data, op, dirs)
    D = torch.stack(dirs)
    torch.testing.assert_close(Q, D @ G @ D.T, rtol=1e-12, atol=1e-14)
    # G is the Hessian of the loss when the residuals are linear in theta:
    # here it is only positive semi-definite
    assert float(torch.linalg.eigvalsh(G).min()) > -1e-10 * float(G.abs().max())


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_jvp_equals_slab_contraction(kind):
    """J_n d = sum_l sum_s g^(l)_{n,s}^T D^(l) z~^(l-1)_{n,s}: the residual's
    directional derivative is the layer slabs contracted with the direction's
    blocks (chain rule through W~ Z~, Section 3.2), for the interior and the
    boundary residuals."""
    p, th, data = tiny(kind, widths=(3, 6, 5, 1))
    op = oracle.operator_of(p)
    g = torch.Generator().manual_seed(5)
    d = torch.randn(th.numel(), generator=g, dtype=DT)
    ji, jb = ks.jacobian_vector_products(th, p.widths, data, op, d)
    Ws = oracle.unpack(th, p.widths)
    Ds = oracle.unpack(d, p.widths)
    ci = oracle.interior_curvature_inputs(Ws, data[0], data[1], op)
    cb = oracle.boundary_curvature_inputs(Ws, data[2], data[3])
    slab_i = sum(torch.einsum("nsj,jk,nsk->n", ci.g[l], Ds[l], ci.zin[l]) for l in range(len(Ws)))
    slab_b = sum(torch.einsum("nj,jk,nk->n", cb.g[l], Ds[l], cb.zin[l]) for l in range(len(Ws)))
    torch.testing.assert_close(ji, slab_i, rtol=1e-12, atol=1e-13)
    torch.testing.assert_close(jb, slab_b, rtol=1e-12, atol=1e-13)


def test_step_minimises_an_exactly_quadratic_loss_over_its_plane():
    """One linear layer u = w.x + b: Lap u = 0, so the interior loss does not
    depend on theta, the boundary residual is linear in theta and the loss is
    exactly quadratic with Hessian G.  With lambda = 0 the model m is the loss
    itself, so the first step's theta_1 minimises L along Delta_0, and the second
    step's theta_2 minimises L over the plane theta_1 + span(Delta_1, delta_0):
    the gradient at the new point is orthogonal to the directions, and nearby
    points of the plane are not lower."""
    p, th, data = tiny(widths=(3, 1), n=8, m=11, pid=62)
    op = oracle.operator_of(p)
    hp = oracle.HParams(lam=0.0, beta=0.5)
    st = oracle.init_state(p.widths, True)
    th1, st1, i1 = ks.kfac_star_step(th, p.widths, data, op, hp, st)
    assert i1.momentum == 0.0 and i1.status == 0
    g1 = oracle.loss_gradient(th1, p.widths, *data, op)[0]
    assert abs(float(g1 @ i1.direction)) < 1e-12 * float(g1.norm() * i1.direction.norm() + 1e-30) + 1e-14
    th2, st2, i2 = ks.kfac_star_step(th1, p.widths, data, op, hp, st1)
    assert i2.status == 0 and i2.momentum != 0.0
    g2 = oracle.loss_gradient(th2, p.widths, *data, op)[0]
    for dvec in (i2.direction, st1.delta):
        assert abs(float(g2 @ dvec)) < 1e-10 * float(dvec.norm())
    L2 = oracle.loss(th2, p.widths, *data, op)[0]
    for a in (-1e-3, 1e-3):
        for b in (-1e-3, 0.0, 1e-3):
            Lp = oracle.loss(th2 + a * i2.direction + b * st1.delta, p.widths, *data, op)[0]
            assert Lp >= L2 - 1e-15


def test_coefficients_solve_the_two_by_two_model():
    """(alpha*, mu*) is the stationary point of the quadratic model: Q (alpha, mu)
    + b = 0, with Q symmetric positive definite (the bottom-right entry is
    delta^T (G + lambda I) delta), and the model decreases from 0."""
    p, th, data = tiny("heat", widths=(3, 6, 5, 1), pid=63)
    op = oracle.operator_of(p)
    hp = oracle.HParams(lam=1e-3, beta=0.886041)
    st = oracle.init_state(p.widths, True)
    th1, st1, _ = ks.kfac_star_step(th, p.widths, data, op, hp, st)
    _, _, info = ks.kfac_star_step(th1, p.widths, data, op, hp, st1)
    Q, b = info.model
    x = torch.tensor([info.lr, info.momentum], dtype=DT)
    torch.testing.assert_close(Q @ x + b, torch.zeros(2, dtype=DT), rtol=0, atol=1e-12 * float(b.abs().max()))
    torch.testing.assert_close(Q, Q.T)
    assert float(torch.linalg.eigvalsh(Q).min()) > 0
    assert float(0.5 * x @ Q @ x + b @ x) < 0
    # the model's Gramian entries agree with a direct recomputation along the
    # applied update
    d = info.update
    q = ks.gramian_forms(th1, p.widths, data, op, [d])[0, 0] + hp.lam * float(d @ d)
    torch.testing.assert_close(q, x @ Q @ x, rtol=1e-10, atol=0)
