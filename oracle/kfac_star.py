"""FP64 CPU oracle for KFAC*: the automatic learning rate and momentum of the
original KFAC optimizer applied to the KFAC-PINN direction.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports it.

Dangel, Mueller & Zeinhofer (NeurIPS 2024), Section 3.4, paragraph "Learning rate
and momentum": the update is delta(alpha, mu) = alpha Delta_t + mu delta_{t-1},
with (alpha, mu) minimising the quadratic model
    m(delta) = L(theta_t) + delta^T g_t + 1/2 delta^T (G(theta_t) + lambda I) delta
built with the exact Gramian G (Eq. gramian, Lambda = I), so that
    (alpha, mu) = -Q^-1 (Delta^T g, delta^T g),   Q_ij = d_i^T (G + lambda I) d_j,
for d_1 = Delta_t, d_2 = delta_{t-1}.  The Gramian enters only through the
products G d_i, which the paper computes with one Jacobian-vector product each
(the outer-product structure G = J^T J / N + J_b^T J_b / M); so does this oracle,
with forward-mode autodiff of the residual vectors.

Readings (listed in the design notes): the bottom-right entry of the printed
2 x 2 matrix is taken as delta^T G delta + lambda |delta|^2 (the matrix is the
Hessian of m in (alpha, mu), so it is symmetric with entries d_i^T (G + lambda I) d_j);
at the first step there is no previous update, so mu = 0 and alpha minimises m
along Delta alone.
"""
from __future__ import annotations

import math
from typing import Sequence

import torch

from .kfac import (DT, TANH, HParams, State, StepInfo, _t, boundary_curvature_inputs,
                   boundary_factors, boundary_residual, damp, ema, forward_laplacian,
                   forward_plain, interior_curvature_inputs, interior_factors,
                   interior_residual, kron_sum_inverse, loss, loss_gradient, pack, unpack)


def residual_vectors(theta, widths, Xi, yi, Xb, yb, op, act=TANH):
    """(r, r_b): interior residuals L u(x_n) - y_n and boundary residuals u - g
    (Section 2.1) as functions of theta."""
    Ws = unpack(theta, widths)
    fi = forward_laplacian(Ws, Xi, op.second_order(Xi.shape[1]), act)
    fb = forward_plain(Ws, Xb, act)
    return interior_residual(fi.out, yi, op, Xi), boundary_residual(fb.out, yb)


def jacobian_vector_products(theta, widths, data, op, d, act=TANH):
    """(J d, J_b d): the residuals' directional derivatives along d, by forward-mode
    autodiff (one JVP per direction, as the paper does)."""
    th = _t(theta).detach()
    Xi, yi, Xb, yb = map(_t, data)
    f = lambda t: residual_vectors(t, widths, Xi, yi, Xb, yb, op, act)
    _, (ji, jb) = torch.func.jvp(f, (th,), (_t(d).detach(),))
    return ji, jb


def gramian_forms(theta, widths, data, op, dirs: Sequence, act=TANH) -> torch.Tensor:
    """Q_ij = d_i^T G(theta) d_j with G = J^T J / N + J_b^T J_b / M, the Gramian of
    L = |r|^2/(2N) + |r_b|^2/(2M) (Eq. gramian with the boundary term)."""
    N, M = _t(data[0]).shape[0], _t(data[2]).shape[0]
    jv = [jacobian_vector_products(theta, widths, data, op, d, act) for d in dirs]
    Q = torch.empty(len(dirs), len(dirs), dtype=DT)
    for i in range(len(dirs)):
        for j in range(len(dirs)):
            Q[i, j] = (jv[i][0] @ jv[j][0]) / N + (jv[i][1] @ jv[j][1]) / M
    return Q


def kfac_star_coefficients(theta, widths, data, op, Delta, delta_prev, grad, lam, first: bool,
                           act=TANH):
    """(alpha*, mu*, Q, b) of the quadratic model (Section 3.4).  Q is the 2 x 2 (or,
    at the first step, 1 x 1) matrix d_i^T (G + lambda I) d_j and b_i = d_i^T g."""
    dirs = [Delta] if first else [Delta, delta_prev]
    Q = gramian_forms(theta, widths, data, op, dirs, act)
    D = torch.stack([_t(d) for d in dirs])
    Q = Q + lam * (D @ D.T)
    b = D @ _t(grad)
    if first:
        return float(-b[0] / Q[0, 0]), 0.0, Q, b
    sol = -torch.linalg.solve(Q, b)
    return float(sol[0]), float(sol[1]), Q, b


def kfac_star_step(theta, widths, data, op, hp: HParams, state: State, act=TANH):
    """One KFAC* iteration: the factors, EMA, damping and preconditioned gradient
    Delta_t exactly as in a KFAC step (Algorithm 1, steps 1-4), then
    delta_t = alpha* Delta_t + mu* delta_{t-1} and theta += delta_t.  Returns
    (theta_next, state_next, info); info.lr holds alpha*, and the returned state's
    delta is the applied update.  A non-finite loss, alpha* or mu* takes no step
    (status 5)."""
    theta = _t(theta).clone()
    Xi, yi, Xb, yb = map(_t, data)
    Ws = unpack(theta, widths)
    ci = interior_curvature_inputs(Ws, Xi, yi, op, act)
    Ai, Bi = interior_factors(ci)
    cb = boundary_curvature_inputs(Ws, Xb, yb, act)
    Ab, Bb = boundary_factors(cb)
    A_int = [ema(p, n, hp.beta) for p, n in zip(state.A_int, Ai)]
    B_int = [ema(p, n, hp.beta) for p, n in zip(state.B_int, Bi)]
    A_bnd = [ema(p, n, hp.beta) for p, n in zip(state.A_bnd, Ab)]
    B_bnd = [ema(p, n, hp.beta) for p, n in zip(state.B_bnd, Bb)]
    inv = [kron_sum_inverse(damp(A_int[l], hp.lam), damp(B_int[l], hp.lam),
                            damp(A_bnd[l], hp.lam), damp(B_bnd[l], hp.lam))
           for l in range(len(Ws))]
    grad, li, lb = loss_gradient(theta, widths, Xi, yi, Xb, yb, op, act)
    gW = unpack(grad, widths)
    Delta = pack([-inv[l].apply(gW[l]) for l in range(len(Ws))])
    first = state.step == 0
    alpha, mu, Q, b = kfac_star_coefficients(theta, widths, (Xi, yi, Xb, yb), op, Delta,
                                             state.delta, grad, hp.lam, first, act)
    status = 0
    if not (math.isfinite(li + lb) and math.isfinite(alpha) and math.isfinite(mu)):
        status, alpha, mu = 5, 0.0, 0.0
    if status == 0:
        delta = alpha * Delta + mu * state.delta
        theta_next = theta + delta
    else:
        delta, theta_next = state.delta.clone(), theta.clone()
    after = loss(theta_next, widths, Xi, yi, Xb, yb, op, act)[0]
    new_state = State(A_int, B_int, A_bnd, B_bnd, delta, state.step + (1 if status == 0 else 0))
    info = StepInfo(li, lb, alpha, after, None, Delta, delta, grad, status)
    info.momentum = mu
    info.model = (Q, b)
    return theta_next, new_state, info
