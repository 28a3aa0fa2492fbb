"""Pins for the oracle's weighted second-order operator sum_{i,j} C_ij d2/dx_i dx_j
(Section 3.1, closing paragraph; Appendix C.3): the collapsed row of the forward
pass against a closed form on a sine network and against the input Hessian by
nested autodiff; the special cases C = I (Laplacian) and C = diag(mask); and
the invariance of the Kronecker factors under an orthogonal change of input
coordinates, which the GPU path relies on (it propagates derivatives along the
eigenvectors of C, where the operator is a weighted sum of squares)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.kfac import DT


def sym(d, seed, psd=False):
    g = torch.Generator().manual_seed(seed)
    A = torch.randn(d, d, generator=g, dtype=DT)
    return A @ A.T / d if psd else (A + A.T) / 2


def test_sine_network_closed_form():
    """u = sum_j v_j sin(w_j . x + b_j) has sum_ik C_ik d_i d_k u =
    -sum_j v_j (w_j^T C w_j) sin(w_j . x + b_j)."""
    d, h, n = 4, 5, 7
    g = torch.Generator().manual_seed(1)
    W1 = torch.randn(h, d + 1, generator=g, dtype=DT)
    W2 = torch.randn(1, h + 1, generator=g, dtype=DT)
    X = torch.rand(n, d, generator=g, dtype=DT)
    C = sym(d, 2)
    U = oracle.forward_laplacian([W1, W2], X, C, oracle.Activation("sin")).out
    w, b, v = W1[:, :d], W1[:, d], W2[0, :h]
    quad = torch.einsum("ji,ik,jk->j", w, C, w)
    ref = -(torch.sin(X @ w.T + b) * (v * quad)).sum(1)
    torch.testing.assert_close(U[:, -1], ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("widths", [(3, 6, 5, 1), (4, 7, 1)])
def test_matches_hessian_contraction(widths):
    """tanh net: the collapsed row equals tr(C H_x u) from the input Hessian by
    nested reverse-mode autodiff, point by point."""
    p = synth.small_problem("poisson", widths, 6, 2, problem_id=81)
    Ws = oracle.unpack(torch.as_tensor(p.theta0()), p.widths)
    X = torch.as_tensor(p.batch()[0])
    C = sym(p.d, 3)
    U = oracle.forward_laplacian(Ws, X, C).out

    def net(x):
        z = x
        for l, W in enumerate(Ws):
            z = W[:, :-1] @ z + W[:, -1]
            if l < len(Ws) - 1:
                z = torch.tanh(z)
        return z[0]

    for n in range(X.shape[0]):
        H = torch.autograd.functional.hessian(net, X[n])
        torch.testing.assert_close(U[n, -1], (C * H).sum(), rtol=1e-11, atol=1e-12)


def test_identity_and_mask_special_cases():
    p = synth.small_problem("heat", (4, 6, 5, 1), 9, 3, n_init=2, problem_id=82)
    Ws = oracle.unpack(torch.as_tensor(p.theta0()), p.widths)
    X = torch.as_tensor(p.batch()[0])
    lap = oracle.forward_laplacian(Ws, X, torch.ones(p.d, dtype=DT)).out
    torch.testing.assert_close(oracle.forward_laplacian(Ws, X, torch.eye(p.d, dtype=DT)).out, lap,
                               rtol=1e-14, atol=1e-14)
    m = oracle.operator_of(p).mask_vec(p.d)
    torch.testing.assert_close(oracle.forward_laplacian(Ws, X, torch.diag(m)).out,
                               oracle.forward_laplacian(Ws, X, m).out, rtol=1e-14, atol=1e-14)


def test_factors_invariant_under_orthogonal_coordinates():
    """Write x = Q y with Q orthogonal.  The network W~_1 on x is the network
    [W_1 Q | b_1] on y, the operator C on x is Q^T C Q on y, and the derivative
    rows along y's axes are those along Q's columns.  The loss, every B factor
    and every A factor after the first layer are the same in both coordinates;
    A_1 transforms as Qt^T A_1 Qt with Qt = diag(Q, 1) and the first layer's
    gradient as G_1 Qt.  So propagating along C's eigenvectors, where Q^T C Q is
    diagonal, yields the factors of the paper's coordinate directions."""
    p = synth.small_problem("poisson", (3, 6, 5, 1), 11, 4, problem_id=83)
    th = torch.as_tensor(p.theta0())
    Xi, yi, Xb, yb = (torch.as_tensor(a) for a in p.batch())
    C = sym(p.d, 4)
    evals, Q = torch.linalg.eigh(C)
    op_x = oracle.Operator(coef=tuple(map(tuple, C.tolist())))
    op_y = oracle.Operator(coef=tuple(map(tuple, (Q.T @ C @ Q).tolist())))
    Ws = oracle.unpack(th, p.widths)
    Qt = torch.block_diag(Q, torch.ones(1, 1, dtype=DT))
    Wy = [Ws[0] @ Qt] + Ws[1:]
    thy = oracle.pack(Wy)
    fx = oracle.interior_factors(oracle.interior_curvature_inputs(Ws, Xi, yi, op_x))
    fy = oracle.interior_factors(oracle.interior_curvature_inputs(Wy, Xi @ Q, yi, op_y))
    torch.testing.assert_close(fy[0][0], Qt.T @ fx[0][0] @ Qt, rtol=1e-12, atol=1e-13)
    for l in range(1, len(Ws)):
        torch.testing.assert_close(fy[0][l], fx[0][l], rtol=1e-12, atol=1e-13)
    for l in range(len(Ws)):
        torch.testing.assert_close(fy[1][l], fx[1][l], rtol=1e-12, atol=1e-13)
    gx, lx, _ = oracle.loss_gradient(th, p.widths, Xi, yi, Xb, yb, op_x)
    gy, ly, _ = oracle.loss_gradient(thy, p.widths, Xi @ Q, yi, Xb @ Q, yb, op_y)
    assert abs(lx - ly) <= 1e-13 * abs(lx)
    Gx, Gy = oracle.unpack(gx, p.widths), oracle.unpack(gy, p.widths)
    torch.testing.assert_close(Gy[0], Gx[0] @ Qt, rtol=1e-12, atol=1e-13)
    for l in range(1, len(Ws)):
        torch.testing.assert_close(Gy[l], Gx[l], rtol=1e-12, atol=1e-13)
