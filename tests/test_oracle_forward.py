"""Pins for the oracle's forward Laplacian (Section 3.1, Eq. forward-laplacian-main).

Each test checks the oracle against something other than itself: closed-form
Laplacians of manufactured solutions represented exactly by sin/cos networks,
a single-neuron closed form, two independent routes (per-direction Taylor mode and
nested autodiff), central finite differences, and the identity-activation case."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle.kfac import Activation, DT, forward_laplacian, laplacian_autodiff, laplacian_taylor_naive

SIN, COS, IDENT = Activation("sin"), Activation("cos"), Activation("identity")


def rand_net(widths, seed):
    g = torch.Generator().manual_seed(seed)
    return [torch.randn(widths[l + 1], widths[l] + 1, generator=g, dtype=DT) / math.sqrt(widths[l])
            for l in range(len(widths) - 1)]


def test_sum_of_sines_closed_form():
    """u* = sum_i sin(pi x_i) is the sin network 1^T sin(pi I x): its value, gradient
    and Laplacian are sum sin, pi cos(pi x_i) and -pi^2 sum sin (the 5d and 100d
    Poisson manufactured solutions, Appendix A)."""
    for d in (2, 5, 17):
        W1 = torch.cat([math.pi * torch.eye(d, dtype=DT), torch.zeros(d, 1, dtype=DT)], 1)
        W2 = torch.cat([torch.ones(1, d, dtype=DT), torch.zeros(1, 1, dtype=DT)], 1)
        X = torch.rand(11, d, dtype=DT, generator=torch.Generator().manual_seed(d))
        U = forward_laplacian([W1, W2], X, torch.ones(d, dtype=DT), SIN).out
        s = torch.sin(math.pi * X)
        torch.testing.assert_close(U[:, 0], s.sum(1), rtol=0, atol=1e-13)
        torch.testing.assert_close(U[:, 1:d + 1], math.pi * torch.cos(math.pi * X), rtol=0, atol=1e-13)
        torch.testing.assert_close(U[:, -1], -math.pi ** 2 * s.sum(1), rtol=0, atol=1e-12)
        # partial Laplacian over coordinates 1..d-1 (the heat equation's spatial part)
        mask = torch.ones(d, dtype=DT); mask[0] = 0
        U = forward_laplacian([W1, W2], X, mask, SIN).out
        torch.testing.assert_close(U[:, -1], -math.pi ** 2 * s[:, 1:].sum(1), rtol=0, atol=1e-12)


def test_product_of_sines_closed_form():
    """sin(pi x) sin(pi y) = (cos(pi(x-y)) - cos(pi(x+y)))/2, a cos network; its
    Laplacian is -2 pi^2 sin(pi x) sin(pi y) = -f of the 2d Poisson problem (Eq. 2D-Poisson)."""
    W1 = torch.tensor([[math.pi, -math.pi, 0.0], [math.pi, math.pi, 0.0]], dtype=DT)
    W2 = torch.tensor([[0.5, -0.5, 0.0]], dtype=DT)
    X = torch.rand(13, 2, dtype=DT, generator=torch.Generator().manual_seed(3))
    U = forward_laplacian([W1, W2], X, torch.ones(2, dtype=DT), COS).out
    ss = torch.sin(math.pi * X[:, 0]) * torch.sin(math.pi * X[:, 1])
    torch.testing.assert_close(U[:, 0], ss, rtol=0, atol=1e-14)
    torch.testing.assert_close(U[:, -1], -2 * math.pi ** 2 * ss, rtol=0, atol=1e-12)


def test_single_tanh_neuron_closed_form():
    """Lap [v tanh(w.x + b)] = v |w|^2 tanh''(w.x + b)."""
    g = torch.Generator().manual_seed(5)
    d = 4
    w = torch.randn(d, dtype=DT, generator=g); b = 0.3; v = -1.7
    W1 = torch.cat([w, torch.tensor([b], dtype=DT)])[None, :]
    W2 = torch.tensor([[v, 0.0]], dtype=DT)
    X = torch.rand(9, d, dtype=DT, generator=g)
    U = forward_laplacian([W1, W2], X, torch.ones(d, dtype=DT)).out
    t = torch.tanh(X @ w + b)
    torch.testing.assert_close(U[:, -1], v * (w @ w) * (-2 * t * (1 - t * t)), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("widths", [[3, 5, 4, 1], [2, 8, 8, 6, 1], [6, 7, 1]])
def test_three_routes_and_fd(widths):
    """Forward Laplacian == per-direction Taylor mode == nested autodiff == central FD."""
    Ws = rand_net(widths, sum(widths))
    d = widths[0]
    X = torch.rand(10, d, dtype=DT, generator=torch.Generator().manual_seed(1))
    fl = forward_laplacian(Ws, X, torch.ones(d, dtype=DT)).out
    tn = laplacian_taylor_naive(Ws, X)
    ad = laplacian_autodiff(Ws, X)
    torch.testing.assert_close(fl[:, -1], tn, rtol=1e-12, atol=1e-12)
    torch.testing.assert_close(fl[:, -1], ad, rtol=1e-12, atol=1e-12)

    def u(x):
        z = x
        for l, W in enumerate(Ws):
            z = z @ W[:, :-1].T + W[:, -1]
            if l < len(Ws) - 1:
                z = torch.tanh(z)
        return z[:, 0]

    h = 1e-3
    fd = torch.zeros(X.shape[0], dtype=DT)
    for i in range(d):
        e = torch.zeros(d, dtype=DT); e[i] = h
        fd += (u(X + e) - 2 * u(X) + u(X - e)) / h ** 2
        gi = (u(X + e) - u(X - e)) / (2 * h)
        torch.testing.assert_close(fl[:, 1 + i], gi, rtol=1e-5, atol=1e-6)
    torch.testing.assert_close(fl[:, -1], fd, rtol=1e-5, atol=1e-5)
    torch.testing.assert_close(fl[:, 0], u(X), rtol=1e-14, atol=1e-14)


def test_identity_activation_has_zero_laplacian():
    Ws = rand_net([4, 6, 5, 1], 9)
    X = torch.rand(8, 4, dtype=DT)
    U = forward_laplacian(Ws, X, torch.ones(4, dtype=DT), IDENT).out
    assert U[:, -1].abs().max() == 0.0
    # the gradient rows are the product of the weight matrices
    Wp = Ws[0][:, :-1]
    for W in Ws[1:]:
        Wp = W[:, :-1] @ Wp
    torch.testing.assert_close(U[:, 1:5], Wp.expand(8, 4), rtol=1e-13, atol=1e-14)


def test_heat_operator_matches_fd():
    """r = d_t u - kappa Lap_x u - y (Appendix A, heat): the residual built from the
    output rows equals finite differences of the network."""
    Ws = rand_net([5, 6, 6, 1], 21)
    X = torch.rand(7, 5, dtype=DT, generator=torch.Generator().manual_seed(2))
    op = oracle.Operator(0, 1.0, -0.25, (0, 1, 1, 1, 1))
    U = forward_laplacian(Ws, X, op.mask_vec(5)).out
    y = torch.rand(7, dtype=DT)
    r = oracle.interior_residual(U, y, op)

    def u(x):
        z = x
        for l, W in enumerate(Ws):
            z = z @ W[:, :-1].T + W[:, -1]
            if l < len(Ws) - 1:
                z = torch.tanh(z)
        return z[:, 0]

    h = 1e-3
    e0 = torch.zeros(5, dtype=DT); e0[0] = h
    ut = (u(X + e0) - u(X - e0)) / (2 * h)
    lap = sum((u(X + e) - 2 * u(X) + u(X - e)) / h ** 2
              for e in [torch.eye(5, dtype=DT)[i] * h for i in range(1, 5)])
    torch.testing.assert_close(r, ut - 0.25 * lap - y, rtol=1e-5, atol=1e-6)
