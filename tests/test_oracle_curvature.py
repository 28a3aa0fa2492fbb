"""Pins for the oracle's output gradients, factors, gradient and Kronecker-sum
inverse (Section 3.2, Eqs. laplace_gramian_block_exact and KFAC-PINN; Section 3.4).

References: central finite differences of the residuals and of the loss, the exact
Gramian block identity built from finite-difference Jacobians, closed forms of
the first- and last-layer factors, exactness of the boundary factors for one point,
invariance under replication of the point set, and a dense Kronecker solve."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.kfac import DT

OPS = {"poisson": oracle.POISSON_OP, "heat": oracle.Operator(0, 1.0, -0.25, (0, 1, 1)),
       # a residual with first-order terms (Section 3.3): the log-Fokker-Planck form
       "logfp": oracle.Operator(0, 1.0, -1.0, (0, 1, 1), None, -0.5, -1.0, -1.0)}


def setup(widths=(3, 4, 3, 1), n=5, m=4, seed=0):
    g = np.random.default_rng(seed)
    th = torch.as_tensor(g.uniform(-1, 1, oracle.num_params(widths)))
    Xi = torch.as_tensor(g.uniform(0, 1, (n, widths[0])))
    Xb = torch.as_tensor(g.uniform(0, 1, (m, widths[0])))
    yi = torch.as_tensor(g.normal(size=n))
    yb = torch.as_tensor(g.normal(size=m))
    return list(widths), th, Xi, yi, Xb, yb


def residuals(th, widths, Xi, yi, Xb, yb, op):
    Ws = oracle.unpack(th, widths)
    fi = oracle.forward_laplacian(Ws, Xi, op.mask_vec(Xi.shape[1]))
    fb = oracle.forward_plain(Ws, Xb)
    return oracle.interior_residual(fi.out, yi, op, Xi), oracle.boundary_residual(fb.out, yb)


def fd_jacobian(fun, th, sl, h=1e-5):
    """Central-difference Jacobian of fun(theta) (vector) w.r.t. theta[sl]."""
    cols = []
    for j in range(sl.start, sl.stop):
        e = torch.zeros_like(th); e[j] = h
        cols.append((fun(th + e) - fun(th - e)) / (2 * h))
    return torch.stack(cols, 1)


@pytest.mark.parametrize("kind", ["poisson", "heat", "logfp"])
def test_per_point_jacobian_identity(kind):
    """J_{W^(l)} r_n = sum_s Z~_{n,s}^T (x) g_{n,s} (Section 3.2): with column
    stacking its entry (j, i) is sum_s Z~_{n,s,j} g_{n,s,i}.  Checked against FD."""
    op = OPS[kind]
    widths, th, Xi, yi, Xb, yb = setup()
    Ws = oracle.unpack(th, widths)
    ci = oracle.interior_curvature_inputs(Ws, Xi, yi, op)
    cb = oracle.boundary_curvature_inputs(Ws, Xb, yb)
    off = np.cumsum([0] + [widths[l + 1] * (widths[l] + 1) for l in range(len(widths) - 1)])
    for l in range(len(widths) - 1):
        sl = slice(int(off[l]), int(off[l + 1]))
        Ji = fd_jacobian(lambda t: residuals(t, widths, Xi, yi, Xb, yb, op)[0], th, sl)
        Jb = fd_jacobian(lambda t: residuals(t, widths, Xi, yi, Xb, yb, op)[1], th, sl)
        Ki = torch.einsum("nsj,nsi->nji", ci.zin[l], ci.g[l]).reshape(Xi.shape[0], -1)
        Kb = torch.einsum("nj,ni->nji", cb.zin[l], cb.g[l]).reshape(Xb.shape[0], -1)
        torch.testing.assert_close(Ki, Ji, rtol=1e-7, atol=1e-8)
        torch.testing.assert_close(Kb, Jb, rtol=1e-7, atol=1e-8)
        # exact Gramian block (Eq. laplace_gramian_block_exact) from the same pieces
        G_exact = torch.einsum("nsj,nsi,ntk,ntm->jikm", ci.zin[l], ci.g[l], ci.zin[l], ci.g[l])
        G_exact = G_exact.reshape(Ki.shape[1], Ki.shape[1]) / Xi.shape[0]
        torch.testing.assert_close(G_exact, Ji.T @ Ji / Xi.shape[0], rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("kind", ["poisson", "heat", "logfp"])
def test_gradient_matches_fd(kind):
    op = OPS[kind]
    widths, th, Xi, yi, Xb, yb = setup(seed=3)
    grad, li, lb = oracle.loss_gradient(th, widths, Xi, yi, Xb, yb, op)
    fd = fd_jacobian(lambda t: torch.tensor([oracle.loss(t, widths, Xi, yi, Xb, yb, op)[0]], dtype=DT),
                     th, slice(0, th.numel()), h=1e-6)[0]
    torch.testing.assert_close(grad, fd, rtol=1e-6, atol=1e-8)
    # the gradient is also  sum_{n,s} (r_n/N) g Z~^T + sum_n (rb_n/M) g z~^T  (Algorithm 1)
    Ws = oracle.unpack(th, widths)
    ci = oracle.interior_curvature_inputs(Ws, Xi, yi, op)
    cb = oracle.boundary_curvature_inputs(Ws, Xb, yb)
    mats = [torch.einsum("n,nsi,nsj->ij", ci.r / Xi.shape[0], ci.g[l], ci.zin[l])
            + torch.einsum("n,ni,nj->ij", cb.r / Xb.shape[0], cb.g[l], cb.zin[l])
            for l in range(len(Ws))]
    torch.testing.assert_close(oracle.pack(mats), grad, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_factor_closed_forms(kind):
    op = OPS[kind]
    widths, th, Xi, yi, Xb, yb = setup(widths=(3, 6, 5, 1), n=9, m=7, seed=4)
    N, d = Xi.shape
    S = d + 2
    Ws = oracle.unpack(th, widths)
    Ai, Bi = oracle.interior_factors(oracle.interior_curvature_inputs(Ws, Xi, yi, op))
    Ab, Bb = oracle.boundary_factors(oracle.boundary_curvature_inputs(Ws, Xb, yb))
    Xt = torch.cat([Xi, torch.ones(N, 1, dtype=DT)], 1)
    E = torch.diag(torch.cat([torch.ones(d, dtype=DT), torch.zeros(1, dtype=DT)]))
    torch.testing.assert_close(Ai[0], (Xt.T @ Xt + N * E) / (N * S), rtol=1e-14, atol=1e-15)
    Xbt = torch.cat([Xb, torch.ones(Xb.shape[0], 1, dtype=DT)], 1)
    torch.testing.assert_close(Ab[0], Xbt.T @ Xbt / Xb.shape[0], rtol=1e-14, atol=1e-15)
    # last layer: g is the residual's seed, so B = c_t^2 + c_lap^2 and B_bnd = 1
    ct = op.coef_time if op.time_coord >= 0 else 0.0
    assert abs(Bi[-1].item() - (ct ** 2 + op.coef_lap ** 2)) < 1e-14
    assert abs(Bb[-1].item() - 1.0) < 1e-14
    for M in Ai + Bi + Ab + Bb:
        assert torch.equal(M, M.T) or torch.allclose(M, M.T, rtol=0, atol=1e-15)
        ev = torch.linalg.eigvalsh(M)
        assert ev.min() >= -1e-12 * max(ev.abs().max().item(), 1e-300)
    # trace of A_Omega = |Z~|_F^2 / (N S)
    ci = oracle.interior_curvature_inputs(Ws, Xi, yi, op)
    for l in range(len(Ws)):
        torch.testing.assert_close(torch.trace(Ai[l]), (ci.zin[l] ** 2).sum() / (N * S))


def test_boundary_factor_exact_for_one_point():
    """With one boundary point the expectation approximation is exact: A (x) B equals
    the Gauss-Newton block J^T J built from FD Jacobians (Eq. kfac-linear)."""
    widths, th, Xi, yi, Xb, yb = setup(widths=(2, 3, 3, 1), m=1, seed=5)
    op = oracle.POISSON_OP
    Ws = oracle.unpack(th, widths)
    Ab, Bb = oracle.boundary_factors(oracle.boundary_curvature_inputs(Ws, Xb, yb))
    off = np.cumsum([0] + [widths[l + 1] * (widths[l] + 1) for l in range(len(widths) - 1)])
    for l in range(len(Ws)):
        J = fd_jacobian(lambda t: residuals(t, widths, Xi, yi, Xb, yb, op)[1], th,
                        slice(int(off[l]), int(off[l + 1])))
        torch.testing.assert_close(torch.kron(Ab[l], Bb[l]), J.T @ J, rtol=1e-7, atol=1e-9)


def test_replication_invariance():
    widths, th, Xi, yi, Xb, yb = setup(seed=6)
    op = OPS["heat"]
    Ws = oracle.unpack(th, widths)
    r3 = lambda t: torch.cat([t, t, t], 0)
    A1, B1 = oracle.interior_factors(oracle.interior_curvature_inputs(Ws, Xi, yi, op))
    A3, B3 = oracle.interior_factors(oracle.interior_curvature_inputs(Ws, r3(Xi), r3(yi), op))
    for a, b in zip(A1 + B1, A3 + B3):
        torch.testing.assert_close(a, b, rtol=1e-13, atol=1e-15)
    g1 = oracle.loss_gradient(th, widths, Xi, yi, Xb, yb, op)[0]
    g3 = oracle.loss_gradient(th, widths, r3(Xi), r3(yi), r3(Xb), r3(yb), op)[0]
    torch.testing.assert_close(g1, g3, rtol=1e-13, atol=1e-15)


def spd(n, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    X = torch.randn(n, n + 3, generator=g, dtype=DT)
    return scale * X @ X.T / n + 1e-3 * torch.eye(n, dtype=DT)


@pytest.mark.parametrize("na,nb", [(4, 3), (7, 5), (1, 6), (6, 1)])
def test_kron_sum_inverse_matches_dense(na, nb):
    A1, A2 = spd(na, 1), spd(na, 2, 0.3)
    B1, B2 = spd(nb, 3), spd(nb, 4, 2.0)
    V = torch.randn(nb, na, dtype=DT, generator=torch.Generator().manual_seed(9))
    X = oracle.kron_sum_inverse(A1, B1, A2, B2).apply(V)
    Xd = oracle.kron_sum_solve_dense(A1, B1, A2, B2, V)
    torch.testing.assert_close(X, Xd, rtol=1e-10, atol=1e-12)
    res = B1 @ X @ A1 + B2 @ X @ A2 - V
    assert res.norm() / V.norm() < 1e-12
    if nb == 1:   # B scalars: one SPD solve with b1 A1 + b2 A2
        Xs = torch.linalg.solve(B1.item() * A1 + B2.item() * A2, V[0])
        torch.testing.assert_close(X[0], Xs, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("widths,D", [([2, 64, 1], 257), ([2, 64, 64, 48, 48, 1], 9873),
                                      ([2, 256, 256, 128, 128, 1], 116097), ([5, 64, 1], 449),
                                      ([5, 64, 64, 48, 48, 1], 10065),
                                      ([5, 256, 256, 128, 128, 1], 116865),
                                      ([10, 256, 256, 128, 128, 1], 118145),
                                      ([100, 768, 768, 512, 512, 1], 1325057)])
def test_parameter_counts_printed_in_paper(widths, D):
    """Parameter dimensions printed in Appendix A pin the bias-inclusive layout."""
    assert oracle.num_params(widths) == D == synth.num_params(widths)
    th = torch.arange(D, dtype=DT)
    torch.testing.assert_close(oracle.pack(oracle.unpack(th, widths)), th)


def test_chunked_factor_assembly_equals_direct():
    """The test helper that assembles the oracle's factors over chunks of points
    (used at full workload sizes) reproduces the direct computation."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from helpers import oracle_curvature, oracle_factors_chunked, oracle_forward_chunked
    p = synth.small_problem("heat", (3, 9, 7, 1), 53, 17, n_init=5, problem_id=91)
    th = p.theta0()
    xi, yi, xb, yb = p.batch()
    direct = oracle_curvature(p, th, xi, yi, xb, yb)
    chunked = oracle_factors_chunked(p, th, xi, yi, xb, yb, chunk=10)
    for k in ("A_int", "B_int", "A_bnd", "B_bnd"):
        for a, b in zip(chunked[k], direct[k]):
            torch.testing.assert_close(a, b, rtol=1e-13, atol=1e-15)
    U = oracle.forward_laplacian(oracle.unpack(torch.as_tensor(th), p.widths), torch.as_tensor(xi),
                                 oracle.operator_of(p).mask_vec(p.d)).out
    torch.testing.assert_close(oracle_forward_chunked(p, th, xi, chunk=8), U, rtol=1e-14, atol=0)
