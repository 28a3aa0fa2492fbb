"""Pins for the oracle's residual with first-order terms (Section 3.3; the
logarithmic Fokker-Planck equation of Section 4 and Appendix A):
r = d_t q - d_x/2 - (1/2) x . grad_x q - |grad_x q|^2 - Lap_x q.  Its
manufactured solution q* = log N(0, (2 - e^-t) I) makes the residual vanish when
the oracle's residual is fed q*'s exact derivatives, which pins the signs and
coefficients of every term; the output-gradient seeds are pinned by the central
differences of test_oracle_curvature (kind logfp)."""
import math

import numpy as np
import torch

import oracle
import synth
from oracle.kfac import DT


def exact_rows(x):
    """Rows (value, d_t, d_x1..d_xk, Lap_x) of q* at the points x = (t, x_1..x_k)."""
    t, y = x[:, 0], x[:, 1:]
    k = y.shape[1]
    s2 = 2.0 - torch.exp(-t)
    ds2 = torch.exp(-t)
    r2 = (y * y).sum(1)
    q = -0.5 * k * torch.log(2 * math.pi * s2) - r2 / (2 * s2)
    qt = -0.5 * k * ds2 / s2 + r2 * ds2 / (2 * s2 * s2)
    qx = -y / s2[:, None]
    lap = -k / s2
    return torch.cat([q[:, None], qt[:, None], qx, lap[:, None]], 1)


def test_manufactured_solution_solves_the_residual():
    p = synth.log_fokker_planck(n_int=400, n_init=10)
    xi, yi, xb, yb = p.batch()
    X = torch.as_tensor(xi)
    U = exact_rows(X)
    op = oracle.operator_of(p)
    assert (op.coef_time, op.coef_lap, op.coef_xgrad, op.coef_gradsq, op.coef_const) == \
        (1.0, -1.0, -0.5, -1.0, -4.5)
    r = oracle.interior_residual(U, torch.as_tensor(yi), op, X)
    scale = U.abs().max()
    assert float(r.abs().max()) < 1e-12 * float(scale) * 100
    # and the initial targets are q*(0, x)
    torch.testing.assert_close(torch.as_tensor(yb), exact_rows(torch.as_tensor(xb))[:, 0])


def test_dropping_a_term_breaks_it():
    """Each coefficient matters: with any one of them changed the residual of the
    exact solution no longer vanishes."""
    p = synth.log_fokker_planck(n_int=50, n_init=5)
    xi, yi, _, _ = p.batch()
    X = torch.as_tensor(xi)
    U = exact_rows(X)
    base = oracle.operator_of(p)
    for field in ("coef_xgrad", "coef_gradsq", "coef_const", "coef_lap", "coef_time"):
        op = oracle.Operator(**{**base.__dict__, field: 0.5 * getattr(base, field)})
        r = oracle.interior_residual(U, torch.as_tensor(yi), op, X)
        assert float(r.abs().max()) > 1e-3, field
