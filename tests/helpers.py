"""Shared helpers for the parity tests: run the oracle on the same (rounded)
inputs the GPU path receives, and compare with norm-wise relative errors."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import synth

DEV = "cuda"


def rel(a, b) -> float:
    a = np.asarray(a.detach().cpu() if isinstance(a, torch.Tensor) else a, dtype=np.float64)
    b = np.asarray(b.detach().cpu() if isinstance(b, torch.Tensor) else b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rounded(a, precision: str) -> np.ndarray:
    """The value the GPU path receives (FP32 master data outside the FP64 path)."""
    a = np.asarray(a, dtype=np.float64)
    return a if precision == "f64" else a.astype(np.float32).astype(np.float64)


def to_dev(a, precision: str) -> torch.Tensor:
    dt = torch.float64 if precision == "f64" else torch.float32
    return torch.as_tensor(np.asarray(a), dtype=dt, device=DEV).contiguous()


def problem_inputs(p: "synth.Problem", precision: str, n_int=None, n_bnd=None, step=0):
    th = rounded(p.theta0(), precision)
    xi, yi, xb, yb = (rounded(a, precision) for a in p.batch(step))
    if n_int is not None:
        xi, yi = xi[:n_int], yi[:n_int]
    if n_bnd is not None:
        xb, yb = xb[:n_bnd], yb[:n_bnd]
    return th, xi, yi, xb, yb


def oracle_curvature(p, th, xi, yi, xb, yb):
    op = oracle.operator_of(p)
    Ws = oracle.unpack(torch.as_tensor(th), p.widths)
    ci = oracle.interior_curvature_inputs(Ws, torch.as_tensor(xi), torch.as_tensor(yi), op)
    cb = oracle.boundary_curvature_inputs(Ws, torch.as_tensor(xb), torch.as_tensor(yb))
    Ai, Bi = oracle.interior_factors(ci)
    Ab, Bb = oracle.boundary_factors(cb)
    grad, li, lb = oracle.loss_gradient(th, p.widths, xi, yi, xb, yb, op)
    return {"A_int": Ai, "B_int": Bi, "A_bnd": Ab, "B_bnd": Bb, "grad": grad, "loss": (li, lb)}
