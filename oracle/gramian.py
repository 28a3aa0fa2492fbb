"""FP64 CPU oracle for the exact per-layer Gramian block.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports it.

Dangel, Mueller & Zeinhofer (NeurIPS 2024), Section 2.2, Eq. (gramian): the
Gramian of the PINN loss is G = (1/N) sum_n J_n^T J_n + (1/M) sum_n J_{b,n}^T J_{b,n}
with J_n the Jacobian of the interior residual of point n and J_{b,n} that of the
boundary residual; Section 3.2, Eq. (laplace_gramian_block_exact), writes layer l's
diagonal block of the interior term through the layer's shared rows.  This oracle
takes the definition literally: the residuals' Jacobian with respect to the
layer's parameters by reverse-mode autodiff, then J^T J / N per term.
"""
from __future__ import annotations

import torch

from .kfac import DT, TANH, _t, num_params
from .kfac_star import residual_vectors


def layer_offsets(widths):
    off = [0]
    for l in range(len(widths) - 1):
        off.append(off[-1] + widths[l + 1] * (widths[l] + 1))
    return off


def residual_jacobian(theta, widths, data, op, term: int, act=TANH) -> torch.Tensor:
    """d r / d theta (rows: points of the term, 0 interior / 1 boundary; columns:
    all parameters in the theta layout), by reverse-mode autodiff."""
    Xi, yi, Xb, yb = map(_t, data)
    f = lambda t: residual_vectors(t, widths, Xi, yi, Xb, yb, op, act)[term]
    return torch.autograd.functional.jacobian(f, _t(theta).detach())


def layer_gramian(theta, widths, data, op, layer: int, term: int, act=TANH) -> torch.Tensor:
    """Layer `layer`'s diagonal block of one term of Eq. (gramian):
    (1/count) J_l^T J_l with J_l the residual Jacobian's columns of that layer."""
    J = residual_jacobian(theta, widths, data, op, term, act)
    off = layer_offsets(widths)
    Jl = J[:, off[layer]:off[layer + 1]]
    return Jl.T @ Jl / J.shape[0]
