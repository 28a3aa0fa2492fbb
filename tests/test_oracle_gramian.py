"""Pins for the exact per-layer Gramian oracle (Eq. gramian; Section 3.2,
Eq. laplace_gramian_block_exact): the autodiff Jacobian against central finite
differences, the block against the slab form sum_s z~_{n,s} (x) g_{n,s}, and the
case where KFAC is exact (the boundary term of the last layer: g = 1, so the
block is A (x) 1)."""
import pytest
import torch

import oracle
import synth
from oracle import gramian as og
from oracle.kfac import DT


def tiny(kind="poisson", widths=(2, 4, 3, 1), n=6, m=5, pid=64):
    p = synth.small_problem(kind, widths, n, m, n_init=2 if kind == "heat" else 0, problem_id=pid)
    return p, torch.as_tensor(p.theta0()), tuple(torch.as_tensor(a) for a in p.batch())


@pytest.mark.parametrize("term", [0, 1])
def test_jacobian_matches_central_differences(term):
    p, th, data = tiny("heat", widths=(3, 4, 3, 1))
    op = oracle.operator_of(p)
    J = og.residual_jacobian(th, p.widths, data, op, term)
    h = 1e-6
    for k in range(0, th.numel(), 5):
        e = torch.zeros_like(th)
        e[k] = h
        rp = og.residual_vectors(th + e, p.widths, *data, op)[term]
        rm = og.residual_vectors(th - e, p.widths, *data, op)[term]
        torch.testing.assert_close(J[:, k], (rp - rm) / (2 * h), rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_block_equals_slab_form(kind):
    """(1/N) sum_n (sum_s z~_{n,s} (x) g_{n,s})(...)^T with the oracle's own slabs."""
    p, th, data = tiny(kind, widths=(3, 5, 4, 1))
    op = oracle.operator_of(p)
    Ws = oracle.unpack(th, p.widths)
    ci = oracle.interior_curvature_inputs(Ws, data[0], data[1], op)
    cb = oracle.boundary_curvature_inputs(Ws, data[2], data[3])
    for l in range(len(Ws)):
        # column-stacked vec(g z~^T) = z~ (x) g
        Jn = torch.einsum("nsk,nsj->nkj", ci.zin[l], ci.g[l]).reshape(ci.zin[l].shape[0], -1)
        G = og.layer_gramian(th, p.widths, data, op, l, 0)
        torch.testing.assert_close(G, Jn.T @ Jn / Jn.shape[0], rtol=1e-12, atol=1e-14)
        Jb = torch.einsum("nk,nj->nkj", cb.zin[l], cb.g[l]).reshape(cb.zin[l].shape[0], -1)
        Gb = og.layer_gramian(th, p.widths, data, op, l, 1)
        torch.testing.assert_close(Gb, Jb.T @ Jb / Jb.shape[0], rtol=1e-12, atol=1e-14)


def test_kfac_is_exact_for_the_boundary_output_layer():
    p, th, data = tiny(widths=(3, 6, 5, 1), m=9)
    op = oracle.operator_of(p)
    L = len(p.widths) - 1
    G = og.layer_gramian(th, p.widths, data, op, L - 1, 1)
    Ws = oracle.unpack(th, p.widths)
    A, B = oracle.boundary_factors(oracle.boundary_curvature_inputs(Ws, data[2], data[3]))
    torch.testing.assert_close(G, torch.kron(A[L - 1], B[L - 1]), rtol=1e-13, atol=1e-15)
    ev = torch.linalg.eigvalsh(og.layer_gramian(th, p.widths, data, op, 1, 0))
    assert float(ev.min()) > -1e-12 * float(ev.max())
