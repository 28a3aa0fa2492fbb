"""The exact per-layer Gramian block (Eq. gramian; Section 3.2,
Eq. laplace_gramian_block_exact) from the stored slabs, through the C ABI, against
the oracle's reverse-mode Jacobian J^T J / N, per layer and term."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import gramian as og
from helpers import problem_inputs, rel, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "poisson2d": synth.poisson2d,
    "tiny_heat": lambda: synth.small_problem("heat", (3, 20, 9, 1), 29, 7, n_init=6, problem_id=72),
    "aniso": lambda: synth.small_problem("poisson", (4, 24, 17, 1), 53, 19, problem_id=84,
                                         op_coef=synth.anisotropic(4).op_coef),
    "logfp": lambda: synth.small_problem("logfp", (4, 16, 11, 1), 31, 0, n_init=9, problem_id=87),
}


def gramian(kp, layer, term, n):
    out = kp.layer_gramian(layer, term, n)
    assert kp.sync() == 0
    return out


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_layer_gramian(case, precision, tol):
    p = CASES[case]()
    th, xi, yi, xb, yb = problem_inputs(p, precision)
    kp = synth_kp(p, precision)
    kp.factors(*(to_dev(a, precision) for a in (th, xi, yi, xb, yb)), beta=0.0)
    assert kp.sync() == 0
    op = oracle.operator_of(p)
    data = (xi, yi, xb, yb)
    for term, n in ((0, xi.shape[0]), (1, xb.shape[0])):
        J = og.residual_jacobian(th, p.widths, data, op, term)
        off = og.layer_offsets(p.widths)
        for l in range(len(p.widths) - 1):
            Jl = J[:, off[l]:off[l + 1]]
            ref = Jl.T @ Jl / J.shape[0]
            got = gramian(kp, l, term, n)
            e = rel(got, ref)
            assert e < tol, (term, l, e)
            assert torch.equal(got, got.T)


def synth_kp(p, precision):
    from paper_2405_15603_amd import KfacPinn
    return KfacPinn.for_problem(p, precision)


def test_layer_gramian_rejects_large_layers():
    from paper_2405_15603_amd import KfacPinnError, _native as N
    p = synth.heat4d()
    th, xi, yi, xb, yb = problem_inputs(p, "f32", 50, 20)
    kp = synth_kp(p, "f32")
    kp.factors(*(to_dev(a, "f32") for a in (th, xi, yi, xb, yb)), beta=0.0)
    buf = torch.empty(1, dtype=torch.float64, device="cuda")
    st = kp.lib.kfac_pinn_layer_gramian(kp.h, 1, 0, C.c_void_p(buf.data_ptr()),
                                        C.c_void_p(buf.data_ptr()))
    assert st == N.KP_ERR_ARG
