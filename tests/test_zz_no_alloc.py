"""kfac_pinn_precondition_layer_noalloc (the one-layer Kronecker-sum apply whose
intermediate products live in the library's static device scratch, for callers
that cannot allocate) against kfac_pinn_precondition of a context: the same
kernels on the same operands, so each layer's block must be identical.  Two calls
in a row, the second on a smaller layer, so the second runs on scratch that still
holds the first call's products; then a call over the limit is refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from helpers import problem_inputs, to_dev

pytestmark = pytest.mark.gpu


def test_noalloc_layer_apply_matches_context_apply():
    from paper_2405_15603_amd import KfacPinn, _native as N
    p = synth.small_problem("poisson", (7, 130, 67, 33, 1), 151, 45, problem_id=73)
    th, xi, yi, xb, yb = problem_inputs(p, "f64")
    kp = KfacPinn.for_problem(p, "f64")
    grad, _ = kp.factors(*(to_dev(a, "f64") for a in (th, xi, yi, xb, yb)), beta=0.0)
    kp.invert(1e-3)
    ref = kp.precondition(grad)
    assert kp.sync() == 0
    off = synth.layer_offsets(p.widths)
    lib = N.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # layer 1 (131 x 67 block), then the smaller layer 2 (68 x 33) on the same scratch
    for l in (1, 2, 0):
        nA, nB = p.widths[l] + 1, p.widths[l + 1]
        PA, a = kp.get_preconditioner(l, 0)
        PB, b = kp.get_preconditioner(l, 1)
        assert kp.sync() == 0
        g = grad[off[l]:off[l + 1]].contiguous()
        out = torch.full_like(g, float("nan"))
        st = lib.kfac_pinn_precondition_layer_noalloc(
            nA, nB, C.c_void_p(PA.data_ptr()), C.c_void_p(a.data_ptr()), C.c_void_p(PB.data_ptr()),
            C.c_void_p(b.data_ptr()), C.c_void_p(g.data_ptr()), C.c_void_p(out.data_ptr()), stream)
        assert st == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref[off[l]:off[l + 1]]), l
    big = torch.zeros(1, dtype=torch.float64, device="cuda")
    p_ = C.c_void_p(big.data_ptr())
    assert lib.kfac_pinn_precondition_layer_noalloc(1025, 1024, p_, p_, p_, p_, p_, p_,
                                                   stream) == N.KP_ERR_ARG
