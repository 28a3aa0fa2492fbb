"""The Jacobi eigensolver's early stop (host reads of each sweep's convergence
flags, no sweeps enqueued past convergence) against the full schedule of
max_sweeps sweeps per call: the same steps must give bit-identical parameters,
preconditioners and sweep counts, from a cold start and from warm starts, with
groups of problems on several streams."""
import pytest
import torch

import synth
from helpers import problem_inputs, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_early_stop_equals_full_schedule(precision):
    from paper_2405_15603_amd import HParams, KfacPinn
    p = synth.small_problem("heat", (4, 100, 70, 1), 301, 97, n_init=31, problem_id=91)
    th, xi, yi, xb, yb = problem_inputs(p, precision)
    hp = HParams(lam=1e-3, beta=0.9, momentum=0.5)
    runs = []
    for wait in (True, False):
        kp = KfacPinn.for_problem(p, precision)
        kp.set_sweep_wait(wait)
        tht = to_dev(th, precision)
        dev = [to_dev(a, precision) for a in (xi, yi, xb, yb)]
        sweeps = []
        for _ in range(4):
            info = KfacPinn.decode_info(kp.step(tht, *dev, hp))
            assert kp.sync() == 0 and info["status"] == 0
            sweeps.append(kp.get_sweeps())
        pre = [kp.get_preconditioner(l, s) for l in range(len(p.widths) - 1) for s in (0, 1)]
        runs.append((tht.clone(), sweeps, pre))
    (ta, sa, pa), (tb, sb, pb) = runs
    assert sa == sb
    assert max(sa[0]) > max(sa[-1]) >= 1   # warm starts converge in fewer sweeps
    assert torch.equal(ta, tb)
    for (Pa, ea), (Pb, eb) in zip(pa, pb):
        assert torch.equal(Pa, Pb) and torch.equal(ea, eb)


def test_sweep_wait_rejects_bad_values():
    from paper_2405_15603_amd import KfacPinn
    from paper_2405_15603_amd import _native as N
    kp = KfacPinn((2, 8, 1), "f64")
    assert kp.lib.kfac_pinn_set_sweep_wait(kp.h, 2) == N.KP_ERR_ARG
    assert kp.lib.kfac_pinn_set_sweep_wait(kp.h, 0) == N.KP_OK
