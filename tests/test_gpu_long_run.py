"""The plain FP32 method on the 5-d Poisson problem as the paper trains it
(Appendix A.3's set-up): 5-64-64-48-48-1 tanh net, 3000 interior + 500 boundary
points drawn afresh every step by the GPU sampler, damping 1e-3, EMA 0.886041,
momentum 0.7075879, grid line search, 1000 steps.  The loss and the relative L2
error on 30 000 seeded uniform evaluation points are a sanity record (printed),
not a parity check: every step must succeed, the loss must fall by orders of
magnitude and the error must end well below that of the initial network."""
import numpy as np
import pytest
import torch

import synth
from helpers import to_dev

pytestmark = pytest.mark.gpu


def l2_error(kp, theta, p, x_eval):
    u = []
    for i in range(0, x_eval.shape[0], p.n_interior):
        ui, _, _ = kp.forward_laplacian(theta, x_eval[i:i + p.n_interior])
        u.append(ui.double().cpu())
    u = torch.cat(u)
    ref = torch.sin(np.pi * x_eval.double().cpu()).sum(1)
    return float((u - ref).norm() / ref.norm())


def test_poisson5d_fp32_1000_resampled_steps():
    from paper_2405_15603_amd import HParams, KfacPinn, sampler_for
    p = synth.poisson5d()
    kp = KfacPinn.for_problem(p, "f32")
    theta = to_dev(p.theta0(), "f32")
    g = torch.Generator().manual_seed(30000)
    x_eval = torch.rand(30000, p.d, generator=g, dtype=torch.float64).float().cuda()
    err0 = l2_error(kp, theta, p, x_eval)
    hp = HParams(lam=1e-3, beta=0.886041, momentum=0.7075879, lr_mode="grid")
    smp = sampler_for(p)
    info = kp.empty(64, dtype=torch.uint8)
    losses = {}
    for step in range(1000):
        xi, yi, xb, yb = kp.sample(smp, step, p.n_interior, p.n_cond)
        kp.step(theta, xi, yi, xb, yb, hp, info)
        if step in (0, 9, 99, 499, 999):
            d = KfacPinn.decode_info(info)
            assert kp.sync() == 0 and d["status"] == 0, (step, d)
            losses[step] = d["loss_interior"] + d["loss_boundary"]
    err = l2_error(kp, theta, p, x_eval)
    print("losses", {k: f"{v:.3e}" for k, v in losses.items()},
          f"L2 error {err0:.3e} -> {err:.3e}", flush=True)
    assert np.isfinite(err) and all(np.isfinite(v) for v in losses.values())
    assert losses[999] < 1e-2 * losses[0]
    assert err < 0.1 * err0
