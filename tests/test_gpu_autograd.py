"""The differentiation pattern: the forward Laplacian as a torch.autograd.Function
whose backward is the library's hand-written adjoint (the paper differentiates with
autodiff, Algorithm 1), checked against the oracle's autodiff and against central
finite differences; and per-layer recomputation under a workspace limit against
the stored-slab path."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import oracle_curvature, problem_inputs, rel, rounded, to_dev

pytestmark = pytest.mark.gpu


def kp_for(p, precision, **kw):
    from paper_2405_15603_amd import KfacPinn
    return KfacPinn.for_problem(p, precision, **kw)


def heat_small():
    return synth.small_problem("heat", (5, 24, 20, 12, 1), 61, 17, n_init=9, problem_id=74)


def objective_weights(n, d, seed, precision):
    g = torch.Generator().manual_seed(seed)
    w = [torch.randn(n, generator=g, dtype=torch.float64),
         torch.randn(n, d, generator=g, dtype=torch.float64),
         torch.randn(n, generator=g, dtype=torch.float64)]
    return [torch.as_tensor(rounded(a.numpy(), precision)) for a in w]


@pytest.mark.parametrize("precision,tol", [("f64", 1e-11), ("f32", 1e-4)])
def test_autograd_function_matches_oracle_autodiff(precision, tol):
    """torch.autograd through ForwardLaplacian equals autodiff of the oracle's
    forward Laplacian, for theta and for the points."""
    from paper_2405_15603_amd import forward_laplacian
    p = heat_small()
    th, xi, _, _, _ = problem_inputs(p, precision)
    kp = kp_for(p, precision)
    n, d = xi.shape
    ub, gb, lb = objective_weights(n, d, 5, precision)
    theta = to_dev(th, precision).requires_grad_(True)
    x = to_dev(xi, precision).requires_grad_(True)
    u, g, lap = forward_laplacian(kp, theta, x)
    obj = (u * to_dev(ub, precision)).sum() + (g * to_dev(gb, precision)).sum() + \
        (lap * to_dev(lb, precision)).sum()
    obj.backward()
    tht = torch.as_tensor(th).clone().requires_grad_(True)
    xr = torch.as_tensor(xi).clone().requires_grad_(True)
    U = oracle.forward_laplacian(oracle.unpack(tht, p.widths), xr,
                                 oracle.operator_of(p).mask_vec(d)).out
    ref = (U[:, 0] * ub).sum() + (U[:, 1:d + 1] * gb).sum() + (U[:, -1] * lb).sum()
    rt, rx = torch.autograd.grad(ref, (tht, xr))
    assert rel(theta.grad, rt) < tol
    assert rel(x.grad, rx) < tol


def test_autograd_function_against_finite_differences():
    """FP64: the adjoint's directional derivatives along 16 random unit directions
    (seed 4004) against central differences with h = 1e-4 of the GPU forward.  The
    FD truncation error is O(h^2 |f'''|) ~ 1e-8 relative (measured 3e-9); the bound
    is 1e-7."""
    from paper_2405_15603_amd import forward_laplacian
    p = synth.heat4d()
    th, xi, _, _, _ = problem_inputs(p, "f64", 400, 10)
    kp = kp_for(p, "f64", max_interior=400, max_boundary=16)
    n, d = xi.shape
    ub, gb, lb = (to_dev(a, "f64") for a in objective_weights(n, d, 6, "f64"))
    x = to_dev(xi, "f64")

    def f(theta):
        u, g, lap = kp.forward_laplacian(theta, x)
        return float((u * ub).sum() + (g * gb).sum() + (lap * lb).sum())

    theta = to_dev(th, "f64").requires_grad_(True)
    u, g, lap = forward_laplacian(kp, theta, x)
    ((u * ub).sum() + (g * gb).sum() + (lap * lb).sum()).backward()
    grad = theta.grad.detach()
    dirs = torch.as_tensor(synth.uniform(p.seed(synth.PURPOSE_DIRECTIONS), 0, 16 * th.size).reshape(16, th.size) - 0.5,
                           dtype=torch.float64)
    dirs = dirs / dirs.norm(dim=1, keepdim=True)
    h = 1e-4
    base = to_dev(th, "f64")
    worst = 0.0
    for v in dirs:
        vd = v.to(base.device)
        fd = (f(base + h * vd) - f(base - h * vd)) / (2 * h)
        ad = float(grad @ vd)
        err = abs(fd - ad) / max(abs(ad), 1e-12 * float(grad.norm()))
        worst = max(worst, err)
    print(f"worst directional-derivative relative error {worst:.2e}")
    assert worst < 1e-7


def test_workspace_limit_recompute_matches_store():
    """Heat (4+1)d in FP32 at its full size (4000 interior, 2000 boundary and
    initial points, R = 28 000 rows): a workspace limit below the slab size
    switches to per-layer recomputation; factors, gradient, loss and a full step
    are identical to the stored-slab path (same kernels, same order), and both
    match the oracle."""
    from paper_2405_15603_amd import HParams
    p = synth.heat4d()
    th, xi, yi, xb, yb = problem_inputs(p, "f32")
    args = [to_dev(a, "f32") for a in (th, xi, yi, xb, yb)]
    full = kp_for(p, "f32")
    lim = kp_for(p, "f32", workspace_limit_bytes=1 << 20)
    assert full.recompute_mode() == (False, False) and lim.recompute_mode()[0]
    out = {}
    for name, kp in (("store", full), ("recompute", lim)):
        kp.reset_state(True)
        grad, loss = kp.factors(*args, beta=0.0)
        assert kp.sync() == 0
        facs = [kp.get_factor(l, t, s).cpu() for l in range(len(p.widths) - 1)
                for t in (0, 1) for s in (0, 1)]
        tht = args[0].clone()
        kp.reset_state(True)
        kp.step(tht, *args[1:], HParams(lam=1e-3, beta=0.886041, momentum=0.707588))
        assert kp.sync() == 0
        out[name] = (grad.cpu(), loss.cpu(), facs, tht.cpu())
    a, b = out["store"], out["recompute"]
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert all(torch.equal(x, y) for x, y in zip(a[2], b[2]))
    assert torch.equal(a[3], b[3])
    ref = oracle_curvature(p, th, xi, yi, xb, yb)
    k = 0
    for l in range(len(p.widths) - 1):
        for tn in ("int", "bnd"):
            for sn in ("A", "B"):
                assert rel(b[2][k], ref[f"{sn}_{tn}"][l]) < 1e-5, (l, tn, sn)
                k += 1
    assert rel(b[0], ref["grad"]) < 1e-4
