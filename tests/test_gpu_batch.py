"""Batches of heterogeneous instances (64-instance recipe: d in {2,5,10,20},
N ~ U{500..4000}, widths 64/128/256) stepped together (one inversion launch
sequence over every instance's factors, captured HIP graphs), against the same
instances stepped one context at a time.  The kernels and their inputs are the
same, so the results must be identical, the Jacobi sweep counts included; every
graph replay is checked, with unrelated eager work and synchronisation in
between."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def inputs(p, dev):
    T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float32, device=dev).contiguous()
    return T(p.theta0()), [T(a) for a in p.batch(0)]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_single_contexts(use_graph):
    from paper_2405_15603_amd import HParams, KfacPinn, KfacPinnBatch
    from paper_2405_15603_amd import _native as N
    dev = torch.device("cuda", 0)
    probs = synth.batch_instances(64)[:12]
    hp = HParams(lam=1e-3, beta=0.886041, momentum=0.707588, lr_mode="grid")
    steps = 3
    # reference: one context per instance, eager
    ref, ref_sweeps = [], []
    for p in probs:
        th, (xi, yi, xb, yb) = inputs(p, dev)
        kp = KfacPinn.for_problem(p, "bf16")
        traj = []
        for _ in range(steps):
            kp.step(th, xi, yi, xb, yb, hp)
            traj.append(th.clone())
        assert kp.sync() == 0
        ref.append(traj)
        ref_sweeps.append(kp.get_sweeps())
        del kp
    # the batch
    b = KfacPinnBatch(probs, "bf16", use_graph=use_graph)
    data = [inputs(p, dev) for p in probs]
    thetas = [d[0] for d in data]
    cols = list(zip(*[d[1] for d in data]))
    infos = torch.zeros(len(probs) * C.sizeof(N.kp_step_info), dtype=torch.uint8, device=dev)
    for it in range(steps):
        b.step(thetas, *cols, hp, infos)
        torch.cuda.synchronize()
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device=dev)
        (junk * 2).sum().item()
        for k in range(len(probs)):
            assert torch.equal(thetas[k], ref[k][it]), (it, k)
    assert b.sync() == [0] * len(probs)
    for k in range(len(probs)):
        assert b.get_sweeps(k) == list(ref_sweeps[k]), k
    raw = infos.cpu().numpy().tobytes()
    sz = C.sizeof(N.kp_step_info)
    for k in range(len(probs)):
        s = N.kp_step_info.from_buffer_copy(raw[k * sz:(k + 1) * sz])
        assert s.status == 0 and s.step == steps


def test_batch_graph_recaptures_on_new_arguments():
    """The second call passes new parameter buffers (holding the values after the
    first step), which recaptures the graph; the two steps still equal two
    consecutive single-context steps."""
    from paper_2405_15603_amd import HParams, KfacPinn, KfacPinnBatch
    dev = torch.device("cuda", 0)
    probs = synth.batch_instances(64)[12:16]
    hp = HParams(lam=1e-3, beta=0.886041, momentum=0.707588, lr_mode="grid")
    b = KfacPinnBatch(probs, "bf16")
    data = [inputs(p, dev) for p in probs]
    cols = list(zip(*[d[1] for d in data]))
    th_a = [d[0].clone() for d in data]
    b.step(th_a, *cols, hp)
    torch.cuda.synchronize()
    th_b = [t.clone() for t in th_a]
    b.step(th_b, *cols, hp)
    torch.cuda.synchronize()
    assert b.sync() == [0] * len(probs)
    for k, p in enumerate(probs):
        th, (xi, yi, xb, yb) = inputs(p, dev)
        ref = KfacPinn.for_problem(p, "bf16")
        ref.step(th, xi, yi, xb, yb, hp)
        torch.cuda.synchronize()
        assert torch.equal(th_a[k], th), k
        ref.step(th, xi, yi, xb, yb, hp)
        torch.cuda.synchronize()
        assert torch.equal(th_b[k], th), k
        assert ref.sync() == 0
        del ref
