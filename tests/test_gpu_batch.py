"""Batches of heterogeneous instances (64-instance recipe: d in {2,5,10,20},
N ~ U{500..4000}, widths 64/128/256) stepped together (one inversion launch
sequence over every instance's factors, the grouped line search whose launches
each cover every instance, captured HIP graphs), against the same instances
stepped one context at a time.  The kernels' bodies and their inputs are the
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


@pytest.mark.parametrize("use_graph,grouped", [(True, True), (False, True), (True, False)])
def test_batch_matches_single_contexts(use_graph, grouped):
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
    b.set_grouped(grouped)
    data = [inputs(p, dev) for p in probs]
    thetas = [d[0] for d in data]
    cols = list(zip(*[d[1] for d in data]))
    infos = torch.zeros(len(probs) * C.sizeof(N.kp_step_info), dtype=torch.uint8, device=dev)
    for it in range(steps):
        b.step(thetas, *cols, hp, infos)
        torch.cuda.synchronize()
        assert b.is_grouped() == grouped and b.grouped_products() == grouped
        assert b.grouped_two_lanes() == grouped
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


def test_grouped_line_search_with_new_point_counts():
    """Grouped line search over instances whose point counts change from one call
    to the next (fewer interior and boundary points on the second call, the job
    tables rewritten): each call equals the single-context step on the same
    points, in direct launches and in captured graphs."""
    from paper_2405_15603_amd import HParams, KfacPinn, KfacPinnBatch
    dev = torch.device("cuda", 0)
    probs = synth.batch_instances(64)[20:26]
    hp = HParams(lam=1e-3, beta=0.886041, momentum=0.707588, lr_mode="grid")
    for use_graph in (False, True):
        b = KfacPinnBatch(probs, "bf16", use_graph=use_graph)
        data = [inputs(p, dev) for p in probs]
        thetas = [d[0] for d in data]
        refs = [KfacPinn.for_problem(p, "bf16") for p in probs]
        ref_th = [d[0].clone() for d in data]
        for frac in (1.0, 0.55, 0.55, 1.0):
            cols = []
            for (th, (xi, yi, xb, yb)) in data:
                ni, nb = max(1, int(xi.shape[0] * frac)), max(1, int(xb.shape[0] * frac))
                cols.append((xi[:ni], yi[:ni], xb[:nb], yb[:nb]))
            b.step(thetas, *list(zip(*cols)), hp)
            torch.cuda.synchronize()
            assert b.is_grouped() and b.grouped_products()
            for k, kp in enumerate(refs):
                kp.step(ref_th[k], *cols[k], hp)
            torch.cuda.synchronize()
            for k in range(len(probs)):
                assert torch.equal(thetas[k], ref_th[k]), (use_graph, frac, k)
        assert b.sync() == [0] * len(probs)
        assert all(kp.sync() == 0 for kp in refs)
        del b, refs


def test_grouped_line_search_fallbacks():
    """The grouped line search needs the grid search and BF16 line-search slabs:
    a fixed step size, the FP32 path or grouping switched off take the
    per-instance launches (and still equal the single contexts)."""
    from paper_2405_15603_amd import HParams, KfacPinn, KfacPinnBatch
    dev = torch.device("cuda", 0)
    probs = synth.batch_instances(64)[30:33]
    cases = [("bf16", HParams(lam=1e-3, beta=0.5, momentum=0.5, lr_mode="fixed", lr=2.0 ** -6)),
             ("f32", HParams(lam=1e-3, beta=0.5, momentum=0.5, lr_mode="grid"))]
    for precision, hp in cases:
        b = KfacPinnBatch(probs, precision)
        data = [inputs(p, dev) for p in probs]
        thetas = [d[0] for d in data]
        cols = list(zip(*[d[1] for d in data]))
        b.step(thetas, *cols, hp)
        torch.cuda.synchronize()
        assert not b.is_grouped()
        # the factor products stay grouped with a fixed step (mixed curvature products)
        assert b.grouped_products() == (precision == "bf16")
        assert b.sync() == [0] * len(probs)
        for k, p in enumerate(probs):
            th, (xi, yi, xb, yb) = inputs(p, dev)
            kp = KfacPinn.for_problem(p, precision)
            kp.step(th, xi, yi, xb, yb, hp)
            torch.cuda.synchronize()
            assert torch.equal(thetas[k], th), (precision, k)
            del kp
        del b
    from paper_2405_15603_amd import _native as N
    b = KfacPinnBatch(probs, "bf16")
    assert b.lib.kfac_pinn_batch_set_grouped(b.h, 2) == N.KP_ERR_ARG


def forced_chunks_cache(b, data, path, nch):
    """A tuning cache that sets every class of the batch to `nch` chunks (at most
    one per derivative row): a first tune writes the timed choices for this
    device, the rewritten file is read back by a second tune (nothing timed)."""
    import json
    thetas = [d[0].clone() for d in data]
    cols = list(zip(*[d[1] for d in data]))
    assert b.tune(thetas, *cols, cache_path=str(path)) > 0
    doc = json.loads(path.read_text())
    assert doc["kfac_pinn_tune"] == 2 and doc["entries"]
    for e in doc["entries"]:
        e["nch"] = min(nch, e["S"] - 2)
    path.write_text(json.dumps(doc))
    assert b.tune(thetas, *cols, cache_path=str(path)) == 0
    return doc


def test_batch_tune_cache_and_choices(tmp_path):
    """The tuner times every class once and writes them to its JSON cache; a second
    tune reads them back without timing.  A step after tuning takes the grouped
    line search and succeeds on every instance; with the single-instance chunk
    count forced for every class (nch 0 in the cache) and every class on one tile
    geometry, each of the three, it equals the single contexts."""
    import json
    from paper_2405_15603_amd import HParams, KfacPinn, KfacPinnBatch
    dev = torch.device("cuda", 0)
    probs = synth.batch_instances(64)[40:48]
    hp = HParams(lam=1e-3, beta=0.886041, momentum=0.707588, lr_mode="grid")
    b = KfacPinnBatch(probs, "bf16")
    data = [inputs(p, dev) for p in probs]
    thetas = [d[0].clone() for d in data]
    cols = list(zip(*[d[1] for d in data]))
    path = tmp_path / "tune.json"
    timed = b.tune(thetas, *cols, cache_path=str(path))
    doc = json.loads(path.read_text())
    keys = {(e["K"], e["h_out"], e["S"], e["value_only"]) for e in doc["entries"]}
    assert timed == len(keys) > 0
    assert all(0 <= e["nch"] <= 8 and 0 <= e["geo"] <= 2 for e in doc["entries"])
    assert any(e["value_only"] == 1 for e in doc["entries"])
    assert b.tune(thetas, *cols, cache_path=str(path)) == 0
    b.step(thetas, *cols, hp)
    torch.cuda.synchronize()
    assert b.is_grouped() and b.sync() == [0] * len(probs)
    ref = []
    for k, p in enumerate(probs):
        th, (xi, yi, xb, yb) = inputs(p, dev)
        kp = KfacPinn.for_problem(p, "bf16")
        kp.step(th, xi, yi, xb, yb, hp)
        torch.cuda.synchronize()
        ref.append(th)
        del kp
    # the single-instance chunk counts on each tile geometry: kfac_pinn_step's results
    for geo in range(3):
        for e in doc["entries"]:
            e["nch"], e["geo"] = 0, geo
        path.write_text(json.dumps(doc))
        b2 = KfacPinnBatch(probs, "bf16")
        assert b2.tune(thetas, *cols, cache_path=str(path)) == 0
        th2 = [d[0].clone() for d in data]
        b2.step(th2, *cols, hp)
        torch.cuda.synchronize()
        assert b2.is_grouped() and b2.sync() == [0] * len(probs)
        for k in range(len(probs)):
            assert torch.equal(th2[k], ref[k]), (geo, k)
        del b2


def test_batch_tune_errors(tmp_path):
    """The tuner's error paths: instances that do not take the grouped line search
    (FP32) give KP_ERR_STATE, an empty boundary set KP_ERR_ARG, and a cache path
    that cannot be written KP_ERR_ARG after the choices are applied (the next step
    still takes the grouped line search and succeeds)."""
    from paper_2405_15603_amd import HParams, KfacPinnBatch
    from paper_2405_15603_amd import _native as N
    dev = torch.device("cuda", 0)
    probs = synth.batch_instances(64)[50:53]
    n = len(probs)

    def call(b, thetas, cols, path, nb_override=None):
        V = C.c_void_p * n
        I = C.c_int32 * n
        xi, yi, xb, yb = cols
        nbs = [t.shape[0] for t in xb] if nb_override is None else nb_override
        return b.lib.kfac_pinn_batch_tune(
            b.h, V(*[t.data_ptr() for t in thetas]), V(*[t.data_ptr() for t in xi]),
            V(*[t.data_ptr() for t in yi]), I(*[t.shape[0] for t in xi]),
            V(*[t.data_ptr() for t in xb]), V(*[t.data_ptr() for t in yb]), I(*nbs),
            path.encode() if path else None, None)

    data = [inputs(p, dev) for p in probs]
    thetas = [d[0] for d in data]
    cols = list(zip(*[d[1] for d in data]))
    b32 = KfacPinnBatch(probs, "f32")
    assert call(b32, thetas, cols, None) == N.KP_ERR_STATE
    del b32
    b = KfacPinnBatch(probs, "bf16")
    assert call(b, thetas, cols, None, nb_override=[0] * n) == N.KP_ERR_ARG
    bad = str(tmp_path / "no_such_dir" / "tune.json")
    assert call(b, thetas, cols, bad) == N.KP_ERR_ARG
    # a malformed cache reads as empty: every class is timed and the file rewritten
    junk = tmp_path / "junk.json"
    junk.write_text('{"entries": [{"device": "x", "K": }, {nonsense')
    assert b.tune(thetas, *cols, cache_path=str(junk)) > 0
    import json
    assert json.loads(junk.read_text())["entries"]
    hp = HParams(lam=1e-3, beta=0.5, momentum=0.5, lr_mode="grid")
    b.step(thetas, *cols, hp)
    torch.cuda.synchronize()
    assert b.is_grouped() and b.sync() == [0] * n


@pytest.mark.parametrize("forced_nch", [None, 1])
def test_batch_instances_against_oracle(forced_nch, tmp_path):
    """Four instances of the 64-instance recipe (d = 20 at widths 256, 64 and 128,
    and a d = 2 one) stepped as a batch in mixed precision, one step from identity
    factors with beta = 0, so the factors after the step are the step's own.  Each
    instance's factors must be within the 1e-3 gate of the oracle's at the same
    parameters and points, and its candidate losses and chosen step must pass the
    BF16 line-search check (helpers.check_bf16_candidates) -- also with the grouped
    line search's layer products in one chunk per class (a tuned choice)."""
    from paper_2405_15603_amd import HParams, KfacPinnBatch
    import oracle
    from helpers import check_bf16_candidates, oracle_curvature, rel
    dev = torch.device("cuda", 0)
    allp = synth.batch_instances(64)
    pick = [0, 28, 36, 15]
    probs = [allp[k] for k in pick]
    assert {p.d for p in probs} >= {20, 2} and 256 in {p.widths[1] for p in probs}
    hp = HParams(lam=1e-3, beta=0.0, momentum=0.0, lr_mode="grid")
    b = KfacPinnBatch(probs, "bf16")
    data = [inputs(p, dev) for p in probs]
    if forced_nch is not None:
        forced_chunks_cache(b, data, tmp_path / "tune.json", forced_nch)
    thetas = [d[0] for d in data]
    th0 = [t.cpu().double().numpy().copy() for t in thetas]
    cols = list(zip(*[d[1] for d in data]))
    infos = torch.zeros(len(probs) * C.sizeof(N_info()), dtype=torch.uint8, device=dev)
    b.step(thetas, *cols, hp, infos)
    torch.cuda.synchronize()
    assert b.sync() == [0] * len(probs)
    assert b.is_grouped()
    raw = infos.cpu().numpy().tobytes()
    sz = C.sizeof(N_info())
    for k, p in enumerate(probs):
        kp = b.contexts[k]
        xi, yi, xb, yb = (np.asarray(a.cpu().double()) for a in data[k][1])
        ref = oracle_curvature(p, th0[k], xi, yi, xb, yb)
        # an instance's context runs on its lane: wait for it after each copy
        def fetch(t):
            assert kp.sync() == 0
            return t.cpu().double().numpy()
        worst = 0.0
        for l in range(len(p.widths) - 1):
            for t, tn in ((0, "int"), (1, "bnd")):
                for s, sn in ((0, "A"), (1, "B")):
                    worst = max(worst, rel(fetch(kp.get_factor(l, t, s)), ref[f"{sn}_{tn}"][l]))
        s = N_info().from_buffer_copy(raw[k * sz:(k + 1) * sz])
        alpha = s.lr_chosen
        dhat = fetch(kp.get_momentum()) / alpha
        ls = fetch(kp.get_line_search(31))
        op = oracle.operator_of(p)
        cand = np.array([oracle.loss(th0[k] + 2.0 ** -j * dhat, p.widths, xi, yi, xb, yb, op)[0]
                         for j in range(31)])
        res = check_bf16_candidates(ls, cand, alpha)
        print(f"instance {pick[k]} {p.widths} N={p.n_interior}: worst factor {worst:.2e}, "
              f"alpha* {alpha:g}, candidates {res}")
        assert worst < 1e-3


def N_info():
    from paper_2405_15603_amd import _native as N
    return N.kp_step_info
