#!/usr/bin/env python
"""KFAC steps/s on the 100-d Poisson problem (u* = sum sin(pi x_i)/100) with the
100 -> 768 -> 768 -> 512 -> 512 -> 1 tanh MLP, 3000 interior + 1000 boundary
points, on one MI355X.

One step = one full KFAC iteration (Algorithm 1): forward Laplacian, residuals,
backward pass, Kronecker factors with EMA, damped Kronecker-sum inverse,
preconditioned direction with momentum, grid line search over 31 step sizes and
the update.  The headline runs the mixed-precision path (BF16 MFMA, FP32
accumulation, FP64 factors and inversion); the plain FP32 path and the core
step (fixed step size, no line search) are timed beside it.  Inputs are resident
in HBM before the timed region.

The roofline object describes the dominant kernel, the line-search layer
product (k_fwdlap in BF16): algorithmic FLOPs of its launches over their
HIP-event durations.  Its HBM traffic comes from the committed rocprofv3
FETCH_SIZE / WRITE_SIZE summary when that summary was taken on the current
kernel source, else it is null.

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits."""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3, "f64": 78.6}
HBM_GBS = 8000.0
KERNEL_CLASSES = {"layer_gemm": 0, "factor_gemm": 1, "invert": 2, "act": 3, "ls_layer": 4}
KERNEL_NAMES = {"ls_layer": "k_fwdlap (line-search forward layer product)",
                "layer_gemm": "k_fwdlap / k_bwdlap (curvature pass layer products)",
                "factor_gemm": "k_tn (Kronecker factor and gradient products)",
                "invert": "Kronecker-sum factorisation (Cholesky + Jacobi)",
                "act": "forward-Laplacian finishing passes"}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_fwdlap_bf16_poisson100d_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2405_15603_amd", "csrc", "fwdlap.hip")


def hparams(lr_mode="grid", lr=1.0):
    from paper_2405_15603_amd import HParams
    # the paper's only printed KFAC hyper-parameters (2d Poisson run): beta, mu;
    # damping 1e-3; grid line search over 2^0 .. 2^-30
    return HParams(lam=1e-3, beta=0.886041, momentum=0.707588, lr_mode=lr_mode, lr=lr)


def run_gpu(problem, precision, steps, warmup, kernel_class=None, lr_mode="grid", ls_lanes=2):
    import numpy as np
    import torch
    from paper_2405_15603_amd import KfacPinn
    dt = torch.float64 if precision == "f64" else torch.float32
    dev = torch.device("cuda", 0)
    T = lambda a: torch.as_tensor(np.asarray(a), dtype=dt, device=dev).contiguous()
    th = T(problem.theta0())
    xi, yi, xb, yb = (T(a) for a in problem.batch(0))
    kp = KfacPinn.for_problem(problem, precision)
    kp.set_line_search_lanes(ls_lanes)
    hp = hparams(lr_mode, lr=2.0 ** -5)
    info = kp.empty(64, dtype=torch.uint8)
    for _ in range(warmup):
        kp.step(th, xi, yi, xb, yb, hp, info)
    torch.cuda.synchronize()
    if kernel_class is not None:
        kp.timing_enable(kernel_class)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        kp.step(th, xi, yi, xb, yb, hp, info)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    tm = kp.timing_read() if kernel_class is not None else None
    sweeps = kp.get_sweeps()
    status = kp.sync()
    last = KfacPinn.decode_info(info)
    last["jacobi_sweeps"] = sweeps
    del kp
    return ms, tm, status, last


def run_batch(count, steps, warmup, use_graph):
    """One step of `count` heterogeneous instances per call (the 64-instance
    recipe), as a captured graph or as direct launches on the internal lanes."""
    import numpy as np
    import torch
    import synth
    from paper_2405_15603_amd import KfacPinnBatch
    dev = torch.device("cuda", 0)
    probs = synth.batch_instances(count)
    T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float32, device=dev).contiguous()
    thetas = [T(p.theta0()) for p in probs]
    cols = list(zip(*[[T(a) for a in p.batch(0)] for p in probs]))
    b = KfacPinnBatch(probs, "bf16", use_graph=use_graph)
    hp = hparams()
    for _ in range(warmup):
        b.step(thetas, *cols, hp)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        b.step(thetas, *cols, hp)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    status = b.sync()
    del b
    return {"ms_per_step": ms, "instance_steps_per_s": count * 1000.0 / ms,
            "status_nonzero": sum(1 for v in status if v != 0)}


def copy_calibration(mib):
    """A plain elementwise copy of `mib` MiB (read once, written once), launched
    so that a rocprofv3 counter run can scale FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def measured_traffic():
    """Bytes per launch of the dominant kernel from the committed counter summary,
    or None when it is absent or was taken on another version of the kernel."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m and t):
        return None
    cur = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    return float(t.group(1)) if cur == m.group(1) else None


def cpu_baseline(problem, frac=0.1):
    """The FP64 oracle's step on a bounded sample of the same workload (same
    network, a fraction of the points), extrapolated to the full point count:
    the per-point work scales with the number of points, the Kronecker-sum
    inverse does not and is timed on its own."""
    import torch
    import oracle
    ns = max(1, int(problem.n_interior * frac))
    ms = max(1, int(problem.n_cond * frac))
    xi, yi, xb, yb = problem.batch(0)
    data = (xi[:ns], yi[:ns], xb[:ms], yb[:ms])
    op = oracle.operator_of(problem)
    h = hparams()
    hp = oracle.HParams(lam=h.lam, beta=h.beta, momentum=h.momentum, lr_mode="grid")
    st = oracle.init_state(problem.widths, True)
    th = problem.theta0()
    t0 = time.perf_counter()
    _, st1, _ = oracle.kfac_step(th, problem.widths, data, op, hp, st)
    t_sample = time.perf_counter() - t0
    t0 = time.perf_counter()
    for l in range(len(problem.widths) - 1):
        oracle.kron_sum_inverse(*(oracle.damp(m[l], hp.lam)
                                  for m in (st1.A_int, st1.B_int, st1.A_bnd, st1.B_bnd)))
    t_inv = time.perf_counter() - t0
    t_full = t_inv + max(t_sample - t_inv, 0.0) / frac
    return {"value": 1.0 / t_full, "unit": "steps/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": (f"oracle step on {ns} of {problem.n_interior} interior and {ms} of "
                       f"{problem.n_cond} boundary points with the full network "
                       f"({t_sample:.1f} s, of which Kronecker-sum inverse {t_inv:.2f} s); "
                       f"per-point work scaled by {1 / frac:.0f}")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "f32", "f64"])
    ap.add_argument("--workload", default="poisson100d")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison leg")
    ap.add_argument("--no-core", action="store_true", help="skip the fixed-step (core) leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch leg")
    ap.add_argument("--kernel", default="ls_layer", choices=list(KERNEL_CLASSES))
    ap.add_argument("--ls-lanes", type=int, default=2, choices=[1, 2],
                    help="streams for the line-search candidates in the timed run")
    ap.add_argument("--roofline-steps", type=int, default=20,
                    help="steps of the one-lane run that times the dominant kernel's launches")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the method's data-parallel sharding "
              "over collocation points is not built here (see the design notes)", file=sys.stderr)
        sys.exit(2)

    import synth
    problem = synth.PROBLEMS[args.workload]()
    if args.copy_calibration_mib > 0:
        copy_calibration(args.copy_calibration_mib)
    kc = KERNEL_CLASSES[args.kernel]
    # The headline run overlaps two line-search candidates on two streams; the
    # dominant kernel's launch durations come from a run with one lane, where each
    # launch has the chip to itself (with two lanes a launch's events also span the
    # other lane's work).
    ms, _, status, last = run_gpu(problem, args.precision, args.steps, args.warmup, None,
                                  ls_lanes=args.ls_lanes)
    if status != 0:
        print(f"device status {status} after the timed steps", file=sys.stderr)
        sys.exit(1)
    rsteps = max(1, min(args.steps, args.roofline_steps))
    ms1, tm, st1, _ = run_gpu(problem, args.precision, rsteps, args.warmup, kc, ls_lanes=1)
    if st1 != 0:
        print(f"device status {st1} after the one-lane steps", file=sys.stderr)
        sys.exit(1)
    out = {
        "metric": "KFAC steps/s, d=100 Poisson 768-wide MLP: mixed-prec vs FP32, rel err<=1e-3",
        "value": 1000.0 / ms,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "f32": "f32", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{problem.name}: -Lap u = f on [0,1]^{problem.d}, "
                               f"tanh MLP {'-'.join(map(str, problem.widths))}, "
                               f"{problem.n_interior} interior + {problem.n_cond} boundary "
                               f"points, grid line search (31 step sizes)",
                   "precision": args.precision, "parallelism": "single GPU"},
        "last_step": last,
    }
    if tm and tm["launches"] > 0:
        sec = tm["ms"] * 1e-3
        ach = tm["flops"] / sec / 1e12
        peak = PEAK_TFLOPS[args.precision]
        traffic = measured_traffic() if (args.kernel == "ls_layer" and args.precision == "bf16") else None
        out["roofline"] = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                           "frac": ach / peak, "traffic": traffic,
                           "kernel": f"{KERNEL_NAMES[args.kernel]}: {tm['launches']} launches, "
                                     f"{tm['ms'] / tm['launches']:.4f} ms average",
                           "algorithmic_bytes_per_launch": tm["bytes"] / tm["launches"],
                           "algorithmic_hbm_GBs": tm["bytes"] / sec / 1e9,
                           "hbm_frac": tm["bytes"] / sec / 1e9 / HBM_GBS,
                           "share_of_step": tm["ms"] / (ms1 * rsteps),
                           "timing_run": f"{rsteps} steps after {args.warmup} warm-up with one "
                                         f"line-search lane ({ms1:.2f} ms per step there)"}
    out["line_search_lanes"] = args.ls_lanes
    side_steps = max(2, min(20, args.steps // 2))   # the comparison legs
    if not args.no_core:
        msc, _, stc, _ = run_gpu(problem, args.precision, side_steps, 1, None, lr_mode="fixed")
        out["core_step"] = {"value": 1000.0 / msc, "ms_per_step": msc, "status": stc,
                            "note": "fixed step size 2^-5, no line search"}
    if not args.no_fp32 and args.precision != "f32":
        ms32, _, st32, _ = run_gpu(problem, "f32", side_steps, 1, None)
        out["fp32"] = {"value": 1000.0 / ms32, "ms_per_step": ms32, "status": st32,
                       "mixed_over_fp32": ms32 / ms}
    if not args.no_batch:
        out["batch64"] = {"instances": 64, "note": "heterogeneous 64-instance recipe, mixed "
                          "precision, grid line search; one step of every instance per call",
                          "graph": run_batch(64, 3, 1, True),
                          "direct": run_batch(64, 3, 1, False)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problem)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
