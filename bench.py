#!/usr/bin/env python
"""KFAC steps/s on the 100-d Poisson problem (u* = sum sin(pi x_i)/100) with the
100 -> 768 -> 768 -> 512 -> 512 -> 1 tanh MLP, 3000 interior + 1000 boundary
points, on one MI355X.

One step = one full KFAC iteration (Algorithm 1): forward Laplacian, residuals,
backward pass, Kronecker factors with EMA, damped Kronecker-sum inverse,
preconditioned direction with momentum, grid line search over 31 step sizes and
the update.  The headline runs a mixed-precision path (FP32 accumulation, FP64
factors and inversion, BF16 line search; curvature products in BF16x3 or FP16,
--precision), the other mixed path is timed beside it; the plain FP32 path and the core
step (fixed step size, no line search) and KFAC* (learning rate and momentum
from the quadratic model, Section 3.4) are timed beside it.  Inputs are resident
in HBM before the timed region.  The headline times --repeats regions of exactly
--steps steps each (after --warmup untimed steps) and reports their median; all
of them are listed under last_step.

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

# dense MFMA peaks of the dominant kernel's arithmetic (the line search is BF16 in
# both mixed paths)
PEAK_TFLOPS = {"bf16": 2500.0, "f16": 2500.0, "f32": 157.3, "f64": 78.6}
HBM_GBS = 8000.0
KERNEL_CLASSES = {"layer_gemm": 0, "factor_gemm": 1, "invert": 2, "act": 3, "ls_layer": 4}
KERNEL_NAMES = {"ls_layer": "k_fwdlap (line-search forward layer product)",
                "layer_gemm": "k_fwdlap / k_bwdlap (curvature pass layer products)",
                "factor_gemm": "k_tn (Kronecker factor and gradient products)",
                "invert": "Kronecker-sum factorisation (Cholesky + Jacobi)",
                "act": "forward-Laplacian finishing passes"}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_fwdlap_bf16_poisson100d_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2405_15603_amd", "csrc", "fwdlap.hip")


def log(msg):
    """Progress of the legs on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def hparams(lr_mode="grid", lr=1.0):
    from paper_2405_15603_amd import HParams
    # the paper's only printed KFAC hyper-parameters (2d Poisson run): beta, mu;
    # damping 1e-3; grid line search over 2^0 .. 2^-30
    return HParams(lam=1e-3, beta=0.886041, momentum=0.707588, lr_mode=lr_mode, lr=lr)


def run_gpu(problem, precision, steps, warmup, kernel_class=None, lr_mode="grid", ls_lanes=2,
            repeats=1):
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
    # `repeats` timed regions of exactly `steps` steps each, back to back
    runs = []
    for _ in range(repeats):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(steps):
            kp.step(th, xi, yi, xb, yb, hp, info)
        t1.record()
        torch.cuda.synchronize()
        runs.append(t0.elapsed_time(t1) / steps)
    ms = sorted(runs)[len(runs) // 2]
    tm = kp.timing_read() if kernel_class is not None else None
    sweeps = kp.get_sweeps()
    status = kp.sync()
    last = KfacPinn.decode_info(info)
    last["jacobi_sweeps"] = sweeps
    last["repeats_ms_per_step"] = runs
    del kp
    return ms, tm, status, last


def run_batch(count, steps, warmup, use_graph, precision="bf16", grouped=True, tuned=False):
    """One step of `count` heterogeneous instances per call (the 64-instance
    recipe), as a captured graph or as direct launches on the internal lanes,
    with the grouped line search (one launch per kernel over every instance) or
    the per-instance one."""
    import numpy as np
    import torch
    import synth
    from paper_2405_15603_amd import KfacPinnBatch
    dev = torch.device("cuda", 0)
    probs = synth.batch_instances(count)
    T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float32, device=dev).contiguous()
    thetas = [T(p.theta0()) for p in probs]
    cols = list(zip(*[[T(a) for a in p.batch(0)] for p in probs]))
    b = KfacPinnBatch(probs, precision, use_graph=use_graph)
    b.set_grouped(grouped)
    timed_classes = b.tune(thetas, *cols) if tuned else 0
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
    was_grouped = b.is_grouped()
    del b
    return {"ms_per_step": ms, "instance_steps_per_s": count * 1000.0 / ms,
            "status_nonzero": sum(1 for v in status if v != 0), "grouped_line_search": was_grouped,
            "tuned_classes": timed_classes}


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


def blas_info():
    """The BLAS and LAPACK the oracle's PyTorch build links (from its build string)."""
    import torch
    cfg = torch.__config__.show()
    found = re.findall(r"(BLAS_INFO|LAPACK_INFO)=([^,\s]+)", cfg)
    return ", ".join(f"{k}={v}" for k, v in found) or "unknown"


def cpu_baseline(problem):
    """The FP64 oracle (plain PyTorch on the host cores) for one step of the same
    workload, timed in three parts whose cost is known to scale: the curvature part
    (forward Laplacian, autodiff backward, factors, gradient) on a 10 % sample of
    the points, scaled by 10 (every point's work is the same); the Kronecker-sum
    inverse of the resulting factors at full size (it does not depend on the point
    count); and one full-size line-search candidate loss, times the 31 candidates.
    The sum is the step time, extrapolated from those measurements.  Timed with all
    the host cores this process may use, and with one thread on smaller samples."""
    import torch
    import oracle
    op = oracle.operator_of(problem)
    h = hparams()
    hp = oracle.HParams(lam=h.lam, beta=h.beta, momentum=h.momentum, lr_mode="fixed", lr=0.0)
    th = problem.theta0()
    xi, yi, xb, yb = problem.batch(0)
    widths = problem.widths

    def leg(frac_curv, frac_loss):
        ns, ms = max(1, int(problem.n_interior * frac_curv)), max(1, int(problem.n_cond * frac_curv))
        st = oracle.init_state(widths, True)
        t0 = time.perf_counter()
        _, st1, info = oracle.kfac_step(th, widths, (xi[:ns], yi[:ns], xb[:ms], yb[:ms]), op, hp, st)
        t_step = time.perf_counter() - t0
        t0 = time.perf_counter()
        for l in range(len(widths) - 1):
            oracle.kron_sum_inverse(*(oracle.damp(m[l], hp.lam)
                                      for m in (st1.A_int, st1.B_int, st1.A_bnd, st1.B_bnd)))
        t_inv = time.perf_counter() - t0
        # kfac_step with a fixed step evaluates the loss once at the end: the part that
        # scales with the points is the step minus that loss and minus the inverse
        nl, ml = max(1, int(problem.n_interior * frac_loss)), max(1, int(problem.n_cond * frac_loss))
        t0 = time.perf_counter()
        oracle.loss(th, widths, xi[:nl], yi[:nl], xb[:ml], yb[:ml], op)
        t_loss = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.loss(th, widths, xi[:ns], yi[:ns], xb[:ms], yb[:ms], op)
        t_loss_sample = time.perf_counter() - t0
        t_curv = max(t_step - t_inv - t_loss_sample, 0.0)
        total = t_curv / frac_curv + t_inv + 31 * t_loss / frac_loss
        return total, {"curvature_sample_s": t_curv, "curvature_points": [ns, ms],
                       "inverse_s": t_inv, "loss_s": t_loss, "loss_points": [nl, ml]}

    cores = len(os.sched_getaffinity(0))
    prev = torch.get_num_threads()
    torch.set_num_threads(cores)
    t_all, parts_all = leg(0.1, 1.0)
    torch.set_num_threads(1)
    t_one, parts_one = leg(0.01, 0.1)
    torch.set_num_threads(prev)
    return {"value": 1.0 / t_all, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 oracle, {cores} threads: curvature part on {parts_all['curvature_points']} "
                       f"interior/boundary points ({parts_all['curvature_sample_s']:.1f} s, x10), "
                       f"full-size Kronecker-sum inverse ({parts_all['inverse_s']:.2f} s), one "
                       f"full-size candidate loss ({parts_all['loss_s']:.1f} s, x31): "
                       f"{t_all:.0f} s per step, extrapolated from these measurements"),
            "one_thread": {"value": 1.0 / t_one, "seconds_per_step": t_one, "parts": parts_one,
                           "note": "1 thread; curvature on 1 % of the points (x100), candidate "
                                   "loss on 10 % (x10, x31)"},
            "seconds_per_step": t_all, "parts": parts_all, "blas": blas_info(),
            "threads": cores}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="f16", choices=["bf16", "f16", "f32", "f64"],
                    help="bf16: BF16x3 curvature products; f16: FP16 curvature products "
                         "(both with a BF16 line search)")
    ap.add_argument("--workload", default="poisson100d")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison leg")
    ap.add_argument("--no-core", action="store_true", help="skip the fixed-step (core) leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch leg")
    ap.add_argument("--kernel", default="ls_layer", choices=list(KERNEL_CLASSES))
    ap.add_argument("--ls-lanes", type=int, default=2, choices=[1, 2],
                    help="streams for the line-search candidates in the timed run")
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed regions of --steps steps each; the headline is their median")
    ap.add_argument("--no-kfac-star", action="store_true", help="skip the KFAC* leg")
    ap.add_argument("--no-other-mixed", action="store_true",
                    help="skip the leg that times the other mixed-precision curvature path")
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
    log(f"headline: {args.repeats} x {args.steps} steps after {args.warmup} warm-up")
    ms, _, status, last = run_gpu(problem, args.precision, args.steps, args.warmup, None,
                                  ls_lanes=args.ls_lanes, repeats=args.repeats)
    log(f"headline done: {ms:.2f} ms per step (repeats {last['repeats_ms_per_step']})")
    if status != 0:
        print(f"device status {status} after the timed steps", file=sys.stderr)
        sys.exit(1)
    rsteps = max(1, min(args.steps, args.roofline_steps))
    log("one-lane run for the dominant kernel's launch durations")
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
        "dtype": {"bf16": "bf16", "f16": "f16", "f32": "f32", "f64": "f64"}[args.precision],
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
        traffic = (measured_traffic() if (args.kernel == "ls_layer" and args.precision in ("bf16", "f16"))
                   else None)
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
        log("core step (fixed step size)")
        msc, _, stc, _ = run_gpu(problem, args.precision, side_steps, 1, None, lr_mode="fixed")
        out["core_step"] = {"value": 1000.0 / msc, "ms_per_step": msc, "status": stc,
                            "note": "fixed step size 2^-5, no line search"}
    if not args.no_kfac_star:
        log("KFAC* step")
        msk, _, stk, lastk = run_gpu(problem, args.precision, side_steps, 2, None,
                                     lr_mode="kfac_star")
        out["kfac_star"] = {"value": 1000.0 / msk, "ms_per_step": msk, "status": stk,
                            "last_step": {k: lastk[k] for k in ("lr", "mu", "step", "status")},
                            "note": "KFAC*: learning rate and momentum from the 2 x 2 quadratic "
                                    "model with the exact damped Gramian (Section 3.4), no line "
                                    "search"}
    if args.precision in ("bf16", "f16") and not args.no_other_mixed:
        other = "f16" if args.precision == "bf16" else "bf16"
        log(f"other mixed path ({other})")
        mso, _, sto, _ = run_gpu(problem, other, side_steps, args.warmup, None)
        out["other_mixed"] = {"precision": other, "value": 1000.0 / mso, "ms_per_step": mso,
                              "status": sto,
                              "note": {"bf16": "BF16x3 curvature products (hi*hi + lo*hi + hi*lo)",
                                       "f16": "FP16 curvature products (slab rounded once, "
                                              "weights as FP16 hi + lo)"}[other]}
    if not args.no_fp32 and args.precision != "f32":
        log("FP32 path")
        ms32, _, st32, _ = run_gpu(problem, "f32", side_steps, 1, None)
        out["fp32"] = {"value": 1000.0 / ms32, "ms_per_step": ms32, "status": st32,
                       "mixed_over_fp32": ms32 / ms}
    if not args.no_batch:
        log("64-instance batch")
        bp = args.precision if args.precision in ("bf16", "f16") else "bf16"
        bw = args.warmup
        out["batch64"] = {"instances": 64, "note": "heterogeneous 64-instance recipe, mixed "
                          f"precision, grid line search; one step of every instance per call; "
                          f"3 timed steps after {bw} warm-up steps (the headline's), and the "
                          "first steps (after 1 warm-up, cold Jacobi start) for comparison",
                          "graph": run_batch(64, 3, bw, True, bp),
                          "graph_tuned": run_batch(64, 3, bw, True, bp, tuned=True),
                          "direct": run_batch(64, 3, bw, False, bp),
                          "graph_per_instance_line_search": run_batch(64, 3, bw, True, bp,
                                                                      grouped=False),
                          "graph_first_steps": run_batch(64, 3, 1, True, bp)}
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(problem)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
