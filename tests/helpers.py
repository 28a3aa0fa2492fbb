"""Shared helpers for the parity tests: run the oracle on the same (rounded)
inputs the GPU path receives, and compare with norm-wise relative errors."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import synth

DEV = "cuda"


def rel(a, b) -> float:
    a = np.asarray(a.detach().cpu() if isinstance(a, torch.Tensor) else a, dtype=np.float64)
    b = np.asarray(b.detach().cpu() if isinstance(b, torch.Tensor) else b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rounded(a, precision: str) -> np.ndarray:
    """The value the GPU path receives (FP32 master data outside the FP64 path)."""
    a = np.asarray(a, dtype=np.float64)
    return a if precision == "f64" else a.astype(np.float32).astype(np.float64)


def to_dev(a, precision: str) -> torch.Tensor:
    dt = torch.float64 if precision == "f64" else torch.float32
    return torch.as_tensor(np.asarray(a), dtype=dt, device=DEV).contiguous()


def problem_inputs(p: "synth.Problem", precision: str, n_int=None, n_bnd=None, step=0):
    th = rounded(p.theta0(), precision)
    xi, yi, xb, yb = (rounded(a, precision) for a in p.batch(step))
    if n_int is not None:
        xi, yi = xi[:n_int], yi[:n_int]
    if n_bnd is not None:
        xb, yb = xb[:n_bnd], yb[:n_bnd]
    return th, xi, yi, xb, yb


def oracle_curvature(p, th, xi, yi, xb, yb):
    op = oracle.operator_of(p)
    Ws = oracle.unpack(torch.as_tensor(th), p.widths)
    ci = oracle.interior_curvature_inputs(Ws, torch.as_tensor(xi), torch.as_tensor(yi), op)
    cb = oracle.boundary_curvature_inputs(Ws, torch.as_tensor(xb), torch.as_tensor(yb))
    Ai, Bi = oracle.interior_factors(ci)
    Ab, Bb = oracle.boundary_factors(cb)
    grad, li, lb = oracle.loss_gradient(th, p.widths, xi, yi, xb, yb, op)
    return {"A_int": Ai, "B_int": Bi, "A_bnd": Ab, "B_bnd": Bb, "grad": grad, "loss": (li, lb)}


def blockwise(a, b, block: int = 64) -> float:
    """Elementwise companion of `rel`: for each block of `block` rows (points, or
    factor rows; a matrix is split along its first axis) the largest |a - b| over
    the largest |b| of that block; returns the worst block.  A wrong edge tile
    whose entries are small hides in a norm-wise error but not here."""
    a = np.asarray(a.detach().cpu() if isinstance(a, torch.Tensor) else a, dtype=np.float64)
    b = np.asarray(b.detach().cpu() if isinstance(b, torch.Tensor) else b, dtype=np.float64)
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    worst = 0.0
    for r in range(0, b.shape[0], block):
        d = np.abs(a[r:r + block] - b[r:r + block]).max()
        m = np.abs(b[r:r + block]).max()
        worst = max(worst, float(d / m) if m > 0 else float(d))
    return worst


def oracle_factors_chunked(p, th, xi, yi, xb, yb, chunk: int = 250):
    """The oracle's factors over the whole point set, assembled from chunks of
    points (each point's rows enter the sums independently): each chunk's
    normalised factors are multiplied back by its point count (times S for A_int),
    summed, and divided by the totals.  Only the oracle's own functions compute."""
    op = oracle.operator_of(p)
    Ws = oracle.unpack(torch.as_tensor(th), p.widths)
    L = len(p.widths) - 1
    S = p.d + 2
    sums = {k: [0.0] * L for k in ("A_int", "B_int", "A_bnd", "B_bnd")}
    N, M = xi.shape[0], xb.shape[0]
    for c0 in range(0, N, chunk):
        n = min(chunk, N - c0)
        ci = oracle.interior_curvature_inputs(Ws, torch.as_tensor(xi[c0:c0 + n]),
                                              torch.as_tensor(yi[c0:c0 + n]), op)
        A, B = oracle.interior_factors(ci)
        for l in range(L):
            sums["A_int"][l] = sums["A_int"][l] + A[l] * (n * S)
            sums["B_int"][l] = sums["B_int"][l] + B[l] * n
    for c0 in range(0, M, chunk):
        m = min(chunk, M - c0)
        cb = oracle.boundary_curvature_inputs(Ws, torch.as_tensor(xb[c0:c0 + m]),
                                              torch.as_tensor(yb[c0:c0 + m]))
        A, B = oracle.boundary_factors(cb)
        for l in range(L):
            sums["A_bnd"][l] = sums["A_bnd"][l] + A[l] * m
            sums["B_bnd"][l] = sums["B_bnd"][l] + B[l] * m
    return {"A_int": [a / (N * S) for a in sums["A_int"]], "B_int": [b / N for b in sums["B_int"]],
            "A_bnd": [a / M for a in sums["A_bnd"]], "B_bnd": [b / M for b in sums["B_bnd"]]}


def oracle_forward_chunked(p, th, x, chunk: int = 500):
    """Oracle forward-Laplacian output rows (N, S) over all points, by chunks."""
    op = oracle.operator_of(p)
    Ws = oracle.unpack(torch.as_tensor(th), p.widths)
    outs = [oracle.forward_laplacian(Ws, torch.as_tensor(x[c0:c0 + chunk]), op.mask_vec(p.d)).out
            for c0 in range(0, x.shape[0], chunk)]
    return torch.cat(outs, 0)


def check_bf16_candidates(ls, ref, alpha, tol: float = 5e-2, band: float = 10.0) -> dict:
    """Line-search candidates of the BF16 path (losses L(theta + 2^-k dhat), k = 0..30)
    against the oracle's FP64 losses `ref`.  BF16 rounds every slab entry and weight
    at 2^-9; through four layers and a squared residual that bounds a candidate's
    error at `tol` where the loss is well conditioned.  At steps far too large the
    updated weights saturate the tanh units: s1 = 1 - t^2 cancels to zero in reduced
    precision while the oracle keeps its tiny value times squared derivatives that
    the same steps made huge, so those losses are ill-conditioned in any precision
    below FP64.  Hence: candidates within `band` times the oracle's best loss must
    match to `tol`; the others must rank above the best GPU candidate (they cannot
    be chosen); the chosen step's oracle loss must be within `tol` of the best."""
    ls = np.asarray(ls, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    best = ref.min()
    err = np.abs(ls - ref) / np.abs(ref)
    near = ref <= band * best
    assert np.all(np.isfinite(ls[near])), ls
    assert np.all(err[near] < tol), (err, near)
    far = ~near
    assert np.all(~(ls[far] <= ls[near].min())), (ls, ref)
    k_star = -int(round(np.log2(alpha)))
    assert ref[k_star] <= best * (1 + tol), (k_star, ref)
    return {"near": int(near.sum()), "worst_near": float(err[near].max()),
            "worst_far": float(err[far].max()) if far.any() else 0.0}
