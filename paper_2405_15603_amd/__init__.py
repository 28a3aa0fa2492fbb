"""MI355X (gfx950) KFAC for PINN losses.

Python binding of libkfac_pinn.so (include/kfac_pinn.h).  PyTorch provides device
memory and the HIP stream; every step of the computation runs in the library's
HIP kernels.  Method names follow the C entry points without the `kfac_pinn_`
prefix; the raw entry points are in `paper_2405_15603_amd._native`.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _native as N
from ._native import KP_F32, KP_F64, KP_MIXED_BF16, KP_MIXED_F16, KfacPinnError

PRECISIONS = {"f64": KP_F64, "f32": KP_F32, "bf16": KP_MIXED_BF16, "f16": KP_MIXED_F16}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclass
class HParams:
    """Hyper-parameters of one step (Section 3.4): damping lambda, EMA beta,
    momentum mu, and the learning rate: a grid line search over 2^k,
    k = grid_max_exp .. grid_min_exp ("grid"), a fixed step ("fixed"), or KFAC*'s
    automatic learning rate and momentum ("kfac_star"; mu is then unused)."""
    lam: float = 1e-3
    beta: float = 0.0
    momentum: float = 0.0
    lr_mode: str = "grid"
    lr: float = 1.0
    grid_min_exp: int = -30
    grid_max_exp: int = 0

    def c(self) -> N.kp_hparams:
        mode = {"fixed": 0, "grid": 1, "kfac_star": 2}[self.lr_mode]
        return N.kp_hparams(self.lam, self.beta, self.momentum, mode, self.lr, self.grid_min_exp,
                            self.grid_max_exp)


class KfacPinn:
    """One KFAC-PINN context: a tanh MLP with the given widths, an interior
    operator c_t d/dx_t + c_lap sum_{i in mask} d2/dx_i^2 (or, with op_coef = C,
    c_lap sum_ij C_ij d2/dx_i dx_j) and capacities."""

    def __init__(self, widths: Sequence[int], precision: str = "f32", time_coord: int = -1,
                 coef_time: float = 0.0, coef_lap: float = -1.0, lap_mask=None,
                 max_interior: int = 4096, max_boundary: int = 4096,
                 workspace_limit_bytes: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 op_coef=None, coef_xgrad: float = 0.0, coef_gradsq: float = 0.0,
                 coef_const: float = 0.0):
        if not torch.cuda.is_available():
            raise RuntimeError("KfacPinn needs a GPU (HIP device); there is no CPU path")
        self.lib = N.lib()
        self.widths = [int(w) for w in widths]
        self.L = len(self.widths) - 1
        self.d = self.widths[0]
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._w = (C.c_int32 * len(self.widths))(*self.widths)
        self._mask = None
        if lap_mask is not None:
            self._mask = (C.c_uint8 * self.d)(*[1 if m else 0 for m in lap_mask])
        self._coef = None
        if op_coef is not None:
            flat = [float(v) for row in op_coef for v in row]
            if len(flat) != self.d * self.d:
                raise ValueError("op_coef must be d x d")
            self._coef = (C.c_double * len(flat))(*flat)
            self._mask = None
        prob = N.kp_problem(self.L, self._w, time_coord, coef_time, coef_lap,
                            self._mask if self._mask is not None else None,
                            PRECISIONS[precision], max_interior, max_boundary,
                            workspace_limit_bytes, self._coef, coef_xgrad, coef_gradsq,
                            coef_const)
        h = C.c_void_p()
        N.check(self.lib.kfac_pinn_create(C.byref(prob), C.c_void_p(self.stream.cuda_stream),
                                          C.byref(h)), "kfac_pinn_create")
        self.h = h
        self.D = int(self.lib.kfac_pinn_num_params(self._w, self.L))
        self.max_interior, self.max_boundary = max_interior, max_boundary

    @classmethod
    def for_problem(cls, problem, precision="f32", **kw):
        """Context for a problem description (synthetic workloads carry widths,
        operator coefficients and point counts)."""
        kw.setdefault("max_interior", problem.n_interior)
        kw.setdefault("max_boundary", problem.n_cond)
        coef = getattr(problem, "op_coef", None)
        if coef is not None:
            kw.setdefault("op_coef", [list(r) for r in coef])
        for k in ("coef_xgrad", "coef_gradsq", "coef_const"):
            kw.setdefault(k, getattr(problem, k, 0.0))
        return cls(problem.widths, precision, problem.time_coord, problem.coef_time,
                   problem.coef_lap, None if coef is not None else list(problem.lap_mask), **kw)

    @classmethod
    def _borrow(cls, handle: C.c_void_p, widths, precision: str, max_interior: int,
                max_boundary: int, stream) -> "KfacPinn":
        """A view of a context owned elsewhere (an instance of a batch)."""
        self = cls.__new__(cls)
        self.lib = N.lib()
        self.widths = [int(w) for w in widths]
        self.L = len(self.widths) - 1
        self.d = self.widths[0]
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream
        self._w = (C.c_int32 * len(self.widths))(*self.widths)
        self.h = handle
        self._owned = False
        self.D = int(self.lib.kfac_pinn_num_params(self._w, self.L))
        self.max_interior, self.max_boundary = max_interior, max_boundary
        return self

    def __del__(self):
        if not getattr(self, "_owned", True):
            return
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize()
                self.lib.kfac_pinn_destroy(h)
            except Exception:
                pass
            self.h = None

    # -- helpers -------------------------------------------------------------
    def _real(self, t: torch.Tensor, name: str) -> torch.Tensor:
        if t.device.type != "cuda" or t.dtype != self.dtype or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {self.dtype} CUDA tensor")
        return t

    def empty(self, *shape, dtype=None) -> torch.Tensor:
        return torch.empty(*shape, dtype=dtype or self.dtype, device=self.device)

    # -- entry points --------------------------------------------------------
    def reset_state(self, init_identity: bool = True) -> None:
        N.check(self.lib.kfac_pinn_reset_state(self.h, 1 if init_identity else 0),
                "kfac_pinn_reset_state")

    def sample(self, sampler: N.kp_sampler, step: int, n_int: int, n_cond: int):
        xi, yi = self.empty(n_int, self.d), self.empty(n_int)
        xb, yb = self.empty(n_cond, self.d), self.empty(n_cond)
        N.check(self.lib.kfac_pinn_sample(self.h, C.byref(sampler), step, _ptr(xi), _ptr(yi),
                                          _ptr(xb), _ptr(yb)), "kfac_pinn_sample")
        return xi, yi, xb, yb

    def forward_laplacian(self, theta: torch.Tensor, x: torch.Tensor):
        theta, x = self._real(theta, "theta"), self._real(x, "x")
        n = x.shape[0]
        u, g, lap = self.empty(n), self.empty(n, self.d), self.empty(n)
        N.check(self.lib.kfac_pinn_forward_laplacian(self.h, _ptr(theta), _ptr(x), n, _ptr(u),
                                                     _ptr(g), _ptr(lap)),
                "kfac_pinn_forward_laplacian")
        return u, g, lap

    def forward_laplacian_vjp(self, theta, x, u_bar=None, grad_bar=None, lap_bar=None,
                              want_x_bar=True):
        theta, x = self._real(theta, "theta"), self._real(x, "x")
        n = x.shape[0]
        tb = self.empty(self.D, dtype=torch.float64)
        xb = self.empty(n, self.d) if want_x_bar else None
        args = [None if a is None else self._real(a, nm)
                for a, nm in ((u_bar, "u_bar"), (grad_bar, "grad_bar"), (lap_bar, "lap_bar"))]
        N.check(self.lib.kfac_pinn_forward_laplacian_vjp(self.h, _ptr(theta), _ptr(x), n,
                                                         *[_ptr(a) for a in args], _ptr(tb),
                                                         _ptr(xb)),
                "kfac_pinn_forward_laplacian_vjp")
        return tb, xb

    def factors(self, theta, xi, yi, xb, yb, beta: float = 0.0):
        grad = self.empty(self.D, dtype=torch.float64)
        loss = self.empty(2, dtype=torch.float64)
        N.check(self.lib.kfac_pinn_factors(self.h, _ptr(theta), _ptr(xi), _ptr(yi), xi.shape[0],
                                           _ptr(xb), _ptr(yb), xb.shape[0], beta, _ptr(grad),
                                           _ptr(loss)), "kfac_pinn_factors")
        return grad, loss

    def invert(self, lam: float) -> None:
        N.check(self.lib.kfac_pinn_invert(self.h, lam), "kfac_pinn_invert")

    def set_max_sweeps(self, max_sweeps: int) -> None:
        """Sweep cap of the Jacobi eigensolver (1..64)."""
        N.check(self.lib.kfac_pinn_set_max_sweeps(self.h, int(max_sweeps)),
                "kfac_pinn_set_max_sweeps")

    def set_sweep_wait(self, enabled: bool) -> None:
        """Early stop of the Jacobi sweeps with host waits (default on); off: every
        inversion enqueues the full sweep cap without waiting.  Same results."""
        N.check(self.lib.kfac_pinn_set_sweep_wait(self.h, int(bool(enabled))),
                "kfac_pinn_set_sweep_wait")

    def layer_gramian(self, layer: int, term: int, n: int) -> torch.Tensor:
        """Exact Gramian block of `layer` for one term (0 interior, 1 boundary) from
        the last curvature pass, which had n points of that term."""
        p = self.widths[layer + 1] * (self.widths[layer] + 1)
        out = self.empty(p, p, dtype=torch.float64)
        work = self.empty(max(n, 1), p, dtype=torch.float64)
        N.check(self.lib.kfac_pinn_layer_gramian(self.h, layer, term, _ptr(out), _ptr(work)),
                "kfac_pinn_layer_gramian")
        return out

    def check_guards(self) -> tuple:
        """(guard bytes overwritten, guarded buffers); (0, 0) without guards."""
        bad, n = C.c_int64(), C.c_int64()
        N.check(self.lib.kfac_pinn_check_guards(self.h, C.byref(bad), C.byref(n)),
                "kfac_pinn_check_guards")
        return int(bad.value), int(n.value)

    def precondition(self, grad: torch.Tensor) -> torch.Tensor:
        out = self.empty(self.D, dtype=torch.float64)
        N.check(self.lib.kfac_pinn_precondition(self.h, _ptr(grad), _ptr(out)),
                "kfac_pinn_precondition")
        return out

    def step(self, theta, xi, yi, xb, yb, hp: HParams, info: Optional[torch.Tensor] = None):
        """One KFAC step; theta is updated in place.  Returns the device step
        summary as 6 doubles' worth of bytes (use `decode_info`)."""
        self._real(theta, "theta")
        if info is None:
            info = self.empty(C.sizeof(N.kp_step_info), dtype=torch.uint8)
        hpc = hp.c()
        N.check(self.lib.kfac_pinn_step(self.h, _ptr(theta), _ptr(xi), _ptr(yi), xi.shape[0],
                                        _ptr(xb), _ptr(yb), xb.shape[0], C.byref(hpc),
                                        _ptr(info)), "kfac_pinn_step")
        return info

    @staticmethod
    def decode_info(info: torch.Tensor) -> dict:
        raw = bytes(info.cpu().numpy().tobytes())
        s = N.kp_step_info.from_buffer_copy(raw)
        return {"loss_interior": s.loss_interior, "loss_boundary": s.loss_boundary,
                "lr": s.lr_chosen, "loss_after": s.loss_after, "status": s.status,
                "step": s.step, "mu": s.momentum_chosen}

    def get_factor(self, layer: int, term: int, side: int) -> torch.Tensor:
        n = self.widths[layer] + 1 if side == 0 else self.widths[layer + 1]
        out = self.empty(n, n, dtype=torch.float64)
        N.check(self.lib.kfac_pinn_get_factor(self.h, layer, term, side, _ptr(out)),
                "kfac_pinn_get_factor")
        return out

    def set_factor(self, layer: int, term: int, side: int, value: torch.Tensor) -> None:
        value = value.to(device=self.device, dtype=torch.float64).contiguous()
        N.check(self.lib.kfac_pinn_set_factor(self.h, layer, term, side, _ptr(value)),
                "kfac_pinn_set_factor")
        self.sync()

    def get_preconditioner(self, layer: int, side: int):
        n = self.widths[layer] + 1 if side == 0 else self.widths[layer + 1]
        P, e = self.empty(n, n, dtype=torch.float64), self.empty(n, dtype=torch.float64)
        N.check(self.lib.kfac_pinn_get_preconditioner(self.h, layer, side, _ptr(P), _ptr(e)),
                "kfac_pinn_get_preconditioner")
        return P, e

    def get_line_search(self, ncand: int = 31) -> torch.Tensor:
        out = self.empty(ncand, dtype=torch.float64)
        N.check(self.lib.kfac_pinn_get_line_search(self.h, _ptr(out)), "kfac_pinn_get_line_search")
        return out

    def get_momentum(self) -> torch.Tensor:
        out = self.empty(self.D)
        N.check(self.lib.kfac_pinn_get_momentum(self.h, _ptr(out)), "kfac_pinn_get_momentum")
        return out

    def set_momentum(self, delta: torch.Tensor, step: int) -> None:
        N.check(self.lib.kfac_pinn_set_momentum(self.h, _ptr(self._real(delta, "delta")), step),
                "kfac_pinn_set_momentum")

    def timing_enable(self, kernel_class: int) -> None:
        N.check(self.lib.kfac_pinn_timing_enable(self.h, kernel_class), "kfac_pinn_timing_enable")

    def timing_read(self) -> dict:
        out = (C.c_double * 4)()
        N.check(self.lib.kfac_pinn_timing_read(self.h, out), "kfac_pinn_timing_read")
        return {"launches": int(out[0]), "ms": out[1], "flops": out[2], "bytes": out[3]}

    def set_line_search_lanes(self, lanes: int) -> None:
        """1 or 2 streams for the grid line search's candidates (results unchanged)."""
        N.check(self.lib.kfac_pinn_set_line_search_lanes(self.h, int(lanes)),
                "kfac_pinn_set_line_search_lanes")

    def get_sweeps(self) -> list:
        out = (C.c_int32 * (2 * self.L))()
        N.check(self.lib.kfac_pinn_get_sweeps(self.h, out), "kfac_pinn_get_sweeps")
        return list(out)

    def recompute_mode(self) -> tuple:
        """(interior, boundary): True where layer inputs are recomputed per layer."""
        out = (C.c_int32 * 2)()
        N.check(self.lib.kfac_pinn_get_workspace(self.h, out), "kfac_pinn_get_workspace")
        return bool(out[0]), bool(out[1])

    def sync(self) -> int:
        """Waits for the stream; returns (and clears) the device status word."""
        return int(self.lib.kfac_pinn_sync(self.h))


class ForwardLaplacian(torch.autograd.Function):
    """(u, du/dx, masked Laplacian) = forward Laplacian of the network at x, with
    the hand-written adjoint of the library as its backward."""

    @staticmethod
    def forward(ctx, theta, x, kp: KfacPinn):
        u, g, lap = kp.forward_laplacian(theta.detach().contiguous(), x.detach().contiguous())
        ctx.kp = kp
        ctx.save_for_backward(theta, x)
        return u, g, lap

    @staticmethod
    def backward(ctx, u_bar, grad_bar, lap_bar):
        theta, x = ctx.saved_tensors
        kp = ctx.kp
        cast = lambda t: None if t is None else t.to(kp.dtype).contiguous()
        tb, xb = kp.forward_laplacian_vjp(theta.detach().contiguous(), x.detach().contiguous(),
                                          cast(u_bar), cast(grad_bar), cast(lap_bar),
                                          want_x_bar=ctx.needs_input_grad[1])
        return tb.to(theta.dtype), (xb if ctx.needs_input_grad[1] else None), None


class KfacPinnBatch:
    """Many independent problems stepped together (kfac_pinn_batch_*): one
    context per problem on internal lanes, the batch step captured into a HIP
    graph on the first call and replayed afterwards."""

    def __init__(self, problems, precision: str = "bf16", use_graph: bool = True,
                 stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("KfacPinnBatch needs a GPU (HIP device); there is no CPU path")
        self.lib = N.lib()
        self.problems = list(problems)
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        n = len(self.problems)
        self._keep = []
        arr = (N.kp_problem * n)()
        for k, p in enumerate(self.problems):
            w = (C.c_int32 * len(p.widths))(*p.widths)
            m = (C.c_uint8 * p.d)(*[1 if v else 0 for v in p.lap_mask])
            self._keep += [w, m]
            coef = getattr(p, "op_coef", None)
            cf = None
            if coef is not None:
                cf = (C.c_double * (p.d * p.d))(*[float(v) for r in coef for v in r])
                self._keep.append(cf)
                m = None
            arr[k] = N.kp_problem(len(p.widths) - 1, w, p.time_coord, p.coef_time, p.coef_lap, m,
                                  PRECISIONS[precision], p.n_interior, p.n_cond, 0, cf,
                                  getattr(p, "coef_xgrad", 0.0), getattr(p, "coef_gradsq", 0.0),
                                  getattr(p, "coef_const", 0.0))
        h = C.c_void_p()
        N.check(self.lib.kfac_pinn_batch_create(arr, n, C.c_void_p(self.stream.cuda_stream),
                                                C.byref(h)), "kfac_pinn_batch_create")
        self.h = h
        self.set_graph(use_graph)
        self.contexts = []
        for k, p in enumerate(self.problems):
            ch = C.c_void_p()
            N.check(self.lib.kfac_pinn_batch_context(self.h, k, C.byref(ch)),
                    "kfac_pinn_batch_context")
            self.contexts.append(KfacPinn._borrow(ch, p.widths, precision, p.n_interior, p.n_cond,
                                                  self.stream))

    def __len__(self):
        return len(self.problems)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize()
                self.lib.kfac_pinn_batch_destroy(h)
            except Exception:
                pass
            self.h = None

    def set_graph(self, enabled: bool) -> None:
        N.check(self.lib.kfac_pinn_batch_set_graph(self.h, 1 if enabled else 0),
                "kfac_pinn_batch_set_graph")

    def set_grouped(self, enabled: bool) -> None:
        N.check(self.lib.kfac_pinn_batch_set_grouped(self.h, 1 if enabled else 0),
                "kfac_pinn_batch_set_grouped")

    def _grouped_bits(self) -> int:
        v = C.c_int32()
        N.check(self.lib.kfac_pinn_batch_is_grouped(self.h, C.byref(v)), "kfac_pinn_batch_is_grouped")
        return v.value

    def is_grouped(self) -> bool:
        """Whether the last step took the grouped line search."""
        return bool(self._grouped_bits() & 1)

    def grouped_two_lanes(self) -> bool:
        """Whether the last step's grouped line search ran on two lanes."""
        return bool(self._grouped_bits() & 4)

    def grouped_products(self) -> bool:
        """Whether the last step took the grouped factor and gradient products."""
        return bool(self._grouped_bits() & 2)

    def step(self, thetas, xi, yi, xb, yb, hp: HParams, infos: Optional[torch.Tensor] = None):
        """One step of every instance; lists of tensors per instance.  `infos`
        (device bytes, len * sizeof(kp_step_info)) receives the summaries."""
        n = len(self.problems)
        V = C.c_void_p * n
        I = C.c_int32 * n
        hpc = hp.c()
        N.check(self.lib.kfac_pinn_batch_step(
            self.h, V(*[t.data_ptr() for t in thetas]), V(*[t.data_ptr() for t in xi]),
            V(*[t.data_ptr() for t in yi]), I(*[t.shape[0] for t in xi]),
            V(*[t.data_ptr() for t in xb]), V(*[t.data_ptr() for t in yb]),
            I(*[t.shape[0] for t in xb]), C.byref(hpc), _ptr(infos)), "kfac_pinn_batch_step")

    def tune(self, thetas, xi, yi, xb, yb, cache_path: Optional[str] = None) -> int:
        """Chunk counts of the grouped line search by timing (kfac_pinn_batch_tune);
        returns the number of classes timed (the rest came from the cache)."""
        n = len(self.problems)
        V = C.c_void_p * n
        I = C.c_int32 * n
        timed = C.c_int32()
        N.check(self.lib.kfac_pinn_batch_tune(
            self.h, V(*[t.data_ptr() for t in thetas]), V(*[t.data_ptr() for t in xi]),
            V(*[t.data_ptr() for t in yi]), I(*[t.shape[0] for t in xi]),
            V(*[t.data_ptr() for t in xb]), V(*[t.data_ptr() for t in yb]),
            I(*[t.shape[0] for t in xb]), cache_path.encode() if cache_path else None,
            C.byref(timed)), "kfac_pinn_batch_tune")
        return timed.value

    def sync(self) -> list:
        return [c.sync() for c in self.contexts]

    def get_sweeps(self, k: int) -> list:
        """Jacobi sweeps of instance k's eigenproblems in the last batch step."""
        n = 2 * (len(self.problems[k].widths) - 1)
        out = (C.c_int32 * n)()
        N.check(self.lib.kfac_pinn_batch_get_sweeps(self.h, k, out), "kfac_pinn_batch_get_sweeps")
        return list(out)


def forward_laplacian(kp: KfacPinn, theta: torch.Tensor, x: torch.Tensor):
    return ForwardLaplacian.apply(theta, x, kp)


def sampler_for(problem, step_counts=None) -> N.kp_sampler:
    """The GPU sampler's description of a synthetic problem's point sets."""
    from synth import PURPOSE_BOUNDARY, PURPOSE_INITIAL, PURPOSE_INTERIOR
    kind = 2 if problem.kind == "heat" else (1 if problem.name == "poisson2d" else 0)
    return N.kp_sampler(problem.seed(PURPOSE_INTERIOR), problem.seed(PURPOSE_BOUNDARY),
                        problem.seed(PURPOSE_INITIAL), problem.n_interior, problem.n_boundary,
                        problem.n_initial, 1 if problem.kind == "heat" else 0, kind,
                        problem.scale, problem.kappa)
