"""Seeded synthetic inputs for the KFAC-PINN hot path.

This module generates *inputs only*: network parameters, collocation points and
their targets for the PDE problems of the paper's experiments (Section 4 and
Appendix A).  It holds none of the method's arithmetic (no forward Laplacian, no
curvature factors, no update).  Both the CPU oracle and the GPU tests/benchmark
draw their inputs from here, so the same seed gives the same bytes on both sides.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based generator:
value i of stream `seed` is  mix(seed + (i + 1) * GAMMA)  (mod 2**64), i.e. the
(i+1)-th output of the sequential generator started at state `seed`.  A uniform
double is the top 53 bits times 2**-53, so it lies in [0, 1) and is exact in FP64.
The GPU sampler implements the same published generator on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Stream purposes: the seed of a stream is 1000 * problem_id + purpose.
PURPOSE_WEIGHTS = 0
PURPOSE_INTERIOR = 1
PURPOSE_BOUNDARY = 2
PURPOSE_INITIAL = 3
PURPOSE_DIRECTIONS = 4
PURPOSE_INSTANCES = 5


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 outputs for the given 0-based counters of stream `seed`."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, start: int, count: int) -> np.ndarray:
    """`count` uniform doubles in [0, 1) from counters start .. start+count-1."""
    z = splitmix64(seed, np.arange(start, start + count, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ----------------------------------------------------------------------------
# Network parameters
# ----------------------------------------------------------------------------

def num_params(widths: Sequence[int]) -> int:
    """D = sum_l h_l (h_{l-1} + 1): weights plus one bias column per layer."""
    return int(sum(widths[l + 1] * (widths[l] + 1) for l in range(len(widths) - 1)))


def layer_offsets(widths: Sequence[int]) -> List[int]:
    off = [0]
    for l in range(len(widths) - 1):
        off.append(off[-1] + widths[l + 1] * (widths[l] + 1))
    return off


def init_theta(widths: Sequence[int], seed: int) -> np.ndarray:
    """Parameters in the paper's flattening (Section 2): per layer the augmented
    matrix [W | b] (h_out x (h_in+1)) is column-stacked, layers concatenated.
    Every entry of layer l is U(-1/sqrt(h_in), +1/sqrt(h_in)), drawn in that order."""
    D = num_params(widths)
    u = uniform(seed, 0, D)
    theta = np.empty(D, dtype=np.float64)
    off = layer_offsets(widths)
    for l in range(len(widths) - 1):
        bound = 1.0 / math.sqrt(widths[l])
        theta[off[l]:off[l + 1]] = (2.0 * u[off[l]:off[l + 1]] - 1.0) * bound
    return theta


# ----------------------------------------------------------------------------
# Collocation points
# ----------------------------------------------------------------------------

def sample_interior(seed: int, step: int, n: int, d: int) -> np.ndarray:
    """n points uniform in [0,1)^d; point i coordinate j uses counter step*n*d + i*d + j."""
    return uniform(seed, step * n * d, n * d).reshape(n, d)


def sample_boundary(seed: int, step: int, n: int, d: int, face_lo: int = 0) -> np.ndarray:
    """n points uniform on the faces x_k in {0,1}, k >= face_lo, of the unit cube.

    Point i uses d+1 counters starting at step*n*(d+1) + i*(d+1): the first picks
    the face f = floor(u * 2*(d-face_lo)) (coordinate face_lo + f//2 is set to f%2),
    the next d give the coordinates.  All faces have equal measure, so this is
    uniform on the (lateral) boundary."""
    u = uniform(seed, step * n * (d + 1), n * (d + 1)).reshape(n, d + 1)
    nf = 2 * (d - face_lo)
    f = np.minimum(np.floor(u[:, 0] * nf).astype(np.int64), nf - 1)
    x = u[:, 1:].copy()
    x[np.arange(n), face_lo + f // 2] = (f % 2).astype(np.float64)
    return x


def sample_initial(seed: int, step: int, n: int, d: int) -> np.ndarray:
    """n points with time coordinate 0 and the other d-1 coordinates uniform."""
    x = uniform(seed, step * n * d, n * d).reshape(n, d)
    x[:, 0] = 0.0
    return x


# ----------------------------------------------------------------------------
# Problems
# ----------------------------------------------------------------------------

POISSON = "poisson"
HEAT = "heat"
LOGFP = "logfp"   # logarithmic Fokker-Planck equation (Section 4, Appendix A)


@dataclass
class Problem:
    """A PDE problem with a manufactured solution and its network architecture.

    The interior residual is  r = c_t * du/dx_t + c_lap * sum_{i in mask} d2u/dx_i^2 - y
    (Poisson: -Laplace u = f, so c_lap = -1 and y = f; heat: u_t - kappa Lap_x u = 0).
    The boundary residual is  u - g."""
    name: str
    kind: str
    widths: List[int]
    n_interior: int
    n_boundary: int
    n_initial: int = 0
    kappa: float = 0.25
    scale: float = 1.0
    problem_id: int = 0
    resample: bool = False
    lam: float = 1e-3
    op_coef: Optional[np.ndarray] = None   # C of sum_ij C_ij d2/dx_i dx_j (None: the mask)

    @property
    def d(self) -> int:
        return self.widths[0]

    @property
    def time_coord(self) -> int:
        return 0 if self.kind in (HEAT, LOGFP) else -1

    @property
    def coef_time(self) -> float:
        return 1.0 if self.kind in (HEAT, LOGFP) else 0.0

    @property
    def coef_lap(self) -> float:
        return -self.kappa if self.kind == HEAT else -1.0

    # first-order terms of the residual: the logarithmic Fokker-Planck equation
    # d_t q - d_x/2 - (1/2) x . grad q - |grad q|^2 - Lap q = 0 (d_x spatial dims)
    @property
    def coef_xgrad(self) -> float:
        return -0.5 if self.kind == LOGFP else 0.0

    @property
    def coef_gradsq(self) -> float:
        return -1.0 if self.kind == LOGFP else 0.0

    @property
    def coef_const(self) -> float:
        return -0.5 * (self.d - 1) if self.kind == LOGFP else 0.0

    @property
    def lap_mask(self) -> np.ndarray:
        m = np.ones(self.d, dtype=np.uint8)
        if self.kind in (HEAT, LOGFP):
            m[0] = 0
        return m

    @property
    def n_cond(self) -> int:
        return self.n_boundary + self.n_initial

    def seed(self, purpose: int) -> int:
        return 1000 * self.problem_id + purpose

    # manufactured solutions -------------------------------------------------
    def u_star(self, x: np.ndarray) -> np.ndarray:
        if self.kind == LOGFP:
            # q* = log p*, p*(t) = N(0, s2(t) I) with s2(t) = e^-t + 2 (1 - e^-t)
            s2 = 2.0 - np.exp(-x[:, 0])
            k = self.d - 1
            return -0.5 * k * np.log(2 * math.pi * s2) - (x[:, 1:] ** 2).sum(1) / (2 * s2)
        if self.kind == HEAT:
            t = x[:, 0]
            return np.exp(-self.kappa * math.pi ** 2 * t) * np.sin(math.pi * x[:, 1:]).sum(1)
        if self.name == "poisson2d":
            return np.sin(math.pi * x[:, 0]) * np.sin(math.pi * x[:, 1])
        return self.scale * np.sin(math.pi * x).sum(1)

    def f_rhs(self, x: np.ndarray) -> np.ndarray:
        """Interior target y: f = -Lap u* for Poisson, 0 for heat; with a coefficient
        matrix C, f = -sum_ij C_ij d2u*/dx_i dx_j, which for u* = c sum sin(pi x_i)
        (no mixed derivatives) is c pi^2 sum_i C_ii sin(pi x_i)."""
        if self.kind in (HEAT, LOGFP):
            return np.zeros(x.shape[0])
        if self.op_coef is not None:
            return self.scale * math.pi ** 2 * (np.sin(math.pi * x) * np.diag(self.op_coef)).sum(1)
        if self.name == "poisson2d":
            return 2 * math.pi ** 2 * np.sin(math.pi * x[:, 0]) * np.sin(math.pi * x[:, 1])
        return self.scale * math.pi ** 2 * np.sin(math.pi * x).sum(1)

    def g_bnd(self, x: np.ndarray) -> np.ndarray:
        if self.name == "poisson2d":
            return np.zeros(x.shape[0])   # u* vanishes on the boundary of the square
        return self.u_star(x)

    # data -------------------------------------------------------------------
    def batch(self, step: int = 0):
        """(X_int, y_int, X_bnd, y_bnd) in FP64.  For the heat equation the
        condition set holds the initial points first, then the boundary points."""
        d = self.d
        st = step if self.resample else 0
        xi = sample_interior(self.seed(PURPOSE_INTERIOR), st, self.n_interior, d)
        if self.kind == LOGFP:
            # t in [0, 1), x in [-5, 5)^(d-1); the loss has the residual and the
            # initial condition q(0, .) = log p*(0, .) only (no spatial boundary)
            xi[:, 1:] = 10.0 * xi[:, 1:] - 5.0
            x0 = sample_initial(self.seed(PURPOSE_INITIAL), st, self.n_initial, d)
            x0[:, 1:] = 10.0 * x0[:, 1:] - 5.0
            return xi, self.f_rhs(xi), x0, self.u_star(x0)
        face_lo = 1 if self.kind == HEAT else 0
        xb = sample_boundary(self.seed(PURPOSE_BOUNDARY), st, self.n_boundary, d, face_lo)
        if self.n_initial:
            x0 = sample_initial(self.seed(PURPOSE_INITIAL), st, self.n_initial, d)
            xb = np.concatenate([x0, xb], 0)
        return xi, self.f_rhs(xi), xb, self.g_bnd(xb)

    def theta0(self) -> np.ndarray:
        return init_theta(self.widths, self.seed(PURPOSE_WEIGHTS))


def poisson2d() -> Problem:
    """2d Poisson, -Lap u = 2 pi^2 sin(pi x) sin(pi y), u = 0 on the boundary; 2->64->64->1."""
    return Problem("poisson2d", POISSON, [2, 64, 64, 1], 900, 120, problem_id=1)


def poisson5d() -> Problem:
    """5d Poisson with u* = sum sin(pi x_i); 5->64->64->48->48->1, resampled each step."""
    return Problem("poisson5d", POISSON, [5, 64, 64, 48, 48, 1], 3000, 500, problem_id=2,
                   resample=True)


def poisson100d() -> Problem:
    """100d Poisson with u* = sum sin(pi x_i)/100; 100->768->768->512->512->1."""
    return Problem("poisson100d", POISSON, [100, 768, 768, 512, 512, 1], 3000, 1000,
                   scale=1.0 / 100, problem_id=3)


def heat4d() -> Problem:
    """(4+1)d heat equation, kappa = 1/4, u* = exp(-kappa pi^2 t) sum sin(pi x_i);
    5->256->256->128->128->1; 4000 interior, 1000 boundary and 1000 initial points."""
    return Problem("heat4d", HEAT, [5, 256, 256, 128, 128, 1], 4000, 1000, n_initial=1000,
                   problem_id=4)


def log_fokker_planck(widths=(10, 256, 256, 128, 128, 1), n_int: int = 3000,
                      n_init: int = 1000, problem_id: int = 7) -> Problem:
    """(9+1)-d logarithmic Fokker-Planck equation of Section 4 / Appendix A:
    drift -x/2, diffusion sqrt(2) I, on [0, 1] x [-5, 5]^9; solution
    q* = log N(0, (2 - e^-t) I); 10->256->256->128->128->1 (D = 118 145)."""
    return Problem("logfp10d", LOGFP, list(widths), n_int, 0, n_initial=n_init,
                   problem_id=problem_id)


def anisotropic(d: int = 8, widths=None, n_int: int = 600, n_bnd: int = 160,
                problem_id: int = 6, scale: float = 1.0) -> Problem:
    """Poisson-type problem -sum_ij C_ij d2u/dx_i dx_j = f with a dense symmetric
    positive-definite C = B B^T / d + I/2 (B uniform in [-1, 1), seeded) and
    u* = c sum sin(pi x_i): the general second-order operator of the paper's
    Section 3.1 / Appendix C.3 on the unit cube."""
    u = uniform(1000 * problem_id + PURPOSE_INSTANCES, 0, d * d).reshape(d, d)
    B = 2.0 * u - 1.0
    C = B @ B.T / d + 0.5 * np.eye(d)
    widths = list(widths) if widths is not None else [d, 64, 64, 48, 48, 1]
    return Problem(f"aniso{d}d", POISSON, widths, n_int, n_bnd, problem_id=problem_id,
                   scale=scale, op_coef=C)


def small_problem(kind: str = POISSON, widths=(3, 8, 8, 1), n_int: int = 7, n_bnd: int = 5,
                  n_init: int = 0, problem_id: int = 90, scale: float = 1.0,
                  op_coef=None) -> Problem:
    """A tiny problem for pins and fast parity cases."""
    return Problem(f"small_{kind}", kind, list(widths), n_int, n_bnd, n_initial=n_init,
                   problem_id=problem_id, scale=scale, op_coef=op_coef)


def batch_instances(count: int = 64, seed: int = 5005) -> List[Problem]:
    """Heterogeneous Poisson instances: d in {2,5,10,20}, u* = c sum sin(pi x_i) with
    c ~ U[0.5, 2], N_int ~ U{500..4000}, N_bnd = ceil(N_int/6), width w in {64,128,256}
    and architecture d -> w -> w -> w' -> w' -> 1 with w' = 48 / 64 / 128."""
    u = uniform(seed, 0, 4 * count).reshape(count, 4)
    out = []
    for k in range(count):
        d = [2, 5, 10, 20][min(int(u[k, 0] * 4), 3)]
        c = 0.5 + 1.5 * u[k, 1]
        n = 500 + min(int(u[k, 2] * 3501), 3500)
        wi = min(int(u[k, 3] * 3), 2)
        w, w2 = [64, 128, 256][wi], [48, 64, 128][wi]
        p = Problem(f"inst{k}", POISSON, [d, w, w, w2, w2, 1], n, -(-n // 6), scale=c,
                    problem_id=10000 + k)
        out.append(p)
    return out


PROBLEMS = {"poisson2d": poisson2d, "poisson5d": poisson5d, "poisson100d": poisson100d,
            "heat4d": heat4d, "logfp10d": log_fokker_planck, "aniso8d": lambda: anisotropic()}
