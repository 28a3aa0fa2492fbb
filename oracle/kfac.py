"""FP64 CPU oracle for one KFAC step on a PINN loss.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The product path never calls it, and it
shares no code with the HIP implementation.

Everything is plain PyTorch on the CPU in float64 (the paper runs all of its
experiments in double precision, Section 4).  Each function follows one passage
of Dangel, Mueller & Zeinhofer, "Kronecker-Factored Approximate Curvature for
Physics-Informed Neural Networks" (NeurIPS 2024), cited in its docstring:

* parameters: Section 2 (column-stacking flattening, bias as an extra column);
* forward Laplacian: Section 3.1, Eq. (forward-laplacian-main), with the bias row
  of Appendix C.2, Eq. (forward-laplacian-linear-layer-compact);
* PINN loss and residuals: Section 2.1, Eq. (pinn-loss); heat equation:
  Appendix A (PINN loss for the heat equation);
* layer output gradients g and the loss gradient: Algorithm 1 (Appendix B), which
  takes both from automatic differentiation -- so does this oracle;
* Kronecker factors: Section 3.2, Eq. (KFAC-PINN) for the interior term and
  Eq. (kfac-linear) for the boundary term;
* EMA, damping, Kronecker-sum inverse, momentum, line search: Section 3.4 and
  Algorithm 1; the Kronecker-sum inverse follows Martens & Grosse (2015), App. I,
  which the paper cites: symmetric inverse square roots of the first pair of
  factors, then eigendecompositions of the whitened second pair.

Readings of passages the paper leaves open are listed in the design notes; the
ones that change arithmetic are repeated where they are used.

parity unpinned: multi-step trajectories (chaotic under rounding; only the step
at a given parameter vector and batch is pinned).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

DT = torch.float64


# ----------------------------------------------------------------------------
# Activations (the method uses tanh; sin, cos and identity serve the pins)
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Activation:
    name: str

    def f(self, a):
        return {"tanh": torch.tanh, "sin": torch.sin, "cos": torch.cos,
                "identity": lambda x: x}[self.name](a)

    def d1(self, a):
        if self.name == "tanh":
            t = torch.tanh(a)
            return 1.0 - t * t
        if self.name == "sin":
            return torch.cos(a)
        if self.name == "cos":
            return -torch.sin(a)
        return torch.ones_like(a)

    def d2(self, a):
        if self.name == "tanh":
            t = torch.tanh(a)
            return -2.0 * t * (1.0 - t * t)
        if self.name == "sin":
            return -torch.sin(a)
        if self.name == "cos":
            return -torch.cos(a)
        return torch.zeros_like(a)


TANH = Activation("tanh")


@dataclass(frozen=True)
class Operator:
    """Interior operator  c_t d/dx_t + c_lap sum_{i,j} C_ij d^2/dx_i dx_j.

    C = diag(mask) unless a coefficient matrix is given (Section 3.1, closing
    paragraph; Appendix C.3: a weighted sum of second derivatives).
    Poisson (Section 2.1 writes -Lap u = f): c_t = 0, c_lap = -1, C = I.
    Heat (Appendix A, x_1 = t): c_t = 1, c_lap = -kappa, mask excludes t."""
    time_coord: int = -1
    coef_time: float = 0.0
    coef_lap: float = -1.0
    mask: Optional[Sequence[int]] = None
    coef: Optional[Sequence[Sequence[float]]] = None   # C, d x d symmetric
    # first-order terms (Section 3.3): sum_{i in mask} (c_x x_i d_i u + c_g (d_i u)^2) + c_0
    coef_xgrad: float = 0.0
    coef_gradsq: float = 0.0
    coef_const: float = 0.0

    def mask_vec(self, d: int) -> torch.Tensor:
        if self.mask is None:
            return torch.ones(d, dtype=DT)
        return torch.as_tensor(np.asarray(self.mask, dtype=np.float64))

    def second_order(self, d: int) -> torch.Tensor:
        """What the forward pass sums over: the mask vector (a diagonal C) or the
        coefficient matrix C."""
        if self.coef is None:
            return self.mask_vec(d)
        return torch.as_tensor(np.asarray(self.coef, dtype=np.float64))


POISSON_OP = Operator()


def operator_of(problem) -> Operator:
    coef = getattr(problem, "op_coef", None)
    if coef is not None:
        coef = tuple(tuple(float(v) for v in row) for row in np.asarray(coef))
    return Operator(problem.time_coord, problem.coef_time, problem.coef_lap,
                    tuple(int(v) for v in problem.lap_mask), coef,
                    getattr(problem, "coef_xgrad", 0.0), getattr(problem, "coef_gradsq", 0.0),
                    getattr(problem, "coef_const", 0.0))


# ----------------------------------------------------------------------------
# Parameters (Section 2: theta^(l) = vec [W | b], column-stacked)
# ----------------------------------------------------------------------------

def num_params(widths: Sequence[int]) -> int:
    return sum(widths[l + 1] * (widths[l] + 1) for l in range(len(widths) - 1))


def unpack(theta: torch.Tensor, widths: Sequence[int]) -> List[torch.Tensor]:
    """Augmented weights W~^(l) = [W | b] of shape h_out x (h_in+1).  Column stacking
    means the flat segment holds column j at [j*h_out, (j+1)*h_out)."""
    Ws, off = [], 0
    for l in range(len(widths) - 1):
        hi, ho = widths[l], widths[l + 1]
        seg = theta[off:off + ho * (hi + 1)]
        Ws.append(seg.reshape(hi + 1, ho).T)
        off += ho * (hi + 1)
    assert off == theta.numel()
    return Ws


def pack(mats: Sequence[torch.Tensor]) -> torch.Tensor:
    """Inverse of `unpack`: column-stack every h_out x (h_in+1) matrix."""
    return torch.cat([m.T.reshape(-1) for m in mats])


# ----------------------------------------------------------------------------
# Forward Laplacian (Section 3.1, Eq. forward-laplacian-main; Appendix C.2)
# ----------------------------------------------------------------------------

def input_slab(X: torch.Tensor) -> torch.Tensor:
    """Z^(0)_n with S = d+2 rows per point (Section 3.1 / 3.2): the value x_n,
    the d first derivatives d x/d x_i = e_i, and the Laplacian row 0.
    Stored as (N, S, d): index s runs over the shared columns of Z_n."""
    N, d = X.shape
    Z = torch.zeros(N, d + 2, d, dtype=DT)
    Z[:, 0, :] = X
    Z[:, 1:d + 1, :] = torch.eye(d, dtype=DT)
    return Z


def augment(Z: torch.Tensor) -> torch.Tensor:
    """Append the bias feature (Eq. forward-laplacian-linear-layer-compact): 1 in
    the value row, 0 in the derivative and Laplacian rows.  A 2-d input (M, h) is a
    plain batch of values and gets a 1 everywhere."""
    if Z.dim() == 2:
        return torch.cat([Z, torch.ones(Z.shape[0], 1, dtype=DT)], -1)
    one = torch.zeros(Z.shape[0], Z.shape[1], 1, dtype=DT)
    one[:, 0, 0] = 1.0
    return torch.cat([Z, one], -1)


def activation_rows(a: torch.Tensor, mask: torch.Tensor, act: Activation) -> torch.Tensor:
    """Elementwise layer on the stacked rows (Eq. forward-laplacian-main, second line,
    restricted to the coordinates in `mask` for a partial Laplacian):
        v = s(a0),  d_i v = s'(a0) d_i a,  Lv = s'(a0) La + s''(a0) sum_{i in M} (d_i a)^2.
    With a coefficient matrix C in place of the mask (Appendix C.3), the collapsed
    second-order row is  s'(a0) La + s''(a0) sum_{i,j} C_ij d_i a d_j a."""
    a0, da, la = a[:, 0, :], a[:, 1:-1, :], a[:, -1, :]
    v = act.f(a0)
    s1, s2 = act.d1(a0), act.d2(a0)
    dv = s1[:, None, :] * da
    if mask.dim() == 2:
        quad = torch.einsum("ij,nik,njk->nk", mask, da, da)
    else:
        quad = (mask[None, :, None] * da * da).sum(1)
    lv = s1 * la + s2 * quad
    return torch.cat([v[:, None, :], dv, lv[:, None, :]], 1)


@dataclass
class Forward:
    zin: List[torch.Tensor]    # Z~^(l-1): layer inputs with bias feature, (N, S, h_in+1)
    pre: List[torch.Tensor]    # pre-activations (linear layer outputs), (N, S, h_out)
    out: torch.Tensor          # network output rows (N, S) or values (M,)


def forward_laplacian(Ws: Sequence[torch.Tensor], X: torch.Tensor, mask: torch.Tensor,
                      act: Activation = TANH) -> Forward:
    """Forward Laplacian with intermediates (Algorithm 1, step 1): per linear layer
    T_out = W~ T~_in (Eq. forward-laplacian-linear-layer-compact), then the
    activation rule on every hidden layer.  Output rows: value, d_1 u .. d_d u, Lu."""
    Z = input_slab(X)
    zin, pre = [], []
    L = len(Ws)
    for l, W in enumerate(Ws):
        Zt = augment(Z)
        a = Zt @ W.T
        zin.append(Zt)
        pre.append(a)
        if l < L - 1:
            Z = activation_rows(a, mask, act)
    return Forward(zin, pre, pre[-1][:, :, 0])


def forward_plain(Ws: Sequence[torch.Tensor], X: torch.Tensor, act: Activation = TANH) -> Forward:
    """Plain forward pass with intermediates for the boundary term (Algorithm 1, step 2)."""
    z = X
    zin, pre = [], []
    for l, W in enumerate(Ws):
        zt = augment(z)
        a = zt @ W.T
        zin.append(zt)
        pre.append(a)
        z = act.f(a) if l < len(Ws) - 1 else a
    return Forward(zin, pre, pre[-1][:, 0])


# ----------------------------------------------------------------------------
# Residuals and loss (Section 2.1, Eq. pinn-loss)
# ----------------------------------------------------------------------------

def interior_residual(U: torch.Tensor, y: torch.Tensor, op: Operator,
                      X: Optional[torch.Tensor] = None) -> torch.Tensor:
    """r_n = L u(x_n) - y_n with L u = c_t d_t u + c_lap (masked) Lap u.  The output
    rows are value (0), derivatives (1..d), Laplacian (d+1).  A residual with
    first-order terms (Section 3.3; e.g. the logarithmic Fokker-Planck equation of
    Section 4) adds sum_{i in mask} (c_x x_i d_i u + c_g (d_i u)^2) + c_0, which
    needs the points X."""
    r = op.coef_lap * U[:, -1] - y
    if op.time_coord >= 0 and op.coef_time != 0.0:
        r = r + op.coef_time * U[:, 1 + op.time_coord]
    if op.coef_xgrad != 0.0 or op.coef_gradsq != 0.0 or op.coef_const != 0.0:
        d = U.shape[1] - 2
        m = op.mask_vec(d)
        du = U[:, 1:d + 1]
        r = r + ((op.coef_xgrad * X + op.coef_gradsq * du) * du * m).sum(1) + op.coef_const
    return r


def boundary_residual(u: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    return u - y


def loss_terms(r: torch.Tensor, rb: torch.Tensor):
    """L_Omega = sum r^2 / (2N), L_dOmega = sum rb^2 / (2M)  (Eq. pinn-loss)."""
    return (r * r).sum() / (2 * r.numel()), (rb * rb).sum() / (2 * rb.numel())


def _t(a) -> torch.Tensor:
    return a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a, dtype=np.float64))


def loss(theta, widths, Xi, yi, Xb, yb, op: Operator = POISSON_OP, act: Activation = TANH):
    """Total loss L(theta) = L_Omega + L_dOmega."""
    with torch.no_grad():
        Ws = unpack(_t(theta), widths)
        Xi, yi, Xb, yb = map(_t, (Xi, yi, Xb, yb))
        fi = forward_laplacian(Ws, Xi, op.second_order(Xi.shape[1]), act)
        fb = forward_plain(Ws, Xb, act)
        li, lb = loss_terms(interior_residual(fi.out, yi, op, Xi), boundary_residual(fb.out, yb))
    return float(li + lb), float(li), float(lb)


# ----------------------------------------------------------------------------
# Layer output gradients by autodiff (Algorithm 1, steps 1 and 2)
# ----------------------------------------------------------------------------

@dataclass
class Curvature:
    zin: List[torch.Tensor]
    g: List[torch.Tensor]
    r: torch.Tensor
    out: torch.Tensor


def interior_curvature_inputs(Ws, Xi, yi, op: Operator, act: Activation = TANH) -> Curvature:
    """Z~^(l-1)_{n,s} and g^(l)_{n,s} = d r_n / d a^(l)_{n,s} for the interior term.
    One backward pass of sum_n r_n gives all of them, since r_n only depends on
    point n's rows (Algorithm 1 differentiates the operator output per point)."""
    Ws = [W.detach() for W in Ws]
    Z = input_slab(Xi)
    zin, pre = [], []
    for l, W in enumerate(Ws):
        Zt = augment(Z)
        a = (Zt @ W.T).requires_grad_(True) if l == 0 else Zt @ W.T
        zin.append(Zt.detach())
        pre.append(a)
        if l < len(Ws) - 1:
            Z = activation_rows(a, op.second_order(Xi.shape[1]), act)
    r = interior_residual(pre[-1][:, :, 0], yi, op, Xi)
    g = torch.autograd.grad(r.sum(), pre, allow_unused=True)
    g = [gi if gi is not None else torch.zeros_like(p) for gi, p in zip(g, pre)]
    return Curvature(zin, [x.detach() for x in g], r.detach(), pre[-1][:, :, 0].detach())


def boundary_curvature_inputs(Ws, Xb, yb, act: Activation = TANH) -> Curvature:
    """z~^(l-1)_n and g^(l)_n = d u_n / d a^(l)_n for the boundary term."""
    Ws = [W.detach() for W in Ws]
    z = Xb
    zin, pre = [], []
    for l, W in enumerate(Ws):
        zt = augment(z)
        a = (zt @ W.T).requires_grad_(True) if l == 0 else zt @ W.T
        zin.append(zt.detach())
        pre.append(a)
        z = act.f(a) if l < len(Ws) - 1 else a
    u = pre[-1][:, 0]
    g = torch.autograd.grad(u.sum(), pre)
    return Curvature(zin, [x.detach() for x in g], boundary_residual(u, yb).detach(), u.detach())


# ----------------------------------------------------------------------------
# Kronecker factors (Eq. KFAC-PINN; Eq. kfac-linear for the boundary)
# ----------------------------------------------------------------------------

def interior_factors(cv: Curvature):
    """A_Omega = 1/(N S) sum_{n,s} Z~ Z~^T,  B_Omega = 1/N sum_{n,s} g g^T."""
    N, S = cv.zin[0].shape[:2]
    A, B = [], []
    for Zt, g in zip(cv.zin, cv.g):
        z2 = Zt.reshape(N * S, -1)
        g2 = g.reshape(N * S, -1)
        A.append(z2.T @ z2 / (N * S))
        B.append(g2.T @ g2 / N)
    return A, B


def boundary_factors(cv: Curvature):
    """A_dOmega = 1/M sum_n z~ z~^T,  B_dOmega = 1/M sum_n g g^T."""
    M = cv.zin[0].shape[0]
    return [z.T @ z / M for z in cv.zin], [g.T @ g / M for g in cv.g]


# ----------------------------------------------------------------------------
# Gradient of the loss by autodiff (Algorithm 1, step 4)
# ----------------------------------------------------------------------------

def loss_gradient(theta, widths, Xi, yi, Xb, yb, op: Operator = POISSON_OP,
                  act: Activation = TANH):
    th = _t(theta).detach().clone().requires_grad_(True)
    Ws = unpack(th, widths)
    Xi, yi, Xb, yb = map(_t, (Xi, yi, Xb, yb))
    fi = forward_laplacian(Ws, Xi, op.second_order(Xi.shape[1]), act)
    fb = forward_plain(Ws, Xb, act)
    li, lb = loss_terms(interior_residual(fi.out, yi, op, Xi), boundary_residual(fb.out, yb))
    (gr,) = torch.autograd.grad(li + lb, th)
    return gr.detach(), float(li.detach()), float(lb.detach())


# ----------------------------------------------------------------------------
# EMA and damping (Section 3.4)
# ----------------------------------------------------------------------------

def ema(prev: torch.Tensor, new: torch.Tensor, beta: float) -> torch.Tensor:
    return beta * prev + (1.0 - beta) * new


def damp(M: torch.Tensor, lam: float) -> torch.Tensor:
    return M + lam * torch.eye(M.shape[0], dtype=DT)


# ----------------------------------------------------------------------------
# Inverse of a Kronecker sum (Section 3.4; Martens & Grosse 2015, App. I)
# ----------------------------------------------------------------------------

def _inv_sqrt(M: torch.Tensor) -> torch.Tensor:
    w, E = torch.linalg.eigh(M)
    return (E / torch.sqrt(w)) @ E.T


@dataclass
class KronSumInverse:
    """(A1 (x) B1 + A2 (x) B2)^-1 = (PA (x) PB) (I + a (x) b)^-1 (PA (x) PB)^T with
    PA = A1^-1/2 EA, EA the eigenvectors of A1^-1/2 A2 A1^-1/2 (eigenvalues a);
    the same for B."""
    PA: torch.Tensor
    a: torch.Tensor
    PB: torch.Tensor
    b: torch.Tensor

    def apply(self, V: torch.Tensor) -> torch.Tensor:
        """Solve B1 X A1 + B2 X A2 = V, i.e. X = mat(K^-1 vec V) with column-major vec
        and (A (x) B) vec X = vec(B X A^T)."""
        Y = self.PB.T @ V @ self.PA
        Y = Y / (1.0 + self.b[:, None] * self.a[None, :])
        return self.PB @ Y @ self.PA.T


def kron_sum_inverse(A1, B1, A2, B2) -> KronSumInverse:
    iA, iB = _inv_sqrt(A1), _inv_sqrt(B1)
    a, EA = torch.linalg.eigh(iA @ A2 @ iA)
    b, EB = torch.linalg.eigh(iB @ B2 @ iB)
    return KronSumInverse(iA @ EA, a, iB @ EB, b)


def kron_sum_solve_dense(A1, B1, A2, B2, V) -> torch.Tensor:
    """Dense reference: build A1 (x) B1 + A2 (x) B2 and solve against vec V."""
    K = torch.kron(A1, B1) + torch.kron(A2, B2)
    x = torch.linalg.solve(K, V.T.reshape(-1))
    return x.reshape(V.shape[1], V.shape[0]).T


# ----------------------------------------------------------------------------
# One KFAC step (Algorithm 1; Section 3.4)
# ----------------------------------------------------------------------------

@dataclass
class HParams:
    lam: float = 1e-3
    beta: float = 0.0
    momentum: float = 0.0
    init_identity: bool = True
    lr_mode: str = "grid"          # "grid": alpha in {2^-30, ..., 2^0}; "fixed": alpha = lr
    lr: float = 1.0
    grid_min_exp: int = -30
    grid_max_exp: int = 0


@dataclass
class State:
    A_int: List[torch.Tensor]
    B_int: List[torch.Tensor]
    A_bnd: List[torch.Tensor]
    B_bnd: List[torch.Tensor]
    delta: torch.Tensor
    step: int = 0


def init_state(widths: Sequence[int], init_identity: bool) -> State:
    """Algorithm 1, step 0: every factor starts at 0 or at the identity."""
    L = len(widths) - 1
    mk = (lambda n: torch.eye(n, dtype=DT)) if init_identity else (lambda n: torch.zeros(n, n, dtype=DT))
    A = [mk(widths[l] + 1) for l in range(L)]
    B = [mk(widths[l + 1]) for l in range(L)]
    return State([a.clone() for a in A], [b.clone() for b in B], [a.clone() for a in A],
                 [b.clone() for b in B], torch.zeros(num_params(widths), dtype=DT), 0)


@dataclass
class StepInfo:
    loss_interior: float
    loss_boundary: float
    lr: float
    loss_after: float
    candidate_losses: Optional[List[float]]
    direction: torch.Tensor       # Delta_t (preconditioned negative gradient)
    update: torch.Tensor          # delta_t (applied)
    gradient: torch.Tensor
    status: int = 0


def line_search(theta, widths, data, op, act, dhat, hp: HParams):
    """alpha* = argmin over the logarithmic grid {2^-30, ..., 2^0} of L(theta + alpha dhat)
    (Section 3.4).  Candidates are scanned from the largest alpha down; the first
    strict minimum wins, so ties go to the larger step.  Non-finite losses count as
    +inf; if all are non-finite, no step is taken."""
    losses, best_k, best = [], None, math.inf
    for k in range(hp.grid_max_exp, hp.grid_min_exp - 1, -1):
        alpha = 2.0 ** k
        val = loss(theta + alpha * dhat, widths, *data, op, act)[0]
        losses.append(val)
        if math.isfinite(val) and val < best:
            best, best_k = val, k
    return best_k, losses


def kfac_step(theta, widths, data, op: Operator, hp: HParams, state: State,
              act: Activation = TANH):
    """One iteration of Algorithm 1 on a fixed batch `data` = (Xi, yi, Xb, yb).
    Returns (theta_next, state_next, info); `state` is not modified."""
    theta = _t(theta).clone()
    Xi, yi, Xb, yb = map(_t, data)
    Ws = unpack(theta, widths)
    # 1) interior curvature (forward Laplacian, output gradients, EMA of factors)
    ci = interior_curvature_inputs(Ws, Xi, yi, op, act)
    Ai, Bi = interior_factors(ci)
    A_int = [ema(p, n, hp.beta) for p, n in zip(state.A_int, Ai)]
    B_int = [ema(p, n, hp.beta) for p, n in zip(state.B_int, Bi)]
    # 2) boundary curvature
    cb = boundary_curvature_inputs(Ws, Xb, yb, act)
    Ab, Bb = boundary_factors(cb)
    A_bnd = [ema(p, n, hp.beta) for p, n in zip(state.A_bnd, Ab)]
    B_bnd = [ema(p, n, hp.beta) for p, n in zip(state.B_bnd, Bb)]
    # 3) preconditioner from the damped factors
    inv = [kron_sum_inverse(damp(A_int[l], hp.lam), damp(B_int[l], hp.lam),
                            damp(A_bnd[l], hp.lam), damp(B_bnd[l], hp.lam))
           for l in range(len(Ws))]
    # 4) gradient, preconditioned direction, momentum
    grad, li, lb = loss_gradient(theta, widths, Xi, yi, Xb, yb, op, act)
    gW = unpack(grad, widths)
    Delta = pack([-inv[l].apply(gW[l]) for l in range(len(Ws))])
    dhat = hp.momentum * state.delta + Delta if state.step > 0 else Delta
    # 5) learning rate and update
    status, cand = 0, None
    if hp.lr_mode == "grid":
        k, cand = line_search(theta, widths, (Xi, yi, Xb, yb), op, act, dhat, hp)
        if k is None:
            status, alpha = 5, 0.0
        else:
            alpha = 2.0 ** k
    else:
        alpha = hp.lr
    if status == 0:
        delta = alpha * dhat
        theta_next = theta + delta
    else:
        delta, theta_next = state.delta.clone(), theta.clone()
    after = loss(theta_next, widths, Xi, yi, Xb, yb, op, act)[0]
    new_state = State(A_int, B_int, A_bnd, B_bnd, delta if status == 0 else state.delta,
                      state.step + (1 if status == 0 else 0))
    return theta_next, new_state, StepInfo(li, lb, alpha, after, cand, Delta, delta, grad, status)


# ----------------------------------------------------------------------------
# Independent routes to the Laplacian, used only to pin the forward Laplacian
# ----------------------------------------------------------------------------

def laplacian_taylor_naive(Ws, X, act: Activation = TANH, coords=None):
    """Second-order Taylor mode along each basis direction separately (Section 3.1,
    Eqs. forward_pass and taylor-forward-activation with i = j), summed at the end."""
    N, d = X.shape
    coords = range(d) if coords is None else coords
    total = torch.zeros(N, dtype=DT)
    for i in coords:
        z = X
        dz = torch.zeros(N, d, dtype=DT); dz[:, i] = 1.0
        d2z = torch.zeros(N, d, dtype=DT)
        for l, W in enumerate(Ws):
            Wm, b = W[:, :-1], W[:, -1]
            z, dz, d2z = z @ Wm.T + b, dz @ Wm.T, d2z @ Wm.T
            if l < len(Ws) - 1:
                s1, s2 = act.d1(z), act.d2(z)
                z, dz, d2z = act.f(z), s1 * dz, s2 * dz * dz + s1 * d2z
        total = total + d2z[:, 0]
    return total


def laplacian_autodiff(Ws, X, act: Activation = TANH, coords=None):
    """Trace of the input Hessian by nested reverse-mode autodiff (the route the
    paper compares against in Appendix C.4)."""
    N, d = X.shape
    coords = range(d) if coords is None else coords
    x = X.clone().requires_grad_(True)

    def net(z):
        for l, W in enumerate(Ws):
            z = z @ W[:, :-1].T + W[:, -1]
            if l < len(Ws) - 1:
                z = act.f(z)
        return z[:, 0]

    u = net(x)
    (gx,) = torch.autograd.grad(u.sum(), x, create_graph=True)
    lap = torch.zeros(N, dtype=DT)
    for i in coords:
        (h,) = torch.autograd.grad(gx[:, i].sum(), x, retain_graph=True)
        lap = lap + h[:, i]
    return lap.detach()
