"""Inversion driver over the GPU gradient (Section 3.5, "The final
algorithm").

    phi(m) = phi_d(m) + beta phi_m(m),   m = ln rho (per active cell)
    phi_m  = 1/2 || grad^alpha (m - m_ref) ||^2
with the anisotropic first-order difference operator grad^alpha =
(alpha_x d_x, alpha_y d_y, alpha_z d_z) between neighbouring cells (reading:
differences in cell index, alpha_d dimensionless, so beta weighs one unit of
ln rho jump between neighbours).  The descent direction is l-BFGS (two-loop
recursion over the last `memory` pairs), the step length comes from a
backtracking line search on the Armijo condition, and after the first
line-search failure l-BFGS restarts from the steepest-descent direction (the
paper's remedy for its approximate gradient); the iteration stops at
`max_iter`.  Bounds m_min <= m <= m_max are kept by projection; beta can be
cooled by a factor per iteration; an optional depth preconditioning
D = (1 + depth / depth0)^p (after Plessix, as the paper cites) enters as the
diagonal initial inverse Hessian of l-BFGS (the steepest-descent direction
is then -D g; the line search and the curvature pairs use the true
gradient).

The data term and its gradient come from a callable (``Objective``), here a
FictitiousForward plan on the GPU; the optimiser itself is host arithmetic
on vectors of the active cells.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# regularisation
# ---------------------------------------------------------------------------
def roughness(m: np.ndarray, m_ref: np.ndarray, alpha=(1.0, 1.0, 1.0)):
    """phi_m = 1/2 sum_d alpha_d^2 sum_faces (dm)^2 over the cell faces normal
    to axis d (dm = difference of m - m_ref between the two cells), and its
    gradient.  m, m_ref [nz][ny][nx] (or a leading axis of parameters, e.g.
    the two VTI resistivities, regularised independently)."""
    u = m - m_ref
    g = np.zeros_like(u)
    val = 0.0
    ax_x, ax_y, ax_z = (u.ndim - 1, u.ndim - 2, u.ndim - 3)
    for a, axis in ((alpha[0], ax_x), (alpha[1], ax_y), (alpha[2], ax_z)):
        if a == 0.0:
            continue
        d = np.diff(u, axis=axis)
        val += 0.5 * a * a * float(np.sum(d * d))
        w = a * a * d
        pad_lo = [(0, 0)] * u.ndim
        pad_hi = [(0, 0)] * u.ndim
        pad_lo[axis] = (1, 0)
        pad_hi[axis] = (0, 1)
        # d phi / d u_i = a^2 ((u_i - u_{i-1}) - (u_{i+1} - u_i))
        g += np.pad(w, pad_lo) - np.pad(w, pad_hi)
    return val, g


# ---------------------------------------------------------------------------
# l-BFGS pieces
# ---------------------------------------------------------------------------
def two_loop(g: np.ndarray, S: list, Y: list, D: np.ndarray | None = None) -> np.ndarray:
    """H g for the l-BFGS inverse-Hessian estimate from the pairs
    (s_i, y_i) (Nocedal and Wright, Algorithm 7.4), with the initial matrix
    gamma D (D = I if None), gamma = s'y / y'D y of the newest pair."""
    q = g.copy()
    rho = [1.0 / float(np.dot(y, s)) for s, y in zip(S, Y)]
    a = [0.0] * len(S)
    for i in range(len(S) - 1, -1, -1):
        a[i] = rho[i] * float(np.dot(S[i], q))
        q -= a[i] * Y[i]
    if S:
        Dy = Y[-1] if D is None else D * Y[-1]
        q *= float(np.dot(S[-1], Y[-1])) / float(np.dot(Y[-1], Dy))
        if D is not None:
            q *= D
    for i in range(len(S)):
        b = rho[i] * float(np.dot(Y[i], q))
        q += (a[i] - b) * S[i]
    return q


@dataclass
class InversionResult:
    m: np.ndarray
    history: list = field(default_factory=list)   # per iteration: dict(phi, phi_d, phi_m, step, evals, restart)
    restarts: int = 0
    evaluations: int = 0


class Objective:
    """phi(m) and its gradient on the active cells.  ``data_term(m_full)``
    returns (phi_d, d phi_d / d m_full) for the full model m_full (shape of
    the model); the regularisation is added here."""

    def __init__(self, data_term, m_ref, active=None, alpha=(1.0, 1.0, 0.1), beta=0.01):
        self.data_term = data_term
        self.m_ref = np.asarray(m_ref, dtype=np.float64)
        self.active = np.ones(self.m_ref.shape, bool) if active is None else np.asarray(active, bool)
        self.alpha = alpha
        self.beta = beta
        self.evaluations = 0

    def full(self, x: np.ndarray) -> np.ndarray:
        m = self.m_ref.copy()
        m[self.active] = x
        return m

    def __call__(self, x: np.ndarray):
        m = self.full(x)
        phi_d, g_d = self.data_term(m)
        phi_m, g_m = roughness(m, self.m_ref, self.alpha)
        self.evaluations += 1
        self._last = (phi_d, np.asarray(g_d, dtype=np.float64), phi_m, g_m)
        return self._combine()

    def _combine(self):
        phi_d, g_d, phi_m, g_m = self._last
        g = g_d + self.beta * g_m
        return phi_d + self.beta * phi_m, g[self.active], (phi_d, phi_m)

    def rescale(self, beta: float):
        """Change beta; phi and its gradient at the last evaluated point
        without a new data-term evaluation."""
        self.beta = beta
        return self._combine()


def depth_preconditioner(z_nodes: np.ndarray, shape, depth0: float, power: float = 1.0,
                         z_top: float = 0.0) -> np.ndarray:
    """Diagonal scaling (1 + max(z_c - z_top, 0) / depth0)^power per cell
    (z positive down, z_c the cell centre), broadcast to ``shape``
    ([nz][ny][nx] or [2][nz][ny][nx]): boosts the weakly sensitive deep
    cells."""
    z = np.asarray(z_nodes, dtype=np.float64)
    zc = 0.5 * (z[:-1] + z[1:])
    f = (1.0 + np.maximum(zc - z_top, 0.0) / depth0) ** power
    return np.broadcast_to(f.reshape(-1, 1, 1), shape).copy()


def lbfgs(obj: Objective, x0: np.ndarray, max_iter: int = 10, memory: int = 5,
          m_min: float = -np.inf, m_max: float = np.inf, c1: float = 1e-4,
          shrink: float = 0.5, max_backtracks: int = 8, first_step: float | None = None,
          cooling: float = 1.0, precond: np.ndarray | None = None) -> InversionResult:
    """Projected l-BFGS with backtracking line search and the paper's restart
    rule (steepest descent after the first line-search failure).

    first_step  length (in m) of the first steepest-descent trial step along
                -D g / max|D g|; later iterations try the l-BFGS step 1 first.
    cooling     beta <- cooling * beta after every iteration (0.7 .. 1).
    precond     diagonal D on the active cells (e.g. depth_preconditioner(...)
                [active]), the initial inverse Hessian."""
    D = None if precond is None else np.asarray(precond, dtype=np.float64)

    def steepest(g):
        d = g if D is None else D * g
        return -d / float(np.max(np.abs(d)))

    x = np.clip(np.asarray(x0, dtype=np.float64), m_min, m_max)
    f, g, parts = obj(x)
    res = InversionResult(m=obj.full(x))
    res.history.append(dict(phi=f, phi_d=parts[0], phi_m=parts[1], step=0.0, evals=1,
                            restart=False))
    S, Y = [], []
    restarted = False
    step0 = 0.1 if first_step is None else first_step
    for it in range(max_iter):
        if float(np.max(np.abs(g))) == 0.0:
            break
        if S:
            p = -two_loop(g, S, Y, D)
            t = 1.0
        else:
            p = steepest(g)
            t = step0
        if float(np.dot(g, p)) >= 0.0:         # not a descent direction: steepest descent
            S, Y = [], []
            p = steepest(g)
            t = step0
        evals = 0
        accepted = False
        for _ in range(max_backtracks):
            xn = np.clip(x + t * p, m_min, m_max)
            fn, gn_, parts = obj(xn)
            evals += 1
            if fn <= f + c1 * float(np.dot(g, xn - x)):
                accepted = True
                break
            t *= shrink
        restart = False
        if not accepted:
            if restarted or not S:
                res.history.append(dict(phi=f, phi_d=res.history[-1]["phi_d"],
                                        phi_m=res.history[-1]["phi_m"], step=0.0, evals=evals,
                                        restart=False))
                break                          # steepest descent failed too: stop
            # first failure: restart from steepest descent (Section 3.5)
            restarted = True
            restart = True
            res.restarts += 1
            S, Y = [], []
            res.history.append(dict(phi=f, phi_d=res.history[-1]["phi_d"],
                                    phi_m=res.history[-1]["phi_m"], step=0.0, evals=evals,
                                    restart=True))
            continue
        s = xn - x
        y = gn_ - g
        if float(np.dot(s, y)) > 1e-12 * float(np.dot(y, y)):
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        x, f, g = xn, fn, gn_
        res.history.append(dict(phi=f, phi_d=parts[0], phi_m=parts[1], step=t, evals=evals,
                                restart=restart))
        if cooling != 1.0:
            # the objective changes with beta: restart the curvature pairs
            f, g, parts = obj.rescale(obj.beta * cooling)
            S, Y = [], []
    res.m = obj.full(x)
    res.evaluations = obj.evaluations
    return res


def gpu_data_term(plan, d_obs, W=1.0, method="basis", snapshot_every=0, gamma_rel=1e-12):
    """phi_d(m) and its gradient from the library (FictitiousForward):
    m [nz][ny][nx] or, for VTI, [2][nz][ny][nx] (ln rho_h, ln rho_v)."""
    import torch

    from .autograd import FictitiousForward, misfit
    dd = torch.as_tensor(d_obs).cuda()
    Wt = W if np.isscalar(W) else torch.as_tensor(W).cuda()

    def term(m):
        mt = torch.tensor(m, dtype=torch.float64, device="cuda", requires_grad=True)
        E = FictitiousForward.apply(mt, plan, snapshot_every, gamma_rel, method)
        L = misfit(E, dd, Wt)
        L.backward()
        return float(L.detach()), mt.grad.cpu().numpy()

    return term
