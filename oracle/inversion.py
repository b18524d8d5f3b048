"""Inversion driver of Section 3.5 ("The final algorithm"), written out plainly.

TEST INFRASTRUCTURE ONLY: the reference against which the library's driver
(``paper_2211_16665_amd.inversion``) is checked.  It shares no code with it.

    phi(m)  = phi_d(m) + beta phi_m(m),         m = ln rho on the active cells
    phi_m   = 1/2 sum_d alpha_d^2 || G_d (m - m_ref) ||^2
where G_d is the sparse forward-difference matrix between neighbouring cells
along axis d (reading: differences in cell index, alpha_d dimensionless).

The optimiser is l-BFGS in its textbook matrix form: the inverse-Hessian
estimate is built as a dense matrix from the stored pairs by the BFGS update
(Nocedal and Wright, eq. 6.17), starting from H0 = gamma D with
gamma = s'y / y'D y of the newest pair (D the diagonal preconditioner, I by
default), and the direction is -H g.  Readings of the parts the paper leaves
open (shared by the library's driver, each side written independently):
  * step length by backtracking on the Armijo condition
    phi(x_t) <= phi(x) + c1 g'(x_t - x), x_t = clip(x + t p), t <- t * shrink;
    the first trial is t = 1 for an l-BFGS direction and t = first_step for
    a steepest-descent direction, which is -D g scaled to unit max norm;
  * after the first line-search failure the pairs are dropped and the
    iteration restarts from steepest descent (the paper's remedy for its
    approximate gradient); a failure with no pairs, or a second failure,
    ends the run;
  * a pair is kept only if s'y > 1e-12 y'y; at most `memory` are kept;
  * an l-BFGS direction that is not a descent direction is replaced by
    steepest descent;
  * bounds m_min <= m <= m_max by projection;
  * beta is multiplied by `cooling` after every accepted step, which
    changes the objective, so the pairs are dropped.
Dense matrices limit this to small models (a few thousand active cells).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def difference_matrix(shape, axis: int) -> sp.csr_matrix:
    """G with (G u)_f = u[c+1] - u[c] for every pair of neighbouring cells
    (c, c+1) along ``axis`` of a C-ordered array of ``shape``."""
    n = int(np.prod(shape))
    idx = np.arange(n).reshape(shape)
    lo = np.take(idx, np.arange(shape[axis] - 1), axis=axis).ravel()
    hi = np.take(idx, np.arange(1, shape[axis]), axis=axis).ravel()
    nf = lo.size
    rows = np.concatenate([np.arange(nf), np.arange(nf)])
    cols = np.concatenate([hi, lo])
    vals = np.concatenate([np.ones(nf), -np.ones(nf)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, n))


def roughness(m: np.ndarray, m_ref: np.ndarray, alpha=(1.0, 1.0, 1.0)):
    """phi_m and its gradient sum_d alpha_d^2 G_d' G_d (m - m_ref).  m is
    [nz][ny][nx], or [P][nz][ny][nx] with P parameters (the two VTI
    resistivities) regularised independently."""
    u = np.asarray(m, dtype=np.float64) - np.asarray(m_ref, dtype=np.float64)
    spatial = u.shape[-3:]
    blocks = u.reshape(-1, *spatial)
    val = 0.0
    grad = np.zeros_like(blocks)
    # spatial axes: x is the last (2), y the middle (1), z the first (0)
    for a, axis in ((alpha[0], 2), (alpha[1], 1), (alpha[2], 0)):
        G = difference_matrix(spatial, axis)
        for b in range(blocks.shape[0]):
            r = G @ blocks[b].ravel()
            val += 0.5 * a * a * float(r @ r)
            grad[b] += (a * a * (G.T @ r)).reshape(spatial)
    return val, grad.reshape(u.shape)


def bfgs_inverse_hessian(S, Y, D=None) -> np.ndarray:
    """Dense H from the pairs by H <- V' H V + r s s', V = I - r y s',
    r = 1 / y's, from H0 = gamma diag(D) (Nocedal and Wright, eq. 6.17)."""
    n = S[0].size
    d = np.ones(n) if D is None else np.asarray(D, dtype=np.float64)
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ (d * Y[-1]))
    H = gamma * np.diag(d)
    I = np.eye(n)
    for s, y in zip(S, Y):
        r = 1.0 / float(y @ s)
        V = I - r * np.outer(y, s)
        H = V.T @ H @ V + r * np.outer(s, s)
    return H


def invert(data_term, m_ref, active, x0, alpha=(1.0, 1.0, 1.0), beta=0.0, max_iter=10,
           memory=5, m_min=-np.inf, m_max=np.inf, c1=1e-4, shrink=0.5, max_backtracks=8,
           first_step=0.1, cooling=1.0, precond=None):
    """Run the driver.  ``data_term(m_full)`` returns (phi_d, d phi_d / d m)
    over the full model; x0 and the returned model values are on the active
    cells.  Returns dict(m (full model), x, history: list of dict(phi, phi_d,
    phi_m, step, restart), restarts, evaluations)."""
    m_ref = np.asarray(m_ref, dtype=np.float64)
    active = np.asarray(active, bool)
    D = None if precond is None else np.asarray(precond, dtype=np.float64)
    count = {"n": 0}
    state = {"beta": beta}

    def full(x):
        m = m_ref.copy()
        m[active] = x
        return m

    def evaluate(x):
        m = full(x)
        phi_d, g_d = data_term(m)
        phi_m, g_m = roughness(m, m_ref, alpha)
        count["n"] += 1
        return phi_d, np.asarray(g_d, dtype=np.float64), phi_m, g_m

    def total(parts):
        phi_d, g_d, phi_m, g_m = parts
        b = state["beta"]
        return phi_d + b * phi_m, (g_d + b * g_m)[active]

    def steepest(g):
        v = g if D is None else D * g
        return -v / np.abs(v).max()

    x = np.clip(np.asarray(x0, dtype=np.float64), m_min, m_max)
    parts = evaluate(x)
    f, g = total(parts)
    history = [dict(phi=f, phi_d=parts[0], phi_m=parts[2], step=0.0, restart=False)]
    S, Y = [], []
    restarts = 0
    for _ in range(max_iter):
        if np.abs(g).max() == 0.0:
            break
        if S:
            p = -bfgs_inverse_hessian(S, Y, D) @ g
            t = 1.0
        else:
            p = steepest(g)
            t = first_step
        if g @ p >= 0.0:
            S, Y = [], []
            p = steepest(g)
            t = first_step
        accepted = False
        for _ in range(max_backtracks):
            xt = np.clip(x + t * p, m_min, m_max)
            parts_t = evaluate(xt)
            ft, gt = total(parts_t)
            if ft <= f + c1 * float(g @ (xt - x)):
                accepted = True
                break
            t *= shrink
        if not accepted:
            last = history[-1]
            if restarts > 0 or not S:
                history.append(dict(phi=f, phi_d=last["phi_d"], phi_m=last["phi_m"], step=0.0,
                                    restart=False))
                break
            restarts += 1
            S, Y = [], []
            history.append(dict(phi=f, phi_d=last["phi_d"], phi_m=last["phi_m"], step=0.0,
                                restart=True))
            continue
        s, y = xt - x, gt - g
        if s @ y > 1e-12 * (y @ y):
            S.append(s)
            Y.append(y)
            S, Y = S[-memory:], Y[-memory:]
        x, f, g, parts = xt, ft, gt, parts_t
        history.append(dict(phi=f, phi_d=parts[0], phi_m=parts[2], step=t, restart=False))
        if cooling != 1.0:
            state["beta"] *= cooling
            f, g = total(parts)
            S, Y = [], []
    return dict(m=full(x), x=x, history=history, restarts=restarts, evaluations=count["n"])
