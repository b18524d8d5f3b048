"""Staggered differences of order 2 and 4 on the stretched grid, and their
transposes (TEST INFRASTRUCTURE, part of the oracle package).

The paper's engine is high order on a non-uniform grid (Section 2, citing
Yang and Mittet 2023, whose coefficients the paper does not print).
Reading used for order 4: the standard fourth-order staggered pair
(9/8, -1/24) applied in the index coordinate of the stretched grid, divided
by a metric length obtained by applying the same pair to the node (or cell
centre) coordinates, so that a linear function is differentiated exactly
and the uniform-grid scheme is recovered when the spacing is constant.
Across the two walls of each axis the fields are continued by images:
tangential E vanishes on the wall and is odd, the H components (at half
nodes) are even; coordinates are odd about the wall.  With these images the
H -> E difference is minus the transpose of the E -> H difference, so the
discrete curl pair stays adjoint under the metric-weighted pairing and
reciprocity and the same-engine adjoint remain exact.  Order 2 is the Yee
difference with the cell widths and dual widths.
"""
from __future__ import annotations

import numpy as np

C1 = 9.0 / 8.0
C2 = -1.0 / 24.0


def _last(f, axis):
    return np.moveaxis(f, axis, -1)


def diff_e(F: np.ndarray, axis: int, order: int) -> np.ndarray:
    """E -> H difference along ``axis``: F on the nodes 0..n (zero on the
    walls), result on the half nodes 0..n-1 (not divided by the metric)."""
    G = _last(F, axis)
    d = G[..., 1:] - G[..., :-1]
    if order == 4:
        ext = np.concatenate([-G[..., 1:2], G, -G[..., -2:-1]], axis=-1)   # nodes -1..n+1
        d = C1 * d + C2 * (ext[..., 3:] - ext[..., :-3])
    return np.moveaxis(d, -1, axis)


def diff_h(H: np.ndarray, axis: int, order: int) -> np.ndarray:
    """H -> E difference along ``axis``: H on the half nodes 0..n-1, result
    on the interior nodes 1..n-1 (not divided by the metric)."""
    G = _last(H, axis)
    d = G[..., 1:] - G[..., :-1]
    if order == 4:
        ext = np.concatenate([G[..., 1:2], G[..., 0:1], G, G[..., -1:], G[..., -2:-1]],
                             axis=-1)                                        # half nodes -2..n+1
        d = C1 * d + C2 * (ext[..., 4:-1] - ext[..., 1:-4])
    return np.moveaxis(d, -1, axis)


def diff_e_t(g: np.ndarray, axis: int, order: int) -> np.ndarray:
    """Transpose of diff_e: g on the half nodes 0..n-1 -> node values 0..n."""
    G = _last(g, axis)
    n = G.shape[-1]
    ext = np.zeros(G.shape[:-1] + (n + 3,))       # nodes -1..n+1 at ext index node + 1
    ext[..., 2:n + 2] += C1 * G if order == 4 else G
    ext[..., 1:n + 1] -= C1 * G if order == 4 else G
    if order == 4:
        ext[..., 3:n + 3] += C2 * G
        ext[..., 0:n] -= C2 * G
    out = ext[..., 1:n + 2].copy()
    out[..., 1] -= ext[..., 0]                    # node -1 is -node 1
    out[..., n - 1] -= ext[..., n + 2]            # node n+1 is -node n-1
    return np.moveaxis(out, -1, axis)


def diff_h_t(g: np.ndarray, axis: int, order: int) -> np.ndarray:
    """Transpose of diff_h: g on the interior nodes 1..n-1 -> half-node
    values 0..n-1."""
    G = _last(g, axis)
    n = G.shape[-1] + 1
    ext = np.zeros(G.shape[:-1] + (n + 4,))       # half nodes -2..n+1 at ext index + 2
    c1 = C1 if order == 4 else 1.0
    ext[..., 3:n + 2] += c1 * G                   # output i uses H[i] (i = 1..n-1)
    ext[..., 2:n + 1] -= c1 * G                   # and H[i-1]
    if order == 4:
        ext[..., 4:n + 3] += C2 * G               # H[i+1]
        ext[..., 1:n] -= C2 * G                   # H[i-2]
    out = ext[..., 2:n + 2].copy()
    out[..., 0] += ext[..., 1]                    # half node -1 is half node 0
    out[..., 1] += ext[..., 0]                    # half node -2 is half node 1
    out[..., n - 1] += ext[..., n + 2]            # half node n is half node n-1
    out[..., n - 2] += ext[..., n + 3]            # half node n+1 is half node n-2
    return np.moveaxis(out, -1, axis)


def metric_half(nodes: np.ndarray, order: int) -> np.ndarray:
    """Metric length at the half nodes (n values): the cell widths for order
    2; the fourth-order difference of the node coordinates for order 4."""
    x = np.asarray(nodes, dtype=np.float64)
    h = np.diff(x)
    if order != 4:
        return h
    ext = np.concatenate([[2 * x[0] - x[1]], x, [2 * x[-1] - x[-2]]])
    return C1 * h + C2 * (ext[3:] - ext[:-3])


def metric_node(nodes: np.ndarray, order: int) -> np.ndarray:
    """Metric length at the nodes (n+1 values): dual widths for order 2
    (half a cell at the two walls); for order 4 the fourth-order difference
    of the cell-centre coordinates at the interior nodes (walls as order 2:
    no field there is updated)."""
    x = np.asarray(nodes, dtype=np.float64)
    h = np.diff(x)
    out = np.empty(len(x))
    out[1:-1] = 0.5 * (h[:-1] + h[1:])
    out[0], out[-1] = 0.5 * h[0], 0.5 * h[-1]
    if order != 4:
        return out
    c = 0.5 * (x[:-1] + x[1:])
    ext = np.concatenate([[2 * x[0] - c[1], 2 * x[0] - c[0]], c,
                          [2 * x[-1] - c[-1], 2 * x[-1] - c[-2]]])
    out[1:-1] = C1 * (c[1:] - c[:-1]) + C2 * (ext[4:-1] - ext[1:-4])
    return out
