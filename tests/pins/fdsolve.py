"""Sparse direct solve of the frequency-domain system that the leapfrog plus
on-the-fly DFT reaches exactly; a pin for the time-stepping oracle that
shares no code with it (grid operators, CPML stretching, averaging and
interpolation are written again here).

Identity used (derived from the leapfrog by summing each update against
z^n, z = exp(i w' dt), with zero initial state): the transforms
E^ = sum_n E^n z^n, H^ = sum_n H^{n+1/2} z^{n+1/2}, J^ = sum J^{n+1/2}
z^{n+1/2} satisfy
    curl_h H^ + i Omega eps E^ = J^,     curl_h E^ - i Omega mu H^ = 0,
    Omega = (2/dt) sin(w' dt / 2),
which is eq. mittet with w' replaced by Omega.  A CPML memory variable
psi <- b psi + a D transforms to psi^ = a D^ / (1 - b z), so every
stretched derivative becomes D^ (1/kappa + a/(1 - b z)) at its node.
Eliminating H^:  (curl_h curl_h / (i Omega mu) + i Omega eps) E^ = J^.

Order 4 (``order=4``): each one-dimensional difference is the pair
(9/8, -1/24) over the four nearest samples, divided by a metric length (the
same pair applied to the coordinates); samples beyond a wall are images
(tangential E odd, H even, coordinates odd).  Rows are assembled here from
those rules, entry by entry.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

MU0 = 4.0e-7 * np.pi


def _profile(nodes, pos, npml, dt, vref, order, R, kmax, amax, z):
    """1/s at positions ``pos`` for the CPML of one axis."""
    n = len(nodes) - 1
    xl, xr = nodes[npml], nodes[n - npml]
    out = np.ones(len(pos), dtype=np.complex128)
    for m, p in enumerate(pos):
        if p < xl:
            L, r = xl - nodes[0], (xl - p) / (xl - nodes[0])
        elif p > xr:
            L, r = nodes[n] - xr, (p - xr) / (nodes[n] - xr)
        else:
            continue
        d = -(order + 1.0) * vref * np.log(R) / (2.0 * L) * r ** order
        kap = 1.0 + (kmax - 1.0) * r ** order
        alp = amax * (1.0 - r)
        b = np.exp(-(d / kap + alp) * dt)
        a = d * (b - 1.0) / (kap * (d + kap * alp)) if d > 0 else 0.0
        out[m] = 1.0 / kap + a / (1.0 - b * z)
    return out


class Grid:
    """Index bookkeeping for the six staggered components."""

    def __init__(self, x, y, z):
        self.x, self.y, self.z = x, y, z
        self.nx, self.ny, self.nz = len(x) - 1, len(y) - 1, len(z) - 1
        nx, ny, nz = self.nx, self.ny, self.nz
        self.eshape = [(nz + 1, ny + 1, nx), (nz + 1, ny, nx + 1), (nz, ny + 1, nx + 1)]
        self.hshape = [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
        self.eoff = np.cumsum([0] + [int(np.prod(s)) for s in self.eshape])
        self.hoff = np.cumsum([0] + [int(np.prod(s)) for s in self.hshape])

    def e(self, c, k, j, i):
        s = self.eshape[c]
        return self.eoff[c] + (k * s[1] + j) * s[2] + i

    def h(self, c, k, j, i):
        s = self.hshape[c]
        return self.hoff[c] + (k * s[1] + j) * s[2] + i


def _dual(nodes):
    h = np.diff(nodes)
    d = np.empty(len(nodes))
    d[0], d[-1] = h[0] / 2, h[-1] / 2
    d[1:-1] = (h[1:] + h[:-1]) / 2
    return d


A1, A2 = 9.0 / 8.0, -1.0 / 24.0


def _e_to_h(r, n, order):
    """Entries (node, weight) of the difference at half node r (between
    nodes r and r+1) of a field on nodes 0..n that vanishes at 0 and n."""
    if order == 2:
        terms = [(r + 1, 1.0), (r, -1.0)]
    else:
        terms = [(r + 1, A1), (r, -A1), (r + 2, A2), (r - 1, -A2)]
    out = []
    for m, w in terms:
        if m < 0:
            m, w = -m, -w                    # odd image across node 0
        elif m > n:
            m, w = 2 * n - m, -w             # odd image across node n
        out.append((m, w))
    return out


def _h_to_e(i, n, order):
    """Entries (half node, weight) of the difference at node i (1..n-1) of a
    field on the half nodes 0..n-1."""
    if order == 2:
        terms = [(i, 1.0), (i - 1, -1.0)]
    else:
        terms = [(i, A1), (i - 1, -A1), (i + 1, A2), (i - 2, -A2)]
    out = []
    for m, w in terms:
        if m < 0:
            m = -1 - m                       # even image across node 0
        elif m > n - 1:
            m = 2 * n - 1 - m                # even image across node n
        out.append((m, w))
    return out


def _metrics(nodes, order):
    """(metric at the half nodes, metric at the nodes)."""
    n = len(nodes) - 1
    if order == 2:
        return np.diff(nodes), _dual(nodes)
    x0, xn = nodes[0], nodes[-1]

    def X(m):                                # node coordinate with odd images
        if m < 0:
            return 2 * x0 - nodes[-m]
        if m > n:
            return 2 * xn - nodes[2 * n - m]
        return nodes[m]
    c = 0.5 * (nodes[:-1] + nodes[1:])

    def Cc(m):                               # cell centre with odd images
        if m < 0:
            return 2 * x0 - c[-1 - m]
        if m > n - 1:
            return 2 * xn - c[2 * n - 1 - m]
        return c[m]
    mh = np.array([A1 * (X(r + 1) - X(r)) + A2 * (X(r + 2) - X(r - 1)) for r in range(n)])
    mn = _dual(nodes)
    for i in range(1, n):
        mn[i] = A1 * (Cc(i) - Cc(i - 1)) + A2 * (Cc(i + 1) - Cc(i - 2))
    return mh, mn


def solve(x, y, z, rho, npml, f0, freq, dt, sources, receivers, rec_comp,
          vref, cpml_order=2.0, cpml_R=1e-6, kappa_max=1.0, alpha_max=0.0,
          rho_cap=1e8, rho_v=None, order=2, src_kind=0, full=False):
    """Frequency-domain field at ``receivers`` for each dipole in ``sources``
    (list of (pos, moment)); returns complex [ns][nr][ncomp].  The field is
    that of J (not J'): the right-hand side is sqrt(-i w/2w0) p w_l / V_l.
    Components 0-2 are E, 3-5 are H, taken from the Faraday row
    H' = (curl E' - M') / (i Omega mu) and H = H' / sqrt(-i w/2w0).
    src_kind 1: magnetic dipoles, M' = M = m w_l / V_l on the H nodes (V_l
    the node length along the component times the cell lengths across it);
    eliminating H' puts curl_h M' / (i Omega mu) on the right-hand side.
    full=True also returns, per source, E on every edge as the three arrays
    of the E lattices (zero on the walls)."""
    g = Grid(x, y, z)
    nx, ny, nz = g.nx, g.ny, g.nz
    hx, hy, hz = np.diff(x), np.diff(y), np.diff(z)
    # metric lengths of the differences (= cell and dual widths for order 2)
    (mx, dx), (my, dy), (mz, dz) = _metrics(x, order), _metrics(y, order), _metrics(z, order)
    w0 = 2 * np.pi * f0
    om = 2 * np.pi * freq
    wp = (1 + 1j) * np.sqrt(om * w0)
    zz = np.exp(1j * wp * dt)
    Om = 2.0 / dt * np.sin(wp * dt / 2)
    prof = {}
    for nm, nodes in (("x", x), ("y", y), ("z", z)):
        mid = 0.5 * (nodes[:-1] + nodes[1:])
        args = (npml, dt, vref, cpml_order, cpml_R, kappa_max, alpha_max, zz)
        prof[nm] = (_profile(nodes, nodes, *args), _profile(nodes, mid, *args))
    isx_n, isx_h = prof["x"]
    isy_n, isy_h = prof["y"]
    isz_n, isz_h = prof["z"]

    # curl E -> faces
    rows, cols, vals = [], [], []

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    for k in range(nz):
        for j in range(ny):
            for i in range(nx + 1):          # H_x = dEz/dy - dEy/dz
                r = g.h(0, k, j, i)
                fy = isy_h[j] / my[j]
                fz = isz_h[k] / mz[k]
                for m, w in _e_to_h(j, ny, order):
                    add(r, g.e(2, k, m, i), fy * w)
                for m, w in _e_to_h(k, nz, order):
                    add(r, g.e(1, m, j, i), -fz * w)
    for k in range(nz):
        for j in range(ny + 1):
            for i in range(nx):              # H_y = dEx/dz - dEz/dx
                r = g.h(1, k, j, i)
                fz = isz_h[k] / mz[k]
                fx = isx_h[i] / mx[i]
                for m, w in _e_to_h(k, nz, order):
                    add(r, g.e(0, m, j, i), fz * w)
                for m, w in _e_to_h(i, nx, order):
                    add(r, g.e(2, k, j, m), -fx * w)
    for k in range(nz + 1):
        for j in range(ny):
            for i in range(nx):              # H_z = dEy/dx - dEx/dy
                r = g.h(2, k, j, i)
                fx = isx_h[i] / mx[i]
                fy = isy_h[j] / my[j]
                for m, w in _e_to_h(i, nx, order):
                    add(r, g.e(1, k, j, m), fx * w)
                for m, w in _e_to_h(j, ny, order):
                    add(r, g.e(0, k, m, i), -fy * w)
    CE = sp.csr_matrix((vals, (rows, cols)), shape=(g.hoff[-1], g.eoff[-1]))

    # curl H -> interior edges
    rows, cols, vals = [], [], []
    interior = []
    for k in range(1, nz):
        for j in range(1, ny):
            for i in range(nx):              # E_x: dHz/dy - dHy/dz
                r = g.e(0, k, j, i)
                interior.append(r)
                fy = isy_n[j] / dy[j]
                fz = isz_n[k] / dz[k]
                for m, w in _h_to_e(j, ny, order):
                    add(r, g.h(2, k, m, i), fy * w)
                for m, w in _h_to_e(k, nz, order):
                    add(r, g.h(1, m, j, i), -fz * w)
    for k in range(1, nz):
        for j in range(ny):
            for i in range(1, nx):           # E_y: dHx/dz - dHz/dx
                r = g.e(1, k, j, i)
                interior.append(r)
                fz = isz_n[k] / dz[k]
                fx = isx_n[i] / dx[i]
                for m, w in _h_to_e(k, nz, order):
                    add(r, g.h(0, m, j, i), fz * w)
                for m, w in _h_to_e(i, nx, order):
                    add(r, g.h(2, k, j, m), -fx * w)
    for k in range(nz):
        for j in range(1, ny):
            for i in range(1, nx):           # E_z: dHy/dx - dHx/dy
                r = g.e(2, k, j, i)
                interior.append(r)
                fx = isx_n[i] / dx[i]
                fy = isy_n[j] / dy[j]
                for m, w in _h_to_e(i, nx, order):
                    add(r, g.h(1, k, j, m), fx * w)
                for m, w in _h_to_e(j, ny, order):
                    add(r, g.h(0, k, m, i), -fy * w)
    CH = sp.csr_matrix((vals, (rows, cols)), shape=(g.eoff[-1], g.hoff[-1]))

    # edge permittivity: volume-weighted cell average, eps = sigma / (2 w0)
    sig = 1.0 / np.minimum(rho, rho_cap)
    # VTI: x and y edges average the horizontal, z edges the vertical value
    sigv = sig if rho_v is None else 1.0 / np.minimum(rho_v, rho_cap)
    eps = np.zeros(g.eoff[-1])
    vol = np.zeros(g.eoff[-1])
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                s = sig[k, j, i]
                for (kk, jj) in ((k, j), (k + 1, j), (k, j + 1), (k + 1, j + 1)):
                    w = hz[k] * hy[j]
                    eps[g.e(0, kk, jj, i)] += s * w
                    vol[g.e(0, kk, jj, i)] += w
                for (kk, ii) in ((k, i), (k + 1, i), (k, i + 1), (k + 1, i + 1)):
                    w = hz[k] * hx[i]
                    eps[g.e(1, kk, j, ii)] += s * w
                    vol[g.e(1, kk, j, ii)] += w
                for (jj, ii) in ((j, i), (j + 1, i), (j, i + 1), (j + 1, i + 1)):
                    w = hy[j] * hx[i]
                    eps[g.e(2, k, jj, ii)] += sigv[k, j, i] * w
                    vol[g.e(2, k, jj, ii)] += w
    eps = eps / vol / (2.0 * w0)

    A = CH @ CE / (1j * Om * MU0) + sp.diags(1j * Om * eps)
    idx = np.array(interior)
    Ai = A[idx][:, idx].tocsc()
    lu = spla.splu(Ai)
    pos_of = {int(r): m for m, r in enumerate(idx)}

    # lattices of the three E components and dual volumes
    xh, yh, zh = 0.5 * (x[1:] + x[:-1]), 0.5 * (y[1:] + y[:-1]), 0.5 * (z[1:] + z[:-1])
    lat = [(xh, y, z), (x, yh, z), (x, y, zh), (x, yh, zh), (xh, y, zh), (xh, yh, z)]
    edge_len = [(hx, None), (hy, None), (hz, None)]

    def dualvol(c, k, j, i):
        if c == 0:
            return mx[i] * dy[j] * dz[k]
        if c == 1:
            return dx[i] * my[j] * dz[k]
        if c == 2:
            return dx[i] * dy[j] * mz[k]
        if c == 3:                               # H_x: x node, y and z cells
            return dx[i] * my[j] * mz[k]
        if c == 4:
            return mx[i] * dy[j] * mz[k]
        return mx[i] * my[j] * dz[k]

    def weights(c, p):
        out = []
        sel = []
        for q, l in zip(p, lat[c]):
            m = int(np.clip(np.searchsorted(l, q) - 1, 0, len(l) - 2))
            t = (q - l[m]) / (l[m + 1] - l[m])
            sel.append([(m, 1 - t), (m + 1, t)])
        for i, wi in sel[0]:
            for j, wj in sel[1]:
                for k, wk in sel[2]:
                    if wi * wj * wk != 0:
                        out.append((k, j, i, wi * wj * wk))
        return out

    src_fac = np.sqrt(-1j * om / (2 * w0))
    out = np.zeros((len(sources), len(receivers), len(rec_comp)), dtype=np.complex128)
    fields = []
    for si, (pos, mom) in enumerate(sources):
        rhs = np.zeros(len(idx), dtype=np.complex128)
        m_full = np.zeros(g.hoff[-1], dtype=np.complex128)
        for c in range(3):
            if mom[c] == 0:
                continue
            if src_kind == 0:
                for (k, j, i, w) in weights(c, pos):
                    rhs[pos_of[int(g.e(c, k, j, i))]] += src_fac * mom[c] * w / dualvol(c, k, j, i)
            else:
                for (k, j, i, w) in weights(c + 3, pos):
                    m_full[int(g.h(c, k, j, i))] += mom[c] * w / dualvol(c + 3, k, j, i)
        if src_kind != 0:
            rhs += (CH @ m_full)[idx] / (1j * Om * MU0)
        sol = lu.solve(rhs)
        e_full = np.zeros(g.eoff[-1], dtype=np.complex128)
        e_full[idx] = sol
        fields.append([e_full[g.eoff[c]:g.eoff[c + 1]].reshape(g.eshape[c]) for c in range(3)])
        h_full = (CE @ e_full - m_full) / (1j * Om * MU0) / src_fac
        for ri, rp in enumerate(receivers):
            for ci, c in enumerate(rec_comp):
                val = 0j
                for (k, j, i, w) in weights(c, rp):
                    if c >= 3:
                        val += w * h_full[int(g.h(c - 3, k, j, i))]
                        continue
                    m = pos_of.get(int(g.e(c, k, j, i)))
                    if m is not None:
                        val += w * sol[m]
                out[si, ri, ci] = val
    return (out, fields) if full else out
