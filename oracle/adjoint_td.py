"""Time-domain adjoint of the fictitious-wave stepping and its gradient
(the alternative adjoint formulation of the Appendix).

TEST INFRASTRUCTURE (part of the oracle package; see oracle/__init__.py).

The Appendix attaches time-domain multipliers (E_adj, H_adj) to the
fictitious-wave equations (eq. fictitiouswave) in a Lagrangian; its
stationarity gives a Maxwell system that runs backward in time from zero
final conditions, driven at the receivers by a time series built directly
from the weighted residual (eqs. lambda1 and appadj1: no basis functions),
and the gradient (eq. chainrule)
    d phi / d sigma = -(1 / 2 omega0) sum_s int E_adj . dE/dt dt.
The same construction is applied here to the discrete stepped system (the
leapfrog with K&M CPML of oracle.stepping): the multipliers of the update
equations obey the transpose of one leapfrog step, including the transposed
CPML memory recursions, taken from the last step to the first and driven by
d phi / d E^m at the receiver nodes.  Writing the E update as
E^{n+1} = E^n + ce (curl H^{n+1/2} - J'^{n+1/2}) with ce = dt / eps =
2 omega0 dt / sigma_e, the derivative with respect to the edge conductivity is
    d phi / d sigma_e = - sum_n Eadj^{n+1}_e (E^{n+1}_e - E^n_e) / sigma_e
(reading: the discrete counterpart of eq. chainrule; Eadj^{n+1} is the
multiplier of the update that produces E^{n+1}, and E^{n+1} - E^n stands for
dt dE/dt).  It is the exact derivative of the stepped misfit.

The forward step is restated here in per-step form (fwd_step) so that its
transpose (adj_step) can be written next to it; a test checks that it
reproduces oracle.stepping.run_stepping, another that the pair passes the
dot-product test <L x, y> = <x, L^T y>.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

from .discretization import MU0, Setup, cell_gradient, edge_sigma_transpose, make_setup
from .stencil import diff_e, diff_e_t, diff_h, diff_h_t
from .stepping import receiver_nodes, source_injection, source_norms

FIELDS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
# CPML memory variables: key -> (field it belongs to, axis of the derivative)
PSI = {
    "Hx_y": ("Hx", "y"), "Hx_z": ("Hx", "z"), "Hy_z": ("Hy", "z"), "Hy_x": ("Hy", "x"),
    "Hz_x": ("Hz", "x"), "Hz_y": ("Hz", "y"),
    "Ex_y": ("Ex", "y"), "Ex_z": ("Ex", "z"), "Ey_z": ("Ey", "z"), "Ey_x": ("Ey", "x"),
    "Ez_x": ("Ez", "x"), "Ez_y": ("Ez", "y"),
}
AXIS = {"z": 0, "y": 1, "x": 2}


def _b(arr, axis):
    sh = [1, 1, 1]
    sh[axis] = -1
    return np.asarray(arr).reshape(sh)


def ops(s: Setup) -> SimpleNamespace:
    """Geometry and coefficients of one step, in the shapes the step uses."""
    o = SimpleNamespace()
    nx, ny, nz = s.nx, s.ny, s.nz
    o.shapes = {
        "Ex": (nz + 1, ny + 1, nx), "Ey": (nz + 1, ny, nx + 1), "Ez": (nz, ny + 1, nx + 1),
        "Hx": (nz, ny, nx + 1), "Hy": (nz, ny + 1, nx), "Hz": (nz + 1, ny, nx),
        "Hx_y": (nz, ny, nx + 1), "Hx_z": (nz, ny, nx + 1), "Hy_z": (nz, ny + 1, nx),
        "Hy_x": (nz, ny + 1, nx), "Hz_x": (nz + 1, ny, nx), "Hz_y": (nz + 1, ny, nx),
        "Ex_y": (nz - 1, ny - 1, nx), "Ex_z": (nz - 1, ny - 1, nx),
        "Ey_z": (nz - 1, ny, nx - 1), "Ey_x": (nz - 1, ny, nx - 1),
        "Ez_x": (nz, ny - 1, nx - 1), "Ez_y": (nz, ny - 1, nx - 1),
    }
    # metric lengths of the differences (cell and dual widths for order 2)
    o.h = {"x": _b(s.mx, 2), "y": _b(s.my, 1), "z": _b(s.mz, 0)}
    o.hd = {"x": _b(s.mdx[1:-1], 2), "y": _b(s.mdy[1:-1], 1), "z": _b(s.mdz[1:-1], 0)}
    o.order = s.order
    # CPML (1/kappa is applied as a division by kappa, as in the stepping)
    o.cp_half = {}
    o.cp_int = {}
    for ax in ("x", "y", "z"):
        (kn, bn, an), (kh, bh, ah) = s.cpml[ax]
        a_ = AXIS[ax]
        o.cp_half[ax] = (_b(kh, a_), _b(bh, a_), _b(ah, a_))
        o.cp_int[ax] = (_b(kn[1:-1], a_), _b(bn[1:-1], a_), _b(an[1:-1], a_))
    cx, cy, cz = s.ce
    o.ci = {"Ex": cx[1:-1, 1:-1, :], "Ey": cy[1:-1, :, 1:-1], "Ez": cz[:, 1:-1, 1:-1]}
    o.dtmu = s.dt / MU0
    return o


def zero_state(o) -> dict:
    return {k: np.zeros(sh) for k, sh in o.shapes.items()}


def _interior(name):
    """Slices of the updated (interior) part of an E component."""
    return {"Ex": np.s_[1:-1, 1:-1, :], "Ey": np.s_[1:-1, :, 1:-1],
            "Ez": np.s_[:, 1:-1, 1:-1]}[name]


# derivative terms of each update: (key, source field, axis, slice of the
# source field before differencing, sign in the update)
H_TERMS = {
    "Hx": (("Hx_y", "Ez", "y", np.s_[:, :, :], +1), ("Hx_z", "Ey", "z", np.s_[:, :, :], -1)),
    "Hy": (("Hy_z", "Ex", "z", np.s_[:, :, :], +1), ("Hy_x", "Ez", "x", np.s_[:, :, :], -1)),
    "Hz": (("Hz_x", "Ey", "x", np.s_[:, :, :], +1), ("Hz_y", "Ex", "y", np.s_[:, :, :], -1)),
}
E_TERMS = {
    "Ex": (("Ex_y", "Hz", "y", np.s_[1:-1, :, :], +1), ("Ex_z", "Hy", "z", np.s_[:, 1:-1, :], -1)),
    "Ey": (("Ey_z", "Hx", "z", np.s_[:, :, 1:-1], +1), ("Ey_x", "Hz", "x", np.s_[1:-1, :, :], -1)),
    "Ez": (("Ez_x", "Hy", "x", np.s_[:, 1:-1, :], +1), ("Ez_y", "Hx", "y", np.s_[:, :, 1:-1], -1)),
}


def fwd_step(o, st: dict) -> None:
    """One leapfrog step without sources, in place (Section 2, eq.
    fictitiouswave; the stepping of oracle.stepping.run_stepping):
        H^{n+1/2} = H^{n-1/2} - dt/mu (d1 - d2)
        E^{n+1}   = E^n + ce (d1 - d2)       on interior edges
    each derivative d = D/kappa + psi with psi <- b psi + a D (K&M CPML)."""
    for hname, terms in H_TERMS.items():
        dd = []
        for key, src, ax, sl, sign in terms:
            kap, b, a = o.cp_half[ax]
            D = diff_e(st[src][sl], AXIS[ax], o.order) / o.h[ax]
            st[key] = b * st[key] + a * D
            dd.append(sign * (D / kap + st[key]))
        st[hname] -= o.dtmu * (dd[0] + dd[1])
    for ename, terms in E_TERMS.items():
        dd = []
        for key, src, ax, sl, sign in terms:
            kap, b, a = o.cp_int[ax]
            D = diff_h(st[src][sl], AXIS[ax], o.order) / o.hd[ax]
            st[key] = b * st[key] + a * D
            dd.append(sign * (D / kap + st[key]))
        st[ename][_interior(ename)] += o.ci[ename] * (dd[0] + dd[1])


def _scatter(target, sl, g):
    view = target[sl]
    view += g


def adj_step(o, ad: dict) -> None:
    """Transpose of fwd_step, in place on the adjoint state ``ad`` (the
    multipliers of every field and memory variable).  The E part is undone
    first, then the H part.  For one stretched derivative d = D/kappa + psi',
    psi' = b psi + a D, the transpose maps (ad, apsi') to
    aD = ad/kappa + a (ad + apsi'),  apsi = b (ad + apsi')."""
    for ename in ("Ez", "Ey", "Ex"):
        g = ad[ename][_interior(ename)] * o.ci[ename]
        for key, src, ax, sl, sign in E_TERMS[ename]:
            kap, b, a = o.cp_int[ax]
            add = sign * g
            tot = ad[key] + add
            aD = add / kap + a * tot
            ad[key] = b * tot
            _scatter(ad[src], sl, diff_h_t(aD / o.hd[ax], AXIS[ax], o.order))
    for hname in ("Hz", "Hy", "Hx"):
        g = -o.dtmu * ad[hname]
        for key, src, ax, sl, sign in H_TERMS[hname]:
            kap, b, a = o.cp_half[ax]
            add = sign * g
            tot = ad[key] + add
            aD = add / kap + a * tot
            ad[key] = b * tot
            _scatter(ad[src], sl, diff_e_t(aD / o.h[ax], AXIS[ax], o.order))


def forward_states(s: Setup, inj: list, tfun: np.ndarray, nt: int):
    """E^0 .. E^nt of a driven run (fwd_step plus the injections of
    oracle.stepping: H += dt/mu w tfun[row, n] before the step for magnetic
    entries, E -= ce w tfun[row, n] after it for electric ones): list of
    (Ex, Ey, Ez)."""
    o = ops(s)
    st = zero_state(o)
    out = [tuple(np.zeros(o.shapes[c]) for c in ("Ex", "Ey", "Ez"))]
    names = FIELDS
    for n in range(nt):
        for (c, k, j, i, w, row) in inj:
            if c >= 3:
                st[names[c]][k, j, i] += o.dtmu * w * tfun[row, n]
        fwd_step(o, st)
        for (c, k, j, i, w, row) in inj:
            if c < 3:
                st[names[c]][k, j, i] -= s.ce[c][k, j, i] * w * tfun[row, n]
        out.append(tuple(st[c].copy() for c in names))
    return out


def adjoint_gradient_td(p, resid: np.ndarray, setup: Setup | None = None,
                        nt: int | None = None):
    """Gradient of phi_d = 1/2 ||W (d - E)||^2 with respect to ln(rho) by the
    time-domain adjoint.  resid = W^2 (d - E) [ns][nr][ncomp][nf].
    Returns dict(grad [nz][ny][nx], grad_sigma, grad_edges (d phi / d sigma_e
    per component))."""
    s = setup if setup is not None else make_setup(p)
    nt = s.nt if nt is None else nt
    o = ops(s)
    nodes, interp = receiver_nodes(s, np.asarray(p.rec_pos), p.rec_comp)
    kind = getattr(p, "src_kind", 0)
    # magnetic rows (components 3-5): H = norm_h sum_n H^{n+1/2} z^{n+1/2}
    norm, norm_h = source_norms(s, nt, kind)
    zm = np.exp(1j * np.outer(np.arange(nt + 1) * s.dt, s.wprime))   # z^m, m = 0..nt
    zh = np.exp(1j * np.outer((np.arange(nt) + 0.5) * s.dt, s.wprime))   # z^{n+1/2}
    names = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
    mag = np.array([c >= 3 for (c, _, _, _) in nodes], dtype=bool)
    ge = [np.zeros(s.sig_e[c].shape) for c in range(3)]
    for si in range(len(p.src_pos)):
        inj = source_injection(s, p.src_pos[si], p.src_mom[si], kind=kind)
        E = forward_states(s, inj, s.wavelet[None, :], nt)
        # E_rec = norm sum_nodes w sum_m E^m z^m, so d phi / d E^m(node) =
        # -Re sum_k c_node,k z_k^m with c_node,k = sum w conj(resid) norm_k
        cnode = np.zeros((len(nodes), len(norm)), dtype=np.complex128)
        for r in range(len(p.rec_pos)):
            for ci in range(len(p.rec_comp)):
                nrm = norm_h if p.rec_comp[ci] >= 3 else norm
                for ni, w in interp[r][ci]:
                    cnode[ni] += w * np.conj(resid[si, r, ci]) * nrm
        ad = zero_state(o)
        for n in range(nt - 1, -1, -1):
            m = n + 1
            # d phi / d E^{n+1} at E nodes, d phi / d H^{n+1/2} at H nodes
            # (H^{n+1/2} is produced by the H part of step n, which the
            # transposed step undoes after its E part)
            gm = np.where(mag, -np.real(cnode @ zh[n]), -np.real(cnode @ zm[m]))
            for ni, (c, k, j, i) in enumerate(nodes):
                ad[names[c]][k, j, i] += gm[ni]
            for c in range(3):
                sl = _interior(names[c])
                dE = E[m][c][sl] - E[n][c][sl]
                ge[c][sl] -= ad[names[c]][sl] * dE / s.sig_e[c][sl]
            adj_step(o, ad)
    g_sigma = edge_sigma_transpose(ge[0], ge[1], ge[2], s.hx, s.hy, s.hz)
    grad_h, grad_v = cell_gradient(s, ge[0], ge[1], ge[2])
    return {"grad": grad_h + grad_v, "grad_h": grad_h, "grad_v": grad_v,
            "grad_sigma": g_sigma, "grad_edges": tuple(ge)}
