"""Leapfrog time stepping with CPML, dipole injection and the on-the-fly DFT.

Follows Section 2 of the paper:
  * fictitious-domain Maxwell (eq. fictitiouswave):
        curl E' + mu dH'/dt' = M',     curl H' - eps dE'/dt' = J'
    stepped by the leapfrog
        H^{n+1/2} = H^{n-1/2} - (dt/mu) (curl E^n - M'^n)
        E^{n+1}   = E^n + (dt/eps) (curl H^{n+1/2} - J'^{n+1/2})
    with E^0 = 0, H^{-1/2} = 0 (zero initial state, Appendix);
  * the damped transform (eq. dft) accumulated while stepping:
        u(omega_k) = sum_n u^n z_k^n,  z_k = exp(i w'_k dt),
        w'_k = (1+i) sqrt(omega_k omega0)
    Reading of the sample times (the paper writes t'_n = n dt without
    saying where H and J' sit): E is sampled at n dt, H and J' at
    (n+1/2) dt.  The sum covers every E^n the Nt steps produce
    (n = 1..Nt; E^0 = 0 adds nothing);
  * the frequency-domain field of a source J is recovered from the
    fictitious source J' = sqrt(-i omega / 2 omega0) J (correspondence
    below eq. mittet): E(omega_k) = u(omega_k) sqrt(-i omega_k/2omega0)/W_k
    with W_k = sum_n w^{n+1/2} z_k^{n+1/2} the transform of the injected
    wavelet.  The same correspondence has H' = sqrt(-i omega/2omega0) H, so
    the magnetic field of the same source is H(omega_k) = u_H(omega_k)/W_k,
    u_H = sum_n H^{n+1/2} z_k^{n+1/2} (eq. dtft lists H' among the
    transformed fields; magnetic data enter the misfit eq. phid);
  * a magnetic current M' (the adjoint source of magnetic data, or a
    magnetic dipole source) enters the H update at n dt, the time of the
    curl E it sits beside;
  * magnetic dipole sources (M = m delta(x - x_s) in the Faraday row of
    eq. freq; M' = M by the correspondence below eq. mittet): the wavelet
    sample w_n is injected as M'^n = m w_n at n dt (reading: the paper fixes
    no forward time function; each source is normalised by the transform of
    what it injects, at the times it injects it), so
    E(omega_k) = u(omega_k) / W^M_k with W^M_k = sum_n w_n z_k^n, and
    H(omega_k) = u_H(omega_k) / (sqrt(-i omega_k / 2 omega0) W^M_k).
  * an option that is not the paper's: the volume transform decimated by D,
    D sum over m = D, 2D, ... of E^m z^m, a coarser Riemann sum of the
    integral of eq. dtft (receivers keep every sample).  Its error is the
    aliasing of the field's content above pi / (D dt); the forward field,
    driven by a wavelet many steps wide, has little there.
Receiver components: 0, 1, 2 = E_x, E_y, E_z; 3, 4, 5 = H_x, H_y, H_z.
Source kinds: 0 = electric dipoles (J), 1 = magnetic dipoles (M).
"""
from __future__ import annotations

import numpy as np

from .discretization import (MU0, Setup, dual_volumes, h_lattices, h_volumes, lattices,
                             make_setup, trilinear)
from .stencil import diff_e, diff_h


def _b(arr, axis, ndim=3):
    """Reshape a 1D profile to broadcast along ``axis`` (0=z, 1=y, 2=x)."""
    sh = [1] * ndim
    sh[axis] = -1
    return arr.reshape(sh)


def point_entries(s: Setup, comp: int, point) -> list:
    """Trilinear (k, j, i, weight) entries of a point on the lattice of
    component ``comp`` (0-2: E, 3-5: H)."""
    lat = lattices(s)[comp] if comp < 3 else h_lattices(s)[comp - 3]
    return [(k, j, i, w) for (k, j, i), w in trilinear(point, *lat)]


def run_stepping(s: Setup, inj: list, tfun: np.ndarray, rec_nodes: list,
                 want_volume: bool, nt: int | None = None, decimate: int = 1):
    """Run the leapfrog for ``nt`` steps (default s.nt).

    inj       list of (comp, k, j, i, weight, row): at step n an E edge
              (comp 0-2) receives J'^{n+1/2} = weight * tfun[row, n], an H
              node (comp 3-5) M'^n = weight * tfun[row, n] (weights already
              divided by the dual volume of the edge or node).
    rec_nodes list of (comp, k, j, i) whose raw transforms are returned.
    decimate  D >= 1: the volume transform takes only the samples E^m with
              m a multiple of D, each weighted by D (the decimated transform;
              D = 1 is eq. dft).  Receiver transforms always take every
              sample.
    Returns (rec_acc [len(rec_nodes), nf], volume [3][nf, ...] or None) with
    the raw sums sum_n E^n z^n (E nodes) and sum_n H^{n+1/2} z^{n+1/2}
    (H nodes)."""
    nt = s.nt if nt is None else nt
    nx, ny, nz = s.nx, s.ny, s.nz
    nf = len(s.freqs)
    Ex = np.zeros((nz + 1, ny + 1, nx))
    Ey = np.zeros((nz + 1, ny, nx + 1))
    Ez = np.zeros((nz, ny + 1, nx + 1))
    Hx = np.zeros((nz, ny, nx + 1))
    Hy = np.zeros((nz, ny + 1, nx))
    Hz = np.zeros((nz + 1, ny, nx))
    (kxn, bxn, axn), (kxh, bxh, axh) = s.cpml["x"]
    (kyn, byn, ayn), (kyh, byh, ayh) = s.cpml["y"]
    (kzn, bzn, azn), (kzh, bzh, azh) = s.cpml["z"]
    # metric lengths of the differences (cell and dual widths for order 2)
    hx, hy, hz = _b(s.mx, 2), _b(s.my, 1), _b(s.mz, 0)
    hdx, hdy, hdz = _b(s.mdx[1:-1], 2), _b(s.mdy[1:-1], 1), _b(s.mdz[1:-1], 0)
    od = s.order

    # CPML memory variables, one per derivative (full size for clarity)
    psi = {
        "Hx_y": np.zeros(Hx.shape), "Hx_z": np.zeros(Hx.shape),
        "Hy_z": np.zeros(Hy.shape), "Hy_x": np.zeros(Hy.shape),
        "Hz_x": np.zeros(Hz.shape), "Hz_y": np.zeros(Hz.shape),
        "Ex_y": np.zeros((nz - 1, ny - 1, nx)), "Ex_z": np.zeros((nz - 1, ny - 1, nx)),
        "Ey_z": np.zeros((nz - 1, ny, nx - 1)), "Ey_x": np.zeros((nz - 1, ny, nx - 1)),
        "Ez_x": np.zeros((nz, ny - 1, nx - 1)), "Ez_y": np.zeros((nz, ny - 1, nx - 1)),
    }

    def stretched(D, key, kap, b, a, axis):
        # K&M CPML: psi <- b psi + a D ; D -> D/kappa + psi
        p = psi[key]
        p *= _b(b, axis)
        p += _b(a, axis) * D
        return D / _b(kap, axis) + p

    cx, cy, cz = s.ce
    cxi, cyi, czi = cx[1:-1, 1:-1, :], cy[1:-1, :, 1:-1], cz[:, 1:-1, 1:-1]
    dtmu = s.dt / MU0
    E = (Ex, Ey, Ez)
    ce_full = (cx, cy, cz)

    zE = np.exp(1j * np.outer((np.arange(nt) + 1.0) * s.dt, s.wprime))   # z^{n+1}
    zH = np.exp(1j * np.outer((np.arange(nt) + 0.5) * s.dt, s.wprime))   # z^{n+1/2}
    H = (Hx, Hy, Hz)
    rec_acc = np.zeros((len(rec_nodes), nf), dtype=np.complex128)
    vol = None
    if want_volume:
        vol = [np.zeros((nf,) + a.shape, dtype=np.complex128) for a in E]

    for n in range(nt):
        # H^{n+1/2} = H^{n-1/2} - dt/mu (curl E^n - M'^n)
        for (c, k, j, i, w, row) in inj:
            if c >= 3:
                H[c - 3][k, j, i] += dtmu * w * tfun[row, n]
        dEz_dy = stretched(diff_e(Ez, 1, od) / hy, "Hx_y", kyh, byh, ayh, 1)
        dEy_dz = stretched(diff_e(Ey, 0, od) / hz, "Hx_z", kzh, bzh, azh, 0)
        Hx -= dtmu * (dEz_dy - dEy_dz)
        dEx_dz = stretched(diff_e(Ex, 0, od) / hz, "Hy_z", kzh, bzh, azh, 0)
        dEz_dx = stretched(diff_e(Ez, 2, od) / hx, "Hy_x", kxh, bxh, axh, 2)
        Hy -= dtmu * (dEx_dz - dEz_dx)
        dEy_dx = stretched(diff_e(Ey, 2, od) / hx, "Hz_x", kxh, bxh, axh, 2)
        dEx_dy = stretched(diff_e(Ex, 1, od) / hy, "Hz_y", kyh, byh, ayh, 1)
        Hz -= dtmu * (dEy_dx - dEx_dy)
        # damped DFT of H^{n+1/2}
        for r, (c, k, j, i) in enumerate(rec_nodes):
            if c >= 3:
                rec_acc[r] += H[c - 3][k, j, i] * zH[n]

        # E^{n+1} = E^n + dt/eps (curl H^{n+1/2} - J'^{n+1/2}); interior edges only
        dHz_dy = stretched(diff_h(Hz[1:-1], 1, od) / hdy, "Ex_y",
                           kyn[1:-1], byn[1:-1], ayn[1:-1], 1)
        dHy_dz = stretched(diff_h(Hy[:, 1:-1], 0, od) / hdz, "Ex_z",
                           kzn[1:-1], bzn[1:-1], azn[1:-1], 0)
        Ex[1:-1, 1:-1, :] += cxi * (dHz_dy - dHy_dz)
        dHx_dz = stretched(diff_h(Hx[:, :, 1:-1], 0, od) / hdz, "Ey_z",
                           kzn[1:-1], bzn[1:-1], azn[1:-1], 0)
        dHz_dx = stretched(diff_h(Hz[1:-1], 2, od) / hdx, "Ey_x",
                           kxn[1:-1], bxn[1:-1], axn[1:-1], 2)
        Ey[1:-1, :, 1:-1] += cyi * (dHx_dz - dHz_dx)
        dHy_dx = stretched(diff_h(Hy[:, 1:-1], 2, od) / hdx, "Ez_x",
                           kxn[1:-1], bxn[1:-1], axn[1:-1], 2)
        dHx_dy = stretched(diff_h(Hx[:, :, 1:-1], 1, od) / hdy, "Ez_y",
                           kyn[1:-1], byn[1:-1], ayn[1:-1], 1)
        Ez[:, 1:-1, 1:-1] += czi * (dHy_dx - dHx_dy)
        for (c, k, j, i, w, row) in inj:
            if c < 3:
                E[c][k, j, i] -= ce_full[c][k, j, i] * w * tfun[row, n]

        # damped DFT of E^{n+1}
        zn = zE[n]
        for r, (c, k, j, i) in enumerate(rec_nodes):
            if c < 3:
                rec_acc[r] += E[c][k, j, i] * zn
        if vol is not None and (n + 1) % decimate == 0:
            for c in range(3):
                vol[c] += decimate * zn[:, None, None, None] * E[c][None]
    return rec_acc, vol


def source_injection(s: Setup, pos, mom, row: int = 0, kind: int = 0) -> list:
    """Injection entries of a point dipole of moment ``mom`` at ``pos``.
    kind 0, electric (J = p delta(x - x_s), eq. freq): each component is
    spread over its E lattice with trilinear weights, divided by the dual
    volume of the edge it lands on.  kind 1, magnetic (M = m delta(x - x_s)):
    the same over the H lattices and the volumes of the H nodes (under which
    the Faraday and Ampere rows form a symmetric pair); entries carry
    components 3-5."""
    vols = dual_volumes(s) if kind == 0 else h_volumes(s)
    inj = []
    for c in range(3):
        if mom[c] == 0.0:
            continue
        cc = c + 3 * kind
        for (k, j, i, w) in point_entries(s, cc, pos):
            inj.append((cc, k, j, i, mom[c] * w / vols[c][k, j, i], row))
    return inj


def source_norms(s: Setup, nt: int, kind: int = 0):
    """(norm_e, norm_h) [nf]: the factors that turn the raw transforms of a
    run of ``nt`` steps into the fields of a unit dipole, for E rows and H
    rows.  Electric sources inject w^{n+1/2} as J' (transform W_k over
    (n+1/2) dt) with J' = sqrt(-i omega / 2 omega0) J; magnetic sources
    inject w_n as M' = M at n dt (transform W^M_k over n dt).  In both,
    H = H' / sqrt(-i omega / 2 omega0)."""
    fac = np.sqrt(-1j * s.omega / (2.0 * s.omega0))
    if kind == 0:
        if nt != s.nt:
            th = (np.arange(nt) + 0.5) * s.dt
            norm = fac / (s.wavelet[:nt] @ np.exp(1j * np.outer(th, s.wprime)))
        else:
            norm = s.norm
    else:
        tn = np.arange(nt) * s.dt
        norm = 1.0 / (s.wavelet[:nt] @ np.exp(1j * np.outer(tn, s.wprime)))
    return norm, norm / fac


def receiver_nodes(s: Setup, rec_pos, rec_comp):
    """Unique lattice nodes touched by the receivers and, per (receiver,
    component), the list of (node index, weight) interpolating the field."""
    nodes, index, interp = [], {}, []
    for r, pos in enumerate(rec_pos):
        per = []
        for c in rec_comp:
            lst = []
            for (k, j, i, w) in point_entries(s, c, pos):
                key = (c, k, j, i)
                if key not in index:
                    index[key] = len(nodes)
                    nodes.append(key)
                lst.append((index[key], w))
            per.append(lst)
        interp.append(per)
    return nodes, interp


def forward(p, want_volume: bool = False, setup: Setup | None = None,
            nt: int | None = None, decimate: int | None = None):
    """Frequency-domain fields at the receivers (and optionally E in the
    volume) for every source of problem ``p``: one leapfrog run per source.

    Returns dict with
      setup  the Setup used
      E_rec  complex [ns][nr][ncomp][nf]  (eq. freq field of the dipole,
             electric or magnetic as p.src_kind says (default electric);
             the components p.rec_comp, E or H)
      vol    per source, [3][nf, ...] normalised volume fields (if asked)."""
    s = setup if setup is not None else make_setup(p)
    nt = s.nt if nt is None else nt
    nodes, interp = receiver_nodes(s, np.asarray(p.rec_pos), p.rec_comp)
    ns = len(p.src_pos)
    ncomp = len(p.rec_comp)
    nf = len(s.freqs)
    kind = getattr(p, "src_kind", 0)
    dec = int(decimate or getattr(p, "dft_decimate", 1))
    # the normalisation uses the wavelet transform over the steps run
    norm, norm_h = source_norms(s, nt, kind)
    E_rec = np.zeros((ns, len(p.rec_pos), ncomp, nf), dtype=np.complex128)
    vols = []
    for si in range(ns):
        inj = source_injection(s, p.src_pos[si], p.src_mom[si], kind=kind)
        acc, vol = run_stepping(s, inj, s.wavelet[None, :], nodes, want_volume, nt, dec)
        for r in range(len(p.rec_pos)):
            for ci in range(ncomp):
                val = sum(w * acc[ni] for ni, w in interp[r][ci])
                E_rec[si, r, ci] = val * (norm if p.rec_comp[ci] < 3 else norm_h)
        if vol is not None:
            vols.append([v * norm[:, None, None, None] for v in vol])
    return {"setup": s, "E_rec": E_rec, "vol": vols if want_volume else None,
            "norm": norm, "decimate": dec}
