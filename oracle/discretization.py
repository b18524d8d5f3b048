"""Discretisation of the fictitious-wave-domain Maxwell system (oracle side).

Section 2 of the paper: the diffusive frequency-domain Maxwell equations
(eq. freq) become a lossless wave system (eq. fictitiouswave) once the
conductivity is read as a fictitious permittivity, sigma = 2 omega0 eps
(eq. mittet and the correspondence below it).  The wave system is stepped by
a staggered-grid leapfrog on a tensor grid with absorbing CPML layers
(Section 2, the paragraph on the modelling engine) and the damped transform
(eq. dtft / eq. dft) is accumulated on the fly.

Grid conventions (readings, where the paper gives no detail):
  * nx, ny, nz cells; node coordinates x[0..nx], y[0..ny], z[0..nz].
  * E_x lives on the edge (x_{i+1/2}, y_j, z_k), E_y on (x_i, y_{j+1/2}, z_k),
    E_z on (x_i, y_j, z_{k+1/2}); H_x on the face (x_i, y_{j+1/2}, z_{k+1/2}),
    H_y on (x_{i+1/2}, y_j, z_{k+1/2}), H_z on (x_{i+1/2}, y_{j+1/2}, z_k).
  * Tangential E on the outer boundary is held at zero.
  * Second-order differences: across a cell the width h, across a node the
    dual width hd (mean of the two adjacent cell widths; half a cell at the
    outer nodes).  The paper's engine is higher order; second order is the
    reading used here.
  * Edge conductivity: volume-weighted mean of the cells around the edge.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .stencil import metric_half, metric_node

MU0 = 4.0e-7 * np.pi

# CPML defaults (the paper cites Komatitsch & Martin 2007 without values).
CPML_ORDER = 2.0
CPML_R = 1.0e-6
CPML_KAPPA_MAX = 1.0
CPML_ALPHA_MAX_FACTOR = 0.5   # alpha_max = factor * a_min (a = sqrt(omega omega0))
NT_TOL = 1.0e-11              # exp(-a_min * Nt * dt) at the last step


def dual_widths(nodes: np.ndarray) -> np.ndarray:
    """Dual widths at the nodes: mean of adjacent cell widths, half a cell
    at the two end nodes."""
    h = np.diff(nodes)
    hd = np.empty(len(nodes))
    hd[1:-1] = 0.5 * (h[:-1] + h[1:])
    hd[0] = 0.5 * h[0]
    hd[-1] = 0.5 * h[-1]
    return hd


def avg_matrix(h: np.ndarray) -> np.ndarray:
    """(n+1) x n matrix M with M[j, j'] = h[j'] for the cells j' in {j-1, j}
    adjacent to node j: the unnormalised volume weights of the averaging
    from cells onto nodes along one axis."""
    n = len(h)
    m = np.zeros((n + 1, n))
    for j in range(n):
        m[j, j] = h[j]
        m[j + 1, j] = h[j]
    return m


def edge_sigma(sig: np.ndarray, hx, hy, hz):
    """Volume-weighted mean conductivity on the E_x, E_y, E_z edges.

    The dual cell of an edge is shared by the (up to four) cells that touch
    the edge; each cell counts with the part of the dual volume it covers.
    Returns (sx, sy, sz) with shapes (nz+1, ny+1, nx), (nz+1, ny, nx+1),
    (nz, ny+1, nx+1)."""
    Mx, My, Mz = avg_matrix(hx), avg_matrix(hy), avg_matrix(hz)
    sx = np.einsum("Kk,Jj,kji->KJi", Mz, My, sig, optimize=True)
    sx /= (Mz.sum(1)[:, None, None] * My.sum(1)[None, :, None])
    sy = np.einsum("Kk,Ii,kji->KjI", Mz, Mx, sig, optimize=True)
    sy /= (Mz.sum(1)[:, None, None] * Mx.sum(1)[None, None, :])
    sz = np.einsum("Jj,Ii,kji->kJI", My, Mx, sig, optimize=True)
    sz /= (My.sum(1)[None, :, None] * Mx.sum(1)[None, None, :])
    return sx, sy, sz


def cell_gradient(s, gx, gy, gz):
    """d phi / d ln rho on cells from d phi / d sigma_e on the edges:
    through the transpose of the averaging and the chain rule
    d / d ln rho = -sigma d / d sigma (Section 3.5).  In VTI (Section 3.1)
    the x and y edges give the gradient for rho_h, the z edges for rho_v.
    Returns (grad_h, grad_v); capped cells get zero."""
    zx, zy, zz = np.zeros_like(gx), np.zeros_like(gy), np.zeros_like(gz)
    g_h = edge_sigma_transpose(gx, gy, zz, s.hx, s.hy, s.hz)
    g_v = edge_sigma_transpose(zx, zy, gz, s.hx, s.hy, s.hz)
    grad_h = -s.sigma * g_h
    grad_v = -s.sigma_v * g_v
    grad_h[s.capped] = 0.0
    grad_v[s.capped_v] = 0.0
    return grad_h, grad_v


def edge_sigma_transpose(gx, gy, gz, hx, hy, hz):
    """Exact transpose of ``edge_sigma``: maps edge quantities g_e to cells,
    sum_e g_e d sigma_e / d sigma_c (used to scatter the edge gradient)."""
    Mx, My, Mz = avg_matrix(hx), avg_matrix(hy), avg_matrix(hz)
    dx = Mz.sum(1)[:, None, None] * My.sum(1)[None, :, None]
    dy = Mz.sum(1)[:, None, None] * Mx.sum(1)[None, None, :]
    dz = My.sum(1)[None, :, None] * Mx.sum(1)[None, None, :]
    out = np.einsum("Kk,Jj,KJi->kji", Mz, My, gx / dx, optimize=True)
    out += np.einsum("Kk,Ii,KjI->kji", Mz, Mx, gy / dy, optimize=True)
    out += np.einsum("Jj,Ii,kJI->kji", My, Mx, gz / dz, optimize=True)
    return out


def cfl_dt(sig, hx, hy, hz, omega0, cfl, order=2):
    """Time step from the CFL bound of the fictitious wave system, taken cell
    by cell: dt <= 1 / (v sqrt(1/hx^2 + 1/hy^2 + 1/hz^2)) with
    v = 1/sqrt(mu eps) and eps = sigma / (2 omega0) (Section 2; the paper
    notes dt ~ dx in the fictitious domain and that resistive cells shrink
    it, Section 5).  Order 4 divides the bound by |9/8| + |1/24| = 7/6, the
    growth of the largest symbol of the staggered difference."""
    eps = sig / (2.0 * omega0)
    v = 1.0 / np.sqrt(MU0 * eps)
    inv = np.sqrt(hx[None, None, :] ** -2 + hy[None, :, None] ** -2
                  + hz[:, None, None] ** -2)
    if order == 4:
        inv = inv * (7.0 / 6.0)
    return cfl * float(np.min(1.0 / (v * inv))), float(np.max(v))


def cpml_profile(nodes, npml, dt, vref, order, R, kappa_max, alpha_max):
    """CPML coefficients (kappa, b, a) at the integer nodes and at the half
    nodes of one axis (unsplit convolutional PML of Komatitsch & Martin 2007,
    cited in Section 2).  Inside the layer of npml cells at each end the
    damping grows as d0 r^order with the normalised depth r; d0 =
    -(order+1) vref ln(R) / (2 L); kappa = 1 + (kappa_max-1) r^order;
    alpha = alpha_max (1 - r).  The memory variable obeys
    psi <- b psi + a D and the derivative D is replaced by D/kappa + psi."""
    n = len(nodes) - 1
    xl, xr = nodes[npml], nodes[n - npml]
    Ll, Lr = max(xl - nodes[0], 1e-300), max(nodes[n] - xr, 1e-300)

    def coeffs(p):
        r = np.zeros_like(p)
        L = np.ones_like(p)
        left = p < xl
        right = p > xr
        r[left] = (xl - p[left]) / Ll
        r[right] = (p[right] - xr) / Lr
        L[left] = Ll
        L[right] = Lr
        inside = left | right
        d0 = -(order + 1.0) * vref * np.log(R) / (2.0 * L)
        d = np.where(inside, d0 * r ** order, 0.0)
        kap = np.where(inside, 1.0 + (kappa_max - 1.0) * r ** order, 1.0)
        alp = np.where(inside, alpha_max * (1.0 - r), 0.0)
        b = np.exp(-(d / kap + alp) * dt)
        den = kap * (d + kap * alp)
        a = np.where(d > 0.0, d * (b - 1.0) / np.where(d > 0.0, den, 1.0), 0.0)
        b = np.where(inside, b, 0.0)
        return kap, b, a

    integer = coeffs(nodes.copy())
    half = coeffs(0.5 * (nodes[:-1] + nodes[1:]))
    return integer, half


def trilinear(point, lat_x, lat_y, lat_z):
    """Trilinear weights of ``point`` on the lattice lat_x x lat_y x lat_z.
    Returns a list of ((k, j, i), weight) with non-zero weights.  Used both
    for receiver interpolation and for source spreading so that source and
    receiver play symmetric roles (reading: the paper's restriction operator
    R samples the field at the receiver, Section 3.1)."""
    out = []
    idx_w = []
    for p, lat in zip(point, (lat_x, lat_y, lat_z)):
        if p < lat[0] or p > lat[-1]:
            raise ValueError("point outside the lattice")
        i = int(np.searchsorted(lat, p, side="right") - 1)
        i = min(i, len(lat) - 2)
        t = (p - lat[i]) / (lat[i + 1] - lat[i])
        idx_w.append(((i, 1.0 - t), (i + 1, t)))
    for (i, wi) in idx_w[0]:
        for (j, wj) in idx_w[1]:
            for (k, wk) in idx_w[2]:
                w = wi * wj * wk
                if w != 0.0:
                    out.append(((k, j, i), w))
    return out


@dataclass
class Setup:
    nx: int
    ny: int
    nz: int
    npml: int
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    hx: np.ndarray
    hy: np.ndarray
    hz: np.ndarray
    hdx: np.ndarray
    hdy: np.ndarray
    hdz: np.ndarray
    sigma: np.ndarray          # capped cell conductivity (horizontal, sigma_h, in VTI)
    capped: np.ndarray         # bool: cell resistivity above the cap
    sig_e: tuple               # edge conductivities (x, y, z)
    ce: tuple                  # dt / eps on the edges (x, y, z)
    dt: float
    nt: int
    f0: float
    omega0: float
    freqs: np.ndarray
    omega: np.ndarray
    a: np.ndarray              # sqrt(omega omega0)
    wprime: np.ndarray         # (1+i) a
    Omega: np.ndarray          # (2/dt) sin(w' dt/2)
    vmax: float
    vref: float
    cpml: dict                 # axis -> (integer (kap,b,a), half (kap,b,a))
    wavelet: np.ndarray        # w((n+1/2) dt), n = 0..nt-1
    tau: float
    t0: float
    What: np.ndarray           # sum_n w^{n+1/2} z^{n+1/2}
    norm: np.ndarray           # sqrt(-i omega / 2 omega0) / What
    sigma_v: np.ndarray = None  # vertical conductivity (VTI); = sigma when isotropic
    capped_v: np.ndarray = None
    order: int = 2             # order of the staggered differences (2 or 4)
    mx: np.ndarray = None      # metric lengths at the half nodes (= hx for order 2)
    my: np.ndarray = None
    mz: np.ndarray = None
    mdx: np.ndarray = None     # metric lengths at the nodes (= hdx for order 2)
    mdy: np.ndarray = None
    mdz: np.ndarray = None


def make_setup(p, dt: float | None = None, nt: int | None = None) -> Setup:
    """Host setup for a problem ``p`` (any object with the attributes of a
    workload: x, y, z, rho, freqs, npml, f0, nt, dt, cfl, rho_air_cap and
    optional cpml_* overrides)."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (p.x, p.y, p.z))
    hx, hy, hz = np.diff(x), np.diff(y), np.diff(z)
    nx, ny, nz = len(hx), len(hy), len(hz)
    rho = np.asarray(p.rho, dtype=np.float64)
    assert rho.shape == (nz, ny, nx)
    cap = float(p.rho_air_cap)
    capped = rho > cap
    sigma = 1.0 / np.minimum(rho, cap)                   # reading: air as capped cells
    # VTI (Section 2): sigma_h = sigma_xx = sigma_yy, sigma_v = sigma_zz
    rho_v = getattr(p, "rho_v", None)
    if rho_v is None:
        sigma_v, capped_v = sigma, capped
    else:
        rho_v = np.asarray(rho_v, dtype=np.float64)
        assert rho_v.shape == rho.shape
        capped_v = rho_v > cap
        sigma_v = 1.0 / np.minimum(rho_v, cap)
    f0 = float(p.f0)
    omega0 = 2.0 * np.pi * f0
    freqs = np.asarray(p.freqs, dtype=np.float64)
    omega = 2.0 * np.pi * freqs
    a = np.sqrt(omega * omega0)
    wprime = (1.0 + 1.0j) * a                            # eq. mittet correspondence

    order = int(getattr(p, "fd_order", 2) or 2)
    if order not in (2, 4):
        raise ValueError("fd_order must be 2 or 4")
    # reading (VTI): the bound of each cell taken with its faster (more
    # resistive) direction
    dt_cfl, vmax = cfl_dt(np.minimum(sigma, sigma_v), hx, hy, hz, omega0, float(p.cfl), order)
    if dt is None:
        dt = float(p.dt) if getattr(p, "dt", 0.0) else dt_cfl
    if nt is None:
        nt = int(p.nt) if getattr(p, "nt", 0) else int(np.ceil(np.log(1.0 / NT_TOL) / (a.min() * dt)))

    sx, sy, sz = edge_sigma(sigma, hx, hy, hz)
    if rho_v is not None:
        sz = edge_sigma(sigma_v, hx, hy, hz)[2]      # z edges see sigma_v
    ce = tuple(dt * 2.0 * omega0 / s for s in (sx, sy, sz))   # dt/eps, eps = sigma/(2 omega0)

    vref = float(getattr(p, "cpml_vref", 0.0) or vmax)
    cpml_order = float(getattr(p, "cpml_order", CPML_ORDER))
    R = float(getattr(p, "cpml_R", CPML_R))
    kmax = float(getattr(p, "cpml_kappa_max", CPML_KAPPA_MAX))
    amax = float(getattr(p, "cpml_alpha_max", 0.0) or CPML_ALPHA_MAX_FACTOR * a.min())
    npml = int(p.npml)
    cp = {ax: cpml_profile(nodes, npml, dt, vref, cpml_order, R, kmax, amax)
          for ax, nodes in (("x", x), ("y", y), ("z", z))}

    # source wavelet: derivative of a Gaussian, sampled at (n+1/2) dt
    # (reading: the paper leaves the forward wavelet open; the normalised
    # result does not depend on it).
    tau = max(0.25 / a.max(), 3.0 * dt)
    t0 = 5.0 * tau
    th = (np.arange(nt) + 0.5) * dt
    u = (th - t0) / tau
    wav = -u * np.exp(-0.5 * u * u)
    zh = np.exp(1j * np.outer(th, wprime))               # z^{n+1/2} = exp(i w' t_{n+1/2})
    What = wav @ zh
    norm = np.sqrt(-1j * omega / (2.0 * omega0)) / What  # J' = sqrt(-i w / 2 w0) J
    Omega = (2.0 / dt) * np.sin(wprime * dt / 2.0)

    return Setup(nx=nx, ny=ny, nz=nz, npml=npml, x=x, y=y, z=z, hx=hx, hy=hy,
                 hz=hz, hdx=dual_widths(x), hdy=dual_widths(y),
                 hdz=dual_widths(z), sigma=sigma, capped=capped,
                 sig_e=(sx, sy, sz), ce=ce, dt=dt, nt=nt, f0=f0,
                 omega0=omega0, freqs=freqs, omega=omega, a=a, wprime=wprime,
                 Omega=Omega, vmax=vmax, vref=vref, cpml=cp, wavelet=wav,
                 tau=tau, t0=t0, What=What, norm=norm, sigma_v=sigma_v,
                 capped_v=capped_v, order=order,
                 mx=metric_half(x, order), my=metric_half(y, order), mz=metric_half(z, order),
                 mdx=metric_node(x, order), mdy=metric_node(y, order), mdz=metric_node(z, order))


def lattices(s: Setup):
    """Coordinates of the E_x, E_y, E_z lattices as (lat_x, lat_y, lat_z)."""
    xh = 0.5 * (s.x[:-1] + s.x[1:])
    yh = 0.5 * (s.y[:-1] + s.y[1:])
    zh = 0.5 * (s.z[:-1] + s.z[1:])
    return ((xh, s.y, s.z), (s.x, yh, s.z), (s.x, s.y, zh))


def h_lattices(s: Setup):
    """Coordinates of the H_x, H_y, H_z lattices (component 3, 4, 5 of a
    receiver): each H component sits on the node of its own axis and at the
    cell centres of the other two."""
    xh = 0.5 * (s.x[:-1] + s.x[1:])
    yh = 0.5 * (s.y[:-1] + s.y[1:])
    zh = 0.5 * (s.z[:-1] + s.z[1:])
    return ((s.x, yh, zh), (xh, s.y, zh), (xh, yh, s.z))


def h_volumes(s: Setup):
    """Dual volume of every H node: the metric node length along its own
    axis times the metric cell lengths of the other two.  Under these weights
    and those of dual_volumes the Faraday and Ampere rows form a symmetric
    system, so a magnetic adjoint source is spread with w / volume exactly
    as an electric one."""
    vx = s.mz[:, None, None] * s.my[None, :, None] * s.mdx[None, None, :]
    vy = s.mz[:, None, None] * s.mdy[None, :, None] * s.mx[None, None, :]
    vz = s.mdz[:, None, None] * s.my[None, :, None] * s.mx[None, None, :]
    return vx, vy, vz


def dual_volumes(s: Setup):
    """Dual volume of every E edge: edge length times dual face area, in
    the metric lengths of the differences (the weights under which the
    discrete curl pair is adjoint; cell and dual widths for order 2)."""
    vx = s.mdz[:, None, None] * s.mdy[None, :, None] * s.mx[None, None, :]
    vy = s.mdz[:, None, None] * s.my[None, :, None] * s.mdx[None, None, :]
    vz = s.mz[:, None, None] * s.mdy[None, :, None] * s.mdx[None, None, :]
    return vx, vy, vz
