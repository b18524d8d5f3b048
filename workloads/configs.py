"""Workload definitions: grids, resistivity models and survey layouts.

Every array here is an *input* of the modelling method.  Coordinates are in
metres, z is depth (positive down, the sea/land surface at z = 0, air above),
resistivity in ohm-metres, frequencies in Hz, dipole moments in ampere-metres.

The five named workloads follow the paper's scales (0.3 ohm-m sea water,
1-2.5 ohm-m sediments, a 100 ohm-m thin reservoir, 0.1-2.25 Hz, offsets of
several km; Section 4 "Application examples").  The paper's own marine model
and data are not available, so these are seeded synthetic stand-ins.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

RHO_AIR = 1.0e8


@dataclass
class Workload:
    name: str
    x: np.ndarray                 # node coordinates, nx+1
    y: np.ndarray                 # ny+1
    z: np.ndarray                 # nz+1
    rho: np.ndarray               # cell resistivity [nz][ny][nx] (horizontal, if rho_v is set)
    freqs: np.ndarray             # Hz
    src_pos: np.ndarray           # [ns][3]
    src_mom: np.ndarray           # [ns][3]  (A m)
    rec_pos: np.ndarray           # [nr][3]
    rec_comp: tuple = (0, 1)      # recorded components (0-2: E_x,E_y,E_z; 3-5: H_x,H_y,H_z)
    npml: int = 8
    f0: float = 1.0
    nt: int = 0                   # 0: derived from the damping of the lowest frequency
    dt: float = 0.0               # 0: derived from the CFL bound
    cfl: float = 0.95
    rho_air_cap: float = 1.0e4
    field_dtype: str = "f32"      # hint: the precision the workload is run in
    acc_mode: str = "f64"
    extra: dict = field(default_factory=dict)
    rho_v: np.ndarray | None = None   # vertical resistivity (VTI); None: isotropic
    fd_order: int = 2             # order of the staggered differences (2 or 4)
    src_kind: int = 0             # 0: electric dipoles (J, moments in A m); 1: magnetic (M, V m)

    @property
    def shape(self):
        return (len(self.z) - 1, len(self.y) - 1, len(self.x) - 1)

    @property
    def ncells(self):
        nz, ny, nx = self.shape
        return nx * ny * nz

    @property
    def ns(self):
        return int(self.src_pos.shape[0])

    @property
    def nr(self):
        return int(self.rec_pos.shape[0])

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def axis_nodes(origin: float, h: float, n_core: int, n_lo: int = 0,
               n_hi: int = 0, ratio: float = 1.0) -> np.ndarray:
    """Nodes of a tensor-grid axis: n_core uniform cells of width h starting
    at ``origin``, with n_lo / n_hi cells growing geometrically by ``ratio``
    below / above the core (Section 4: constant growth factor away from the
    densely sampled zone)."""
    core = origin + h * np.arange(n_core + 1, dtype=np.float64)
    lo = [core[0]]
    w = h
    for _ in range(n_lo):
        w *= ratio
        lo.append(lo[-1] - w)
    hi = [core[-1]]
    w = h
    for _ in range(n_hi):
        w *= ratio
        hi.append(hi[-1] + w)
    return np.concatenate([np.array(lo[:0:-1]), core, np.array(hi[1:])])


def _cell_centres(nodes):
    return 0.5 * (nodes[:-1] + nodes[1:])


def c1_wholespace(n: int = 32, h: float = 100.0, nt: int = 2000) -> Workload:
    """Homogeneous 1 S/m whole space, uniform 32^3 grid of 100 m cells, an
    x-directed unit dipole on the centre E_x edge, one frequency (0.25 Hz),
    20 receivers on E_x edges 2-6 cells inline, broadside, diagonal and
    below the source."""
    half = n // 2
    x = axis_nodes(-(half + 0.5) * h, h, n)      # E_x edge centres at multiples of h
    y = axis_nodes(-half * h, h, n)
    z = axis_nodes(-half * h, h, n)
    rho = np.ones((n, n, n))
    recs = []
    for m in range(2, 7):
        recs.append((m * h, 0.0, 0.0))          # inline
        recs.append((0.0, m * h, 0.0))          # broadside
        recs.append((m * h, m * h, 0.0))        # diagonal
        recs.append((0.0, 0.0, m * h))          # below
    return Workload(name="c1_wholespace", x=x, y=y, z=z, rho=rho,
                    freqs=np.array([0.25]),
                    src_pos=np.array([[0.0, 0.0, 0.0]]),
                    src_mom=np.array([[1.0, 0.0, 0.0]]),
                    rec_pos=np.array(recs, dtype=np.float64),
                    rec_comp=(0, 1, 2), nt=nt, field_dtype="f64",
                    acc_mode="f64", rho_air_cap=1.0e8)


def _marine_layers(z_nodes, water_depth, reservoir_top, reservoir_thick,
                   rho_sed=1.0, rho_res=100.0, rho_water=0.3):
    """Cell resistivity of a 1D marine column: air (z<0), water, sediment
    and a thin resistive layer."""
    zc = _cell_centres(z_nodes)
    col = np.full(zc.shape, rho_sed)
    col[zc < water_depth] = rho_water
    col[zc < 0.0] = RHO_AIR
    res = (zc > reservoir_top) & (zc < reservoir_top + reservoir_thick)
    col[res] = rho_res
    return col


def c2_marine1d() -> Workload:
    """1D layered marine model: air above 300 m of 0.3 ohm-m sea water, 1
    ohm-m sediment, a 100 ohm-m reservoir 100 m thick 1000 m below the
    seabed; 101x101x61 grid of 100 m core cells stretched outward by 1.05;
    0.25/0.75/1.25 Hz; x-dipole 50 m above the seabed; 50 seabed receivers
    every 100 m along the tow line."""
    x = axis_nodes(-3050.0, 100.0, 61, 20, 20, 1.05)
    y = axis_nodes(-3000.0, 100.0, 61, 20, 20, 1.05)
    z = axis_nodes(0.0, 100.0, 16, 12, 33, 1.05)
    nx, ny, nz = len(x) - 1, len(y) - 1, len(z) - 1
    col = _marine_layers(z, 300.0, 1300.0, 100.0)
    rho = np.broadcast_to(col[:, None, None], (nz, ny, nx)).copy()
    recs = np.array([(-2500.0 + 100.0 * m, 0.0, 300.0) for m in range(50)])
    return Workload(name="c2_marine1d", x=x, y=y, z=z, rho=rho,
                    freqs=np.array([0.25, 0.75, 1.25]),
                    src_pos=np.array([[0.0, 0.0, 250.0]]),
                    src_mom=np.array([[1.0, 0.0, 0.0]]),
                    rec_pos=recs, rec_comp=(0, 1))


def c3_blocks(seed: int = 0) -> Workload:
    """1 S/m background on a 128x128x96 grid (100 m core, ratio 1.05) with 3
    random resistive blocks (log10 rho ~ U[0,2], sizes U[300,1000] m per
    axis, centres in the core at least 300 m from the source); one x-dipole
    and 64 receivers on an 8x8 plane 300 m below it."""
    rng = np.random.default_rng(seed)
    x = axis_nodes(-4450.0, 100.0, 88, 20, 20, 1.05)
    y = axis_nodes(-4400.0, 100.0, 88, 20, 20, 1.05)
    z = axis_nodes(-3200.0, 100.0, 64, 16, 16, 1.05)
    xc, yc, zc = _cell_centres(x), _cell_centres(y), _cell_centres(z)
    rho = np.ones((len(zc), len(yc), len(xc)))
    nb = 0
    while nb < 3:
        size = rng.uniform(300.0, 1000.0, 3)
        ctr = np.array([rng.uniform(-3000, 3000), rng.uniform(-3000, 3000),
                        rng.uniform(-2000, 2000)])
        if np.linalg.norm(ctr) < 300.0 + 0.5 * np.linalg.norm(size):
            continue
        lr = rng.uniform(0.0, 2.0)
        mx = np.abs(xc - ctr[0]) < size[0] / 2
        my = np.abs(yc - ctr[1]) < size[1] / 2
        mz = np.abs(zc - ctr[2]) < size[2] / 2
        rho[np.ix_(mz, my, mx)] = 10.0 ** lr
        nb += 1
    g = -1400.0 + 400.0 * np.arange(8)
    recs = np.array([(gx, gy, 300.0) for gy in g for gx in g])
    return Workload(name="c3_blocks", x=x, y=y, z=z, rho=rho,
                    freqs=np.array([0.25, 0.75, 1.25]),
                    src_pos=np.array([[0.0, 0.0, 0.0]]),
                    src_mom=np.array([[1.0, 0.0, 0.0]]),
                    rec_pos=recs, rec_comp=(0, 1), rho_air_cap=1.0e8,
                    extra={"snapshot_every": 200})


def c4_batched() -> Workload:
    """Marine physics as c2 on a 200x200x100 grid; 16 x-dipoles every 250 m
    along the tow line, 50 m above the seabed; 100 seabed receivers every
    100 m; 5 frequencies 0.1-1.25 Hz."""
    x = axis_nodes(-8000.0, 100.0, 160, 20, 20, 1.05)
    y = axis_nodes(-8000.0, 100.0, 160, 20, 20, 1.05)
    z = axis_nodes(0.0, 100.0, 30, 20, 50, 1.05)
    nx, ny, nz = len(x) - 1, len(y) - 1, len(z) - 1
    col = _marine_layers(z, 300.0, 1300.0, 100.0)
    rho = np.broadcast_to(col[:, None, None], (nz, ny, nx)).copy()
    srcs = np.array([(-1875.0 + 250.0 * m, 0.0, 250.0) for m in range(16)])
    moms = np.tile([1.0, 0.0, 0.0], (16, 1))
    recs = np.array([(-5000.0 + 100.0 * m, 0.0, 300.0) for m in range(100)])
    return Workload(name="c4_batched", x=x, y=y, z=z, rho=rho,
                    freqs=np.array([0.1, 0.25, 0.5, 0.75, 1.25]),
                    src_pos=srcs, src_mom=moms, rec_pos=recs, rec_comp=(0, 1))


def _gaussian_random_field(shape, cell, corr, rng):
    """Zero-mean, unit-variance Gaussian random field on a uniform lattice
    with a Gaussian correlation of length ``corr`` (white noise filtered by
    a Gaussian kernel in the Fourier domain)."""
    noise = rng.standard_normal(shape)
    ks = [np.fft.fftfreq(n, d=cell) * 2 * np.pi for n in shape]
    kk = np.zeros(shape)
    for ax, k in enumerate(ks):
        sh = [1] * len(shape)
        sh[ax] = -1
        kk = kk + k.reshape(sh) ** 2
    filt = np.exp(-kk * corr ** 2 / 8.0)
    f = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    f -= f.mean()
    return f / f.std()


def c5_large(seed: int = 2) -> Workload:
    """400x400x200 grid (about 32M cells): air and water as c2, sediment ln
    rho a Gaussian random field (geometric mean 1 ohm-m, std 0.5, correlation
    500 m), a 100 ohm-m 2x2 km x 100 m reservoir 1000 m below the seabed;
    8 log-spaced frequencies 0.1-2 Hz; 32 x-dipoles every 250 m; 400
    receivers on a 20x20 seabed array at 500 m."""
    rng = np.random.default_rng(seed)
    x = axis_nodes(-18000.0, 100.0, 360, 20, 20, 1.05)
    y = axis_nodes(-18000.0, 100.0, 360, 20, 20, 1.05)
    z = axis_nodes(0.0, 100.0, 100, 20, 80, 1.05)
    xc, yc, zc = _cell_centres(x), _cell_centres(y), _cell_centres(z)
    nx, ny, nz = len(xc), len(yc), len(zc)
    grf = _gaussian_random_field((nz, ny, nx), 100.0, 500.0, rng)
    rho = np.exp(0.5 * grf)
    rho[zc < 300.0, :, :] = 0.3
    rho[zc < 0.0, :, :] = RHO_AIR
    mz = (zc > 1300.0) & (zc < 1400.0)
    my = np.abs(yc) < 1000.0
    mx = np.abs(xc) < 1000.0
    rho[np.ix_(mz, my, mx)] = 100.0
    srcs = np.array([(-3875.0 + 250.0 * m, 0.0, 250.0) for m in range(32)])
    moms = np.tile([1.0, 0.0, 0.0], (32, 1))
    g = -4750.0 + 500.0 * np.arange(20)
    recs = np.array([(gx, gy, 300.0) for gy in g for gx in g])
    return Workload(name="c5_large", x=x, y=y, z=z, rho=rho,
                    freqs=np.geomspace(0.1, 2.0, 8), src_pos=srcs,
                    src_mom=moms, rec_pos=recs, rec_comp=(0, 1),
                    acc_mode="kahan")


def tiny(seed: int = 0, n=(14, 12, 10), npml: int = 3, ns: int = 1,
         nfreq: int = 2, stretch: float = 1.15, contrast: float = 1.0,
         nr: int = 6, rec_comp=(0, 1, 2), off_grid: bool = True,
         moment_dirs: bool = False) -> Workload:
    """Small seeded workload for exactness and gradient tests: a randomly
    stretched tensor grid, a random heterogeneous model (log10 rho spread
    ``contrast``), sources and receivers at random off-grid positions inside
    the non-absorbing interior."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n

    def ax(m):
        w = 100.0 * stretch ** rng.uniform(-1, 1, m)
        nodes = np.concatenate([[0.0], np.cumsum(w)])
        return nodes - nodes[m // 2]

    x, y, z = ax(nx), ax(ny), ax(nz)
    rho = 10.0 ** rng.uniform(0.0, contrast, (nz, ny, nx))

    def inner_point():
        lo = npml + 1
        p = []
        for nodes in (x, y, z):
            m = len(nodes) - 1
            a, b = nodes[lo], nodes[m - lo]
            p.append(rng.uniform(a, b) if off_grid else nodes[rng.integers(lo, m - lo)])
        return p

    srcs = np.array([inner_point() for _ in range(ns)])
    if moment_dirs:
        moms = rng.standard_normal((ns, 3))
    else:
        moms = np.tile([1.0, 0.0, 0.0], (ns, 1))
    recs = np.array([inner_point() for _ in range(nr)])
    freqs = np.sort(rng.uniform(0.2, 1.5, nfreq))
    return Workload(name=f"tiny{seed}", x=x, y=y, z=z, rho=rho, freqs=freqs,
                    src_pos=srcs, src_mom=moms, rec_pos=recs,
                    rec_comp=tuple(rec_comp), npml=npml, field_dtype="f64",
                    rho_air_cap=1.0e8)


def with_vti(w: Workload, ratio: float = 2.0, seed: int | None = None,
             rho_min: float = 0.9) -> Workload:
    """The same workload made vertically transverse isotropic (VTI): the
    vertical resistivity of every cell with rho >= rho_min (sediment,
    reservoir; not water or air) is ``ratio`` times the horizontal one, or,
    with a seed, times a random factor in [1, ratio]."""
    rv = w.rho.copy()
    sel = w.rho >= rho_min
    if seed is None:
        rv[sel] *= ratio
    else:
        rng = np.random.default_rng(seed)
        rv[sel] *= rng.uniform(1.0, ratio, int(sel.sum()))
    return w.replace(rho_v=rv, name=f"{w.name}_vti")


def with_window(w: Workload, nt: int) -> Workload:
    """The same workload stopped after ``nt`` steps (a window of the full
    run, used where the full run is too long for the CPU oracle)."""
    return w.replace(nt=int(nt), name=f"{w.name}_nt{nt}")


_BY_NAME = {
    "c1_wholespace": c1_wholespace,
    "c2_marine1d": c2_marine1d,
    "c3_blocks": c3_blocks,
    "c4_batched": c4_batched,
    "c5_large": c5_large,
}


def by_name(name: str) -> Workload:
    return _BY_NAME[name]()
