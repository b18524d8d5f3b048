"""Pins of the oracle's fourth-order staggered differences (the paper's engine
is high order on the stretched grid, Section 2).

The one-dimensional differences are pinned by polynomials (exact for cubics
on a uniform grid, for linear functions on any stretched grid), by their
fourth-order convergence, by the transposes the time-domain adjoint uses,
and by the adjointness of the E -> H and H -> E pair under the metric
weighting.  The stepped system is pinned by the sparse direct solve of its
frequency-domain identity (tests/pins/fdsolve.py, whose order-4 rows are
assembled entry by entry from the image rules), by reciprocity, by the
closed-form whole-space dipole (order 4 much closer than order 2 at the
same cells), by the CFL bound, and the gradients (basis-function and
time-domain adjoint) by central differences.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint_td as td
from oracle import stencil as st
from oracle.discretization import make_setup
from oracle.stepping import point_entries, run_stepping, source_injection
from tests.pins.dipole import dipole_field_discrete_time
from tests.pins.fdsolve import solve as fd_solve
from tests.test_oracle_td import _dot_test
from workloads import c1_wholespace, tiny


def _stretched_nodes(n, h0=1.0, ratio=1.06, seed=0):
    rng = np.random.default_rng(seed)
    h = h0 * ratio ** np.arange(n) * (1 + 0.02 * rng.standard_normal(n))
    return np.concatenate([[0.0], np.cumsum(h)])


def test_uniform_grid_metrics_are_the_spacing():
    x = np.arange(11) * 2.5
    assert np.allclose(st.metric_half(x, 4), 2.5, rtol=1e-14)
    assert np.allclose(st.metric_node(x, 4)[1:-1], 2.5, rtol=1e-14)


def test_cubics_exact_on_a_uniform_grid_and_linear_exact_when_stretched():
    x = np.arange(13) * 0.7
    c = 0.5 * (x[:-1] + x[1:])
    # the rows next to the walls use images; the others see the plain cubic
    f = lambda t: 0.3 * t ** 3 - t ** 2 + 2 * t - 1.0          # noqa: E731
    df = lambda t: 0.9 * t ** 2 - 2 * t + 2                    # noqa: E731
    de = st.diff_e(f(x), 0, 4) / st.metric_half(x, 4)
    assert np.allclose(de[1:-1], df(c)[1:-1], rtol=1e-12)
    dh = st.diff_h(f(c), 0, 4) / st.metric_node(x, 4)[1:-1]
    assert np.allclose(dh[1:-1], df(x[1:-1])[1:-1], rtol=1e-12)
    xs = _stretched_nodes(15)
    cs = 0.5 * (xs[:-1] + xs[1:])
    de = st.diff_e(3.0 * xs + 1.0, 0, 4) / st.metric_half(xs, 4)
    dh = st.diff_h(3.0 * cs + 1.0, 0, 4) / st.metric_node(xs, 4)[1:-1]
    assert np.allclose(de[1:-1], 3.0, rtol=1e-12) and np.allclose(dh[1:-1], 3.0, rtol=1e-12)


def test_fourth_order_convergence_on_a_uniform_grid():
    errs = []
    for n in (16, 32):
        x = np.linspace(0.0, 1.0, n + 1)
        c = 0.5 * (x[:-1] + x[1:])
        d = st.diff_e(np.sin(3 * x), 0, 4) / st.metric_half(x, 4)
        errs.append(np.abs(d - 3 * np.cos(3 * c))[2:-2].max())
    assert errs[0] / errs[1] > 14.0                 # 16 for the exact order


@pytest.mark.parametrize("order", [2, 4])
def test_transposes_and_adjoint_pair(order):
    rng = np.random.default_rng(1)
    n = 9
    F = rng.standard_normal((3, n + 1, 4))
    H = rng.standard_normal((3, n, 4))
    g = rng.standard_normal((3, n, 4))
    gi = rng.standard_normal((3, n - 1, 4))
    assert np.isclose(np.sum(st.diff_e(F, 1, order) * g), np.sum(F * st.diff_e_t(g, 1, order)))
    assert np.isclose(np.sum(st.diff_h(H, 1, order) * gi), np.sum(H * st.diff_h_t(gi, 1, order)))
    # with E zero on the walls, the H -> E difference is minus the transpose
    # of the E -> H difference
    F[:, 0] = 0.0
    F[:, -1] = 0.0
    lhs = np.sum(st.diff_e(F, 1, order) * H)
    rhs = -np.sum(F[:, 1:-1] * st.diff_h(H, 1, order))
    assert np.isclose(lhs, rhs, rtol=1e-13)


@pytest.mark.parametrize("seed,npml,contrast", [(0, 3, 1.0), (1, 0, 1.0)])
def test_order4_stepping_equals_sparse_solve(seed, npml, contrast):
    w = tiny(seed=seed, npml=npml, contrast=contrast, ns=2, moment_dirs=True).replace(fd_order=4)
    res = oracle.forward(w)
    s = res["setup"]
    for kf, f in enumerate(w.freqs):
        ref = fd_solve(w.x, w.y, w.z, w.rho, w.npml, w.f0, f, s.dt,
                       list(zip(w.src_pos, w.src_mom)), w.rec_pos, w.rec_comp,
                       s.vref, alpha_max=0.5 * s.a.min(), order=4)
        err = np.abs(res["E_rec"][..., kf] - ref).max() / np.abs(ref).max()
        assert err < 1e-9, (f, err)
        ref2 = fd_solve(w.x, w.y, w.z, w.rho, w.npml, w.f0, f, s.dt,
                        list(zip(w.src_pos, w.src_mom)), w.rec_pos, w.rec_comp,
                        s.vref, alpha_max=0.5 * s.a.min(), order=2)
        assert np.abs(ref2 - ref).max() > 1e-3 * np.abs(ref).max()   # the orders differ


def test_order4_reciprocity_off_grid():
    w = tiny(seed=4, npml=3, contrast=1.5, nr=1).replace(fd_order=4)
    A, B = w.src_pos[0], w.rec_pos[0]
    out = {}
    for (src, rec) in ((A, B), (B, A)):
        for a in range(3):
            mom = np.zeros(3)
            mom[a] = 1.0
            ww = w.replace(src_pos=np.array([src]), src_mom=np.array([mom]),
                           rec_pos=np.array([rec]), rec_comp=(0, 1, 2))
            out[(tuple(src), a)] = oracle.forward(ww)["E_rec"][0, 0]
    for a in range(3):
        for b in range(3):
            gab, gba = out[(tuple(A), a)][b], out[(tuple(B), b)][a]
            assert np.allclose(gab, gba, rtol=1e-9, atol=1e-12 * np.abs(gab).max())


@pytest.mark.slow
def test_order4_is_closer_to_the_closed_form_dipole():
    """Whole space, 1 S/m, 0.25 Hz, 100 m and 50 m cells: at receivers beyond
    300 m the order-4 error is below 1 % (median) and 5 % (max) on the coarse
    grid, at least ten times below order 2's median, and shrinks with h."""
    def errs(n, h, order):
        w = c1_wholespace(n=n, h=h, nt=600).replace(npml=8, rec_pos=c1_wholespace().rec_pos,
                                                    fd_order=order)
        res = oracle.forward(w)
        s = res["setup"]
        E = res["E_rec"][0][..., 0]
        ref = dipole_field_discrete_time(w.rec_pos, [1, 0, 0], 1.0, s.omega[0], s.omega0,
                                         s.Omega[0])
        return (np.abs(E - ref).max(1) / np.abs(ref).max(1),
                np.linalg.norm(w.rec_pos, axis=1))
    e2, r = errs(32, 100.0, 2)
    e4, _ = errs(32, 100.0, 4)
    e4f, _ = errs(48, 50.0, 4)
    far = r >= 300.0
    assert np.median(e4[far]) < 0.01 and e4[far].max() < 0.05
    assert np.median(e2[far]) > 10.0 * np.median(e4[far])
    assert np.median(e4f[far]) < 0.25 * np.median(e4[far]) and e4f[far].max() < 0.01


def test_order4_cfl_bound():
    """The order-4 step is 6/7 of the order-2 step; running at twice it
    blows up, running at it for 300 steps does not."""
    w = tiny(seed=7, npml=2, n=(10, 10, 10))
    s2 = make_setup(w)
    s4 = make_setup(w.replace(fd_order=4))
    assert np.isclose(s4.dt, s2.dt * 6.0 / 7.0, rtol=1e-12)
    node = [(0,) + tuple(point_entries(s4, 0, w.rec_pos[0])[0][:3])]
    bad = make_setup(w.replace(fd_order=4), dt=2.0 * s4.dt / 0.95, nt=300)
    inj = source_injection(bad, w.src_pos[0], w.src_mom[0])
    with np.errstate(over="ignore", invalid="ignore"):
        acc, _ = run_stepping(bad, inj, bad.wavelet[None, :], node, False)
    assert not np.all(np.isfinite(acc)) or np.abs(acc).max() > 1e20
    good = make_setup(w.replace(fd_order=4), nt=300)
    inj = source_injection(good, w.src_pos[0], w.src_mom[0])
    acc, _ = run_stepping(good, inj, good.wavelet[None, :], node, False)
    assert np.all(np.isfinite(acc)) and np.abs(acc).max() < 1.0


@pytest.mark.parametrize("npml", [0, 3])
def test_order4_transposed_step_passes_dot_product_test(npml):
    w = tiny(seed=2, npml=npml, contrast=1.5, stretch=1.3).replace(fd_order=4)
    assert _dot_test(w) < 1e-13


def _problem(seed=3):
    w_true = tiny(seed=seed, n=(14, 12, 10), npml=3, contrast=1.0, nr=8,
                  nfreq=2).replace(fd_order=4)
    rng = np.random.default_rng(seed + 100)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    return w0, d


@pytest.mark.slow
def test_order4_gradients_match_finite_differences():
    """Both adjoints at order 4: central differences in ln rho agree to 1e-5
    (time-domain) and 1e-4 (basis-function) on interior cells, and the two
    gradients agree outside the CPML layers."""
    w0, d = _problem()
    fwd = oracle.forward(w0, want_volume=True)
    resid = d - fwd["E_rec"]
    gb = oracle.adjoint_gradient(w0, fwd, resid)["grad"]
    gt = td.adjoint_gradient_td(w0, resid)["grad"]
    h = 1e-3
    for c in [(4, 5, 6), (5, 5, 5), (6, 4, 8)]:
        vals = []
        for sgn in (1, -1):
            rho = w0.rho.copy()
            rho[c] *= np.exp(sgn * h)
            wp = w0.replace(rho=rho)
            wp.cpml_vref = w0.cpml_vref
            vals.append(oracle.misfit(oracle.forward(wp)["E_rec"], d))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gt[c]) < 1e-5 * abs(fd), (c, fd, gt[c])
        assert abs(fd - gb[c]) < 1e-4 * abs(fd), (c, fd, gb[c])
    m = w0.npml
    inner = (slice(m, -m),) * 3
    assert np.linalg.norm((gt - gb)[inner]) < 1e-9 * np.linalg.norm(gb[inner])


def test_sparse_solve_catches_a_wrong_image(monkeypatch):
    """Plant: the E -> H difference continues E evenly across the walls
    (instead of oddly); the identity with the sparse solve must break."""
    import oracle.stepping as stepping
    w = tiny(seed=0, npml=0, ns=1, moment_dirs=True).replace(fd_order=4)
    s = make_setup(w)
    ref = fd_solve(w.x, w.y, w.z, w.rho, w.npml, w.f0, w.freqs[0], s.dt,
                   list(zip(w.src_pos, w.src_mom)), w.rec_pos, w.rec_comp, s.vref,
                   alpha_max=0.5 * s.a.min(), order=4)

    def even_images(F, axis, order):
        G = np.moveaxis(F, axis, -1)
        ext = np.concatenate([G[..., 1:2], G, G[..., -2:-1]], axis=-1)
        d = st.C1 * (G[..., 1:] - G[..., :-1]) + st.C2 * (ext[..., 3:] - ext[..., :-3])
        return np.moveaxis(d, -1, axis)
    monkeypatch.setattr(stepping, "diff_e", even_images)
    bad = oracle.forward(w)["E_rec"][..., 0]
    assert np.abs(bad - ref).max() > 1e-6 * np.abs(ref).max()
