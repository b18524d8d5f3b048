"""Pins of the oracle's magnetic-data path against what the mathematics fixes.

Magnetic data are receiver components 3, 4, 5 (H_x, H_y, H_z), weighted by
W2 in the misfit (eq. phid).  The forward field is H = u_H / W_k with
u_H = sum_n H^{n+1/2} z^{n+1/2}.  The adjoint source of a magnetic residual
is a magnetic current in the M' slot with coefficients conj(resid) z^{1/2}.
The pins are:
  * the closed-form magnetic field of a dipole, checked against the curl of
    the closed-form electric field and against Biot-Savart in the static
    limit;
  * the exact frequency-domain identity of the stepped system: the sparse
    solve, which takes H from its Faraday row;
  * the whole-space dipole, with second-order convergence in h;
  * two independent adjoints: the basis-function adjoint against the
    time-domain adjoint of the Appendix (exact derivative of the stepped
    misfit), both against central finite differences.
Some tests plant a mistake in the oracle (on the CPU): a half-step shift of
the H samples, no z^{1/2} on the magnetic coefficients, or the electric
factor on them.  Each plant must break its pin.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
from oracle import adjoint_td as td
from oracle.discretization import make_setup
from tests.pins.dipole import (MU0, dipole_field, magnetic_field,
                               magnetic_field_discrete_time, wavenumber)
from tests.pins.fdsolve import solve as fd_solve
from workloads import c1_wholespace, tiny


# --------------------------------------------------------------------------
# the closed form itself
# --------------------------------------------------------------------------
def _curl(f, p, h):
    J = np.zeros((3, 3), dtype=np.complex128)
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        J[:, b] = (f(p + e) - f(p - e)) / (2 * h)
    return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])


@pytest.mark.parametrize("pt", [(350.0, 120.0, -80.0), (-90.0, 600.0, 210.0),
                                (40.0, -30.0, 900.0)])
def test_closed_form_h_is_the_faraday_row(pt):
    """curl E = i omega mu H for the closed-form pair (eq. freq, M = 0)."""
    sigma, omega = 0.7, 2 * np.pi * 0.5
    k = wavenumber(omega, sigma)
    p = np.array([0.3, -1.0, 0.4])
    pt = np.array(pt)
    curl_e = _curl(lambda q: dipole_field(q, p, k, sigma), pt, 0.05)
    H = magnetic_field(pt, p, k)
    assert np.abs(curl_e - 1j * omega * MU0 * H).max() < 1e-6 * np.abs(omega * MU0 * H).max()


def test_closed_form_h_static_limit():
    """As omega -> 0, H tends to the Biot-Savart field of a current element:
    H = p x r / (4 pi r^3)."""
    r = np.array([300.0, -200.0, 100.0])
    p = np.array([1.0, 0.5, -0.3])
    H = magnetic_field(r, p, wavenumber(1e-12, 2.0))
    H0 = np.cross(p, r) / (4 * np.pi * np.linalg.norm(r) ** 3)
    assert np.allclose(H, H0, rtol=1e-6, atol=0)


# --------------------------------------------------------------------------
# exact identity of the stepped system
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,npml,contrast,order", [(0, 3, 1.0, 2), (1, 0, 1.0, 2),
                                                      (2, 3, 2.0, 2), (3, 3, 1.0, 4)])
def test_h_receivers_equal_sparse_solve(seed, npml, contrast, order):
    w = tiny(seed=seed, npml=npml, contrast=contrast, ns=2, moment_dirs=True,
             rec_comp=(0, 3, 4, 5)).replace(fd_order=order)
    res = oracle.forward(w)
    s = res["setup"]
    for kf, f in enumerate(w.freqs):
        ref = fd_solve(w.x, w.y, w.z, w.rho, w.npml, w.f0, f, s.dt,
                       list(zip(w.src_pos, w.src_mom)), w.rec_pos, w.rec_comp,
                       s.vref, alpha_max=0.5 * s.a.min(), order=order)
        for ci in range(len(w.rec_comp)):
            got = res["E_rec"][:, :, ci, kf]
            err = np.abs(got - ref[:, :, ci]).max() / np.abs(ref[:, :, ci]).max()
            assert err < 1e-9, (f, w.rec_comp[ci], err)


def test_h_half_step_sampling_is_what_the_identity_fixes():
    """Plant: H samples taken at (n+1) dt instead of (n+1/2) dt, i.e. the
    sums multiplied by z^{1/2}.  The sparse solve rejects it by far more than
    its tolerance."""
    w = tiny(seed=0, npml=3, rec_comp=(3, 4, 5))
    res = oracle.forward(w)
    s = res["setup"]
    ref = fd_solve(w.x, w.y, w.z, w.rho, w.npml, w.f0, w.freqs[0], s.dt,
                   list(zip(w.src_pos, w.src_mom)), w.rec_pos, w.rec_comp,
                   s.vref, alpha_max=0.5 * s.a.min())
    shifted = res["E_rec"][..., 0] * np.exp(0.5j * s.wprime[0] * s.dt)
    err = np.abs(shifted - ref).max() / np.abs(ref).max()
    assert err > 1e-3


# --------------------------------------------------------------------------
# physics: whole-space dipole
# --------------------------------------------------------------------------
def _c1_h_errors(n, h, nt):
    w = c1_wholespace(n=n, h=h, nt=nt).replace(npml=8, rec_pos=c1_wholespace().rec_pos,
                                               rec_comp=(3, 4, 5))
    res = oracle.forward(w)
    s = res["setup"]
    H = res["E_rec"][0][..., 0]
    ref = magnetic_field_discrete_time(w.rec_pos, [1, 0, 0], 1.0, s.omega0, s.Omega[0])
    scale = np.abs(ref).max(1)
    r = np.linalg.norm(w.rec_pos, axis=1)
    off = scale > 1e-3 * scale.max()          # inline receivers see no H
    err = np.abs(H - ref).max(1)[off] / scale[off]
    m = np.abs(ref).argmax(1)[off]
    i = np.arange(len(H))[off]
    ph = np.degrees(np.angle(H[i, m] / ref[i, m]))
    return err, ph, r[off], np.abs(H[~off]).max() / scale.max()


def test_h_wholespace_closed_form_and_convergence():
    """Config c1 (sigma = 1 S/m, 0.25 Hz), magnetic components: the oracle
    approaches the closed form with second-order accuracy in h, as E does.
    Inline receivers see no H (r_hat x p = 0), and neither does the oracle.
    On 100 m cells the error is a near-field one (28 % at 3 cells, 6 % at 6
    cells broadside; E has 37 % and 9 % there) and the phase is within 1
    degree.  Halving the cell cuts every error above 5 % at 300 m or more by
    more than 4x, and the fine grid is within 2 % from 500 m."""
    e1, p1, r, inline1 = _c1_h_errors(32, 100.0, 600)
    e2, p2, _, _ = _c1_h_errors(48, 50.0, 600)
    far = r >= 300.0
    assert inline1 < 1e-12
    assert np.abs(p1).max() < 1.0 and np.abs(p2).max() < 0.3
    assert e1[r >= 500.0].max() < 0.1 and e2[r >= 500.0].max() < 0.02
    big = far & (e1 > 0.05)
    assert big.sum() >= 6
    assert np.all(e1[big] / e2[big] > 4.0), (e1[big], e2[big])
    assert np.all(e2[far] < e1[far])


# --------------------------------------------------------------------------
# adjoint and gradient with magnetic data
# --------------------------------------------------------------------------
def _problem(rec_comp, seed=3):
    w_true = tiny(seed=seed, n=(14, 12, 10), npml=3, contrast=1.0, nr=8, nfreq=2,
                  rec_comp=rec_comp)
    rng = np.random.default_rng(seed + 100)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    return w0, d


def _basis_vs_td(w0, d):
    fwd = oracle.forward(w0, want_volume=True)
    resid = d - fwd["E_rec"]
    g_b = oracle.adjoint_gradient(w0, fwd, resid)["grad"]
    g_t = td.adjoint_gradient_td(w0, resid)["grad"]
    m = w0.npml
    inner = (slice(m, -m),) * 3
    return np.linalg.norm((g_t - g_b)[inner]) / np.linalg.norm(g_b[inner]), g_b, g_t


@pytest.mark.parametrize("rec_comp", [(3, 4, 5), (0, 4, 5)])
def test_magnetic_basis_gradient_equals_time_domain_gradient(rec_comp):
    """The basis-function adjoint (M' sources with conj(resid) z^{1/2}) and
    the time-domain adjoint (d phi / d H^{n+1/2} into the H multipliers)
    agree on every cell outside the CPML layers, for magnetic data alone and
    mixed with electric data."""
    w0, d = _problem(rec_comp)
    err, _, _ = _basis_vs_td(w0, d)
    assert err < 1e-9, err


def _fd(w0, d, c, h):
    vals = []
    for sgn in (1, -1):
        rho = w0.rho.copy()
        rho[c] *= np.exp(sgn * h)
        wp = w0.replace(rho=rho)
        wp.cpml_vref = w0.cpml_vref
        vals.append(oracle.misfit(oracle.forward(wp)["E_rec"], d))
    return (vals[0] - vals[1]) / (2 * h)


@pytest.mark.slow
def test_magnetic_gradients_match_finite_differences():
    """Magnetic data only: both gradients against central differences,
    h = 1e-3 in ln rho on interior cells (1e-5 for the time-domain adjoint,
    1e-4 for the basis-function one), and the time-domain one on a CPML cell
    (h = 1e-2, 1e-4)."""
    w0, d = _problem((3, 4, 5))
    _, g_b, g_t = _basis_vs_td(w0, d)
    for c in [(5, 5, 5), (4, 7, 6)]:
        fd = _fd(w0, d, c, 1e-3)
        assert abs(fd - g_t[c]) / abs(fd) < 1e-5, (c, fd, g_t[c])
        assert abs(fd - g_b[c]) / abs(fd) < 1e-4, (c, fd, g_b[c])
    c = (5, 7, 2)                                       # x index < npml = 3
    fd = _fd(w0, d, c, 1e-2)
    assert abs(fd - g_t[c]) / abs(fd) < 1e-4, (c, fd, g_t[c])


def test_magnetic_adjoint_catches_planted_mistakes(monkeypatch):
    """Dropping z^{1/2} from the magnetic coefficients (M' placed as if it
    acted at the J' times) or giving them the electric factor sqrt(-i w/2w0)
    breaks the agreement with the time-domain adjoint by far more than its
    tolerance."""
    w0, d = _problem((3, 4, 5))
    orig = adj.source_factors

    def no_shift(s, rec_comp):
        f = orig(s, rec_comp)
        mag = np.asarray(rec_comp) >= 3
        return np.where(mag[:, None], 1.0 + 0j, f)
    monkeypatch.setattr(adj, "source_factors", no_shift)
    err, _, _ = _basis_vs_td(w0, d)
    assert err > 1e-4, err

    def electric(s, rec_comp):
        return orig(s, [0] * len(rec_comp))
    monkeypatch.setattr(adj, "source_factors", electric)
    err, _, _ = _basis_vs_td(w0, d)
    assert err > 0.1, err
