"""Pins of the oracle's magnetic dipole sources (M in the Faraday row of
eq. freq; M' = M by the correspondence below eq. mittet) against what the
mathematics fixes, sharing no code with the oracle:
  * the closed-form field of a magnetic dipole in a whole space
    (tests/pins/dipole.py), checked against both rows of eq. freq and its
    static limit;
  * the exact frequency-domain identity of the stepped system (the sparse
    solve of tests/pins/fdsolve.py with M' on the H nodes): E and H
    receivers to 1e-9, orders 2 and 4;
  * the whole-space magnetic dipole with second-order convergence in h;
  * reciprocity between the two source kinds: H_b at B from an electric
    dipole p_a at A equals E_a at A from a magnetic dipole m_b at B (Lorentz
    reciprocity of eq. freq), on the discrete system exactly;
  * the basis-function gradient against the time-domain adjoint.
Planted mistakes (in the oracle, on the CPU) must break their pins: the
magnetic wavelet normalised at (n+1/2) dt as for J', the E dual volumes in
place of the H node volumes, and the sign of M' in the H update.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint_td as td
from oracle import discretization as disc
from oracle import stepping
from oracle.discretization import make_setup
from tests.pins.dipole import (MU0, dipole_field, magnetic_dipole_discrete_time,
                               magnetic_dipole_e, magnetic_dipole_h, wavenumber)
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
def test_closed_form_magnetic_dipole_obeys_both_rows(pt):
    """Away from the source: curl E = i omega mu H (Faraday, M = 0 there) and
    curl H = sigma E (Ampere, J = 0)."""
    sigma, omega = 0.7, 2 * np.pi * 0.5
    k = wavenumber(omega, sigma)
    m = np.array([0.3, -1.0, 0.4])
    pt = np.array(pt)
    E = magnetic_dipole_e(pt, m, k)
    H = magnetic_dipole_h(pt, m, k, sigma, omega)
    curl_e = _curl(lambda q: magnetic_dipole_e(q, m, k), pt, 0.05)
    curl_h = _curl(lambda q: magnetic_dipole_h(q, m, k, sigma, omega), pt, 0.05)
    assert np.abs(curl_e - 1j * omega * MU0 * H).max() < 1e-6 * np.abs(omega * MU0 * H).max()
    assert np.abs(curl_h - sigma * E).max() < 1e-6 * np.abs(sigma * E).max()


def test_closed_form_magnetic_dipole_static_limit():
    """As omega -> 0, E tends to the dual of Biot-Savart, m x r / (4 pi r^3)."""
    r = np.array([300.0, -200.0, 100.0])
    m = np.array([1.0, 0.5, -0.3])
    E = magnetic_dipole_e(r, m, wavenumber(1e-12, 2.0))
    E0 = np.cross(m, r) / (4 * np.pi * np.linalg.norm(r) ** 3)
    assert np.allclose(E, E0, rtol=1e-6, atol=0)


# --------------------------------------------------------------------------
# exact identity of the stepped system
# --------------------------------------------------------------------------
def _mag_tiny(seed, npml, order=2, rec_comp=(0, 1, 2, 3, 4, 5)):
    return tiny(seed=seed, npml=npml, ns=2, moment_dirs=True,
                rec_comp=rec_comp).replace(fd_order=order, src_kind=1)


def _solve(w, s, kf):
    return fd_solve(w.x, w.y, w.z, w.rho, w.npml, w.f0, w.freqs[kf], s.dt,
                    list(zip(w.src_pos, w.src_mom)), w.rec_pos, w.rec_comp,
                    s.vref, alpha_max=0.5 * s.a.min(), order=w.fd_order, src_kind=w.src_kind)


def _max_rel(got, ref):
    return max(np.abs(got[:, :, ci] - ref[:, :, ci]).max() / np.abs(ref[:, :, ci]).max()
               for ci in range(ref.shape[2]))


@pytest.mark.parametrize("seed,npml,order", [(3, 3, 2), (4, 0, 2), (3, 3, 4)])
def test_magnetic_source_equals_sparse_solve(seed, npml, order):
    """E and H receivers of magnetic dipoles (random directions, off-grid)
    against the sparse solve, every frequency."""
    w = _mag_tiny(seed, npml, order)
    res = oracle.forward(w)
    s = res["setup"]
    for kf in range(len(w.freqs)):
        assert _max_rel(res["E_rec"][..., kf], _solve(w, s, kf)) < 1e-9


def test_plant_magnetic_wavelet_at_half_steps(monkeypatch):
    """Plant: the magnetic source normalised by the transform over
    (n+1/2) dt (the J' times) without the J' factor.  The identity rejects it."""
    w = _mag_tiny(3, 3)
    orig = stepping.source_norms

    def planted(s, nt, kind=0):
        ne, nh = orig(s, nt, kind)
        if kind == 1:
            shift = np.exp(-0.5j * s.wprime * s.dt)
            return ne * shift, nh * shift
        return ne, nh
    monkeypatch.setattr(stepping, "source_norms", planted)
    res = oracle.forward(w)
    assert _max_rel(res["E_rec"][..., 0], _solve(w, res["setup"], 0)) > 1e-3


def test_plant_edge_volumes_for_magnetic_sources(monkeypatch):
    """Plant: magnetic moments divided by the E edges' dual volumes."""
    w = _mag_tiny(3, 3)
    monkeypatch.setattr(stepping, "h_volumes", disc.dual_volumes)
    res = oracle.forward(w)
    assert _max_rel(res["E_rec"][..., 0], _solve(w, res["setup"], 0)) > 1e-3


def test_plant_sign_of_magnetic_current(monkeypatch):
    """Plant: M' subtracted from H instead of added."""
    w = _mag_tiny(3, 3)
    orig = stepping.source_injection

    def planted(s, pos, mom, row=0, kind=0):
        inj = orig(s, pos, mom, row, kind)
        return [(c, k, j, i, -v if c >= 3 else v, r) for (c, k, j, i, v, r) in inj]
    monkeypatch.setattr(stepping, "source_injection", planted)
    res = oracle.forward(w)
    assert _max_rel(res["E_rec"][..., 0], _solve(w, res["setup"], 0)) > 1e-3


# --------------------------------------------------------------------------
# physics: whole-space magnetic dipole
# --------------------------------------------------------------------------
def _c1_mag_errors(n, h, nt):
    base = c1_wholespace()
    w = c1_wholespace(n=n, h=h, nt=nt).replace(npml=8, rec_pos=base.rec_pos, src_kind=1,
                                               rec_comp=(1, 2, 4, 5))
    res = oracle.forward(w)
    s = res["setup"]
    got = res["E_rec"][0][..., 0]                     # [nr][4]
    E, H = magnetic_dipole_discrete_time(w.rec_pos, [1, 0, 0], 1.0, s.omega[0], s.omega0,
                                         s.Omega[0])
    ref = np.concatenate([E[:, 1:3], H[:, 1:3]], axis=1)
    r = np.linalg.norm(w.rec_pos, axis=1)
    out = {}
    for name, cols in (("E", slice(0, 2)), ("H", slice(2, 4))):
        scale = np.abs(ref[:, cols]).max(1)
        on = scale > 1e-3 * scale.max()              # receivers the field reaches
        err = np.abs(got[:, cols] - ref[:, cols]).max(1)[on] / scale[on]
        out[name] = (err, r[on], np.abs(got[~on][:, cols]).max(initial=0.0) / scale.max())
    return out


@pytest.mark.slow
def test_magnetic_source_wholespace_closed_form_and_convergence():
    """Config c1 (sigma = 1 S/m, 0.25 Hz) with an x-directed magnetic dipole
    at the origin (the centre of eight H_x nodes): E_y, E_z, H_y and H_z
    approach the closed form with second-order accuracy in h; inline
    receivers see no E (r_hat x m = 0) in the oracle either."""
    coarse = _c1_mag_errors(32, 100.0, 600)
    fine = _c1_mag_errors(48, 50.0, 600)
    for name in ("E", "H"):
        e1, r, inline = coarse[name]
        e2, _, _ = fine[name]
        far = r >= 300.0
        if name == "E":
            assert inline < 1e-12
        assert e1[r >= 500.0].max() < 0.1 and e2[r >= 500.0].max() < 0.03
        big = far & (e1 > 0.02)
        assert np.all(e1[big] / e2[big] > 3.0), (name, e1[big], e2[big])


# --------------------------------------------------------------------------
# reciprocity across the source kinds
# --------------------------------------------------------------------------
def test_electric_magnetic_reciprocity():
    """H_b(B) from p_a at A equals E_a(A) from m_b at B, for all nine
    component pairs and every frequency, on a heterogeneous stretched grid
    with CPML: the stepped operator is symmetric under the dual-volume
    pairing, with the E-to-H coupling carried by the kinds' normalisations."""
    w = tiny(seed=6, npml=3, contrast=1.0)
    A = np.array(w.src_pos[0])
    B = np.array(w.rec_pos[2])
    ga = oracle.forward(w.replace(src_pos=np.array([A, A, A]), src_mom=np.eye(3),
                                  rec_pos=np.array([B]), rec_comp=(3, 4, 5)))
    gb = oracle.forward(w.replace(src_pos=np.array([B, B, B]), src_mom=np.eye(3),
                                  rec_pos=np.array([A]), rec_comp=(0, 1, 2), src_kind=1))
    Hab = ga["E_rec"][:, 0]                       # [a][b][nf]: H_b at B from p_a at A
    Eba = np.swapaxes(gb["E_rec"][:, 0], 0, 1)    # E_a at A from m_b at B, as [a][b]
    err = np.abs(Hab - Eba).max() / np.abs(Hab).max()
    assert err < 1e-9, err


# --------------------------------------------------------------------------
# adjoint with magnetic sources
# --------------------------------------------------------------------------
def test_magnetic_source_basis_gradient_equals_time_domain_gradient():
    """With magnetic sources the gradient uses the forward E of M; the
    basis-function adjoint and the time-domain adjoint (whose forward replay
    injects M' into H) agree outside the CPML layers, electric and magnetic
    data mixed."""
    w_true = tiny(seed=3, n=(14, 12, 10), npml=3, contrast=1.0, nr=8, nfreq=2,
                  rec_comp=(0, 1, 4)).replace(src_kind=1)
    rng = np.random.default_rng(103)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    fwd = oracle.forward(w0, want_volume=True)
    resid = d - fwd["E_rec"]
    g_b = oracle.adjoint_gradient(w0, fwd, resid)["grad"]
    g_t = td.adjoint_gradient_td(w0, resid)["grad"]
    m = w0.npml
    inner = (slice(m, -m),) * 3
    err = np.linalg.norm((g_t - g_b)[inner]) / np.linalg.norm(g_b[inner])
    assert err < 1e-9, err
