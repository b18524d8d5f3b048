"""Pins of the oracle's VTI (vertically transverse isotropic) modelling and
gradient (Section 2: sigma_h = sigma_xx = sigma_yy, sigma_v = sigma_zz;
Section 3.1: the VTI gradient, x and y edges for sigma_h, z edges for
sigma_v).

The anisotropic stepped system is pinned by the independent sparse direct
solve of its frequency-domain identity (tests/pins/fdsolve.py, z-edge
permittivities from the vertical conductivity); the isotropic case is
recovered exactly when rho_v = rho; both gradients (basis-function and
time-domain adjoint) match central differences with respect to ln rho_h
and ln rho_v separately.
"""
import numpy as np
import pytest

import oracle
from oracle.adjoint_td import adjoint_gradient_td
from oracle.discretization import make_setup
from tests.pins.fdsolve import solve as fd_solve
from workloads import tiny, with_vti


def test_vti_with_equal_resistivities_is_the_isotropic_run():
    w = tiny(seed=3, npml=3, ns=1, contrast=1.0)
    a = oracle.forward(w)["E_rec"]
    b = oracle.forward(w.replace(rho_v=w.rho.copy()))["E_rec"]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("seed,npml", [(0, 3), (2, 0)])
def test_vti_stepping_equals_sparse_solve(seed, npml):
    w = with_vti(tiny(seed=seed, npml=npml, contrast=1.0, ns=2, moment_dirs=True,
                      rec_comp=(0, 1, 2)), ratio=4.0, seed=seed, rho_min=0.0)
    res = oracle.forward(w)
    iso = oracle.forward(w.replace(rho_v=None))["E_rec"]
    s = res["setup"]
    # the anisotropy matters at the receivers
    assert np.abs(res["E_rec"] - iso).max() > 1e-2 * np.abs(iso).max()
    for kf, f in enumerate(w.freqs):
        ref = fd_solve(w.x, w.y, w.z, w.rho, w.npml, w.f0, f, s.dt,
                       list(zip(w.src_pos, w.src_mom)), w.rec_pos, w.rec_comp,
                       s.vref, alpha_max=0.5 * s.a.min(), rho_v=w.rho_v)
        err = np.abs(res["E_rec"][..., kf] - ref).max() / np.abs(ref).max()
        assert err < 1e-9, (f, err)


def _vti_inverse_problem(seed=3):
    w_true = with_vti(tiny(seed=seed, n=(14, 12, 10), npml=3, contrast=1.0, nr=8, nfreq=2),
                      ratio=3.0, seed=seed, rho_min=0.0)
    rng = np.random.default_rng(seed + 200)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)),
                        rho_v=w_true.rho_v * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    return w0, d


def _fd(w0, d, which, c, h=1e-3):
    vals = []
    for sgn in (1, -1):
        kw = {}
        arr = (w0.rho if which == "h" else w0.rho_v).copy()
        arr[c] *= np.exp(sgn * h)
        kw["rho" if which == "h" else "rho_v"] = arr
        wp = w0.replace(**kw)
        wp.cpml_vref = w0.cpml_vref
        vals.append(oracle.misfit(oracle.forward(wp)["E_rec"], d))
    return (vals[0] - vals[1]) / (2 * h)


@pytest.mark.slow
def test_vti_gradients_match_finite_differences():
    """d phi / d ln rho_h and d phi / d ln rho_v from the basis-function
    adjoint (Section 3.1 VTI expression) and from the time-domain adjoint
    agree with central differences on interior cells."""
    w0, d = _vti_inverse_problem()
    fwd = oracle.forward(w0, want_volume=True)
    resid = d - fwd["E_rec"]
    gb = oracle.adjoint_gradient(w0, fwd, resid)
    gt = adjoint_gradient_td(w0, resid)
    for c in [(4, 5, 6), (5, 6, 7), (6, 4, 8)]:
        for which in ("h", "v"):
            fd = _fd(w0, d, which, c)
            for g in (gb, gt):
                val = g["grad_" + which][c]
                assert abs(fd - val) < 1e-4 * abs(fd), (c, which, fd, val)
    # the isotropic gradient is the sum of the two
    assert np.array_equal(gb["grad"], gb["grad_h"] + gb["grad_v"])
