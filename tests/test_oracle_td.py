"""Pins of the oracle's time-domain adjoint (the Appendix formulation).

The transposed step is checked against the forward step by the
dot-product test <L x, y> = <x, L^T y> over several steps of random states
(with and without CPML, and with a planted mistake that it must catch); the
per-step forward restated next to it is checked against the oracle's
stepping; the gradient is checked against central finite differences of the
misfit and against the frequency-domain (basis-function) gradient of
Section 3, which reaches the same derivative by another route.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint_td as td
from oracle.discretization import make_setup
from oracle.stepping import receiver_nodes, run_stepping, source_injection
from tests.test_oracle import _tiny_inverse_problem
from workloads import tiny


def test_per_step_forward_reproduces_the_stepping():
    w = tiny(seed=1, npml=3, ns=1, moment_dirs=True, contrast=1.5)
    s = make_setup(w)
    nt = 80
    inj = source_injection(s, w.src_pos[0], w.src_mom[0])
    nodes, _ = receiver_nodes(s, np.asarray(w.rec_pos), w.rec_comp)
    acc, _ = run_stepping(s, inj, s.wavelet[None, :], nodes, False, nt)
    E = td.forward_states(s, inj, s.wavelet[None, :], nt)
    zE = np.exp(1j * np.outer((np.arange(nt) + 1.0) * s.dt, s.wprime))
    acc2 = np.array([sum(E[n + 1][c][k, j, i] * zE[n] for n in range(nt))
                     for (c, k, j, i) in nodes])
    assert np.abs(acc2 - acc).max() <= 1e-13 * np.abs(acc).max()


def _dot_test(w, nsteps=6, seed=0):
    s = make_setup(w)
    o = td.ops(s)
    rng = np.random.default_rng(seed)
    x = {k: rng.standard_normal(sh) for k, sh in o.shapes.items()}
    y = {k: rng.standard_normal(sh) for k, sh in o.shapes.items()}
    Lx = {k: v.copy() for k, v in x.items()}
    Ly = {k: v.copy() for k, v in y.items()}
    for _ in range(nsteps):
        td.fwd_step(o, Lx)
        td.adj_step(o, Ly)
    lhs = sum(float(np.sum(Lx[k] * y[k])) for k in x)
    rhs = sum(float(np.sum(x[k] * Ly[k])) for k in x)
    scale = sum(float(np.sum(np.abs(Lx[k] * y[k]))) for k in x)
    return abs(lhs - rhs) / scale


@pytest.mark.parametrize("npml", [0, 3])
def test_transposed_step_passes_dot_product_test(npml):
    """<L x, y> = <x, L^T y> for six steps of random states (fields and
    every CPML memory variable), stretched heterogeneous grid."""
    w = tiny(seed=2, npml=npml, contrast=1.5, stretch=1.3)
    assert _dot_test(w) < 1e-13


def test_dot_product_test_catches_a_dropped_memory_term(monkeypatch):
    """Plant: the transposed CPML recursion forgets the a (ad + apsi) term
    of the derivative's adjoint; the dot-product test must fail."""
    w = tiny(seed=2, npml=3, contrast=1.5, stretch=1.3)
    orig = td.adj_step

    def wrong(o, ad):
        saved = {ax: v for ax, v in o.cp_half.items()}
        o.cp_half = {ax: (k, b, 0.0 * a) for ax, (k, b, a) in saved.items()}
        try:
            orig(o, ad)
        finally:
            o.cp_half = saved
    monkeypatch.setattr(td, "adj_step", wrong)
    assert _dot_test(w) > 1e-6


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
def test_td_gradient_matches_finite_differences():
    """The time-domain adjoint gradient is the exact derivative of the stepped
    misfit: central differences agree to 1e-5 on interior cells (h = 1e-3 in
    ln rho) and to 1e-4 on cells inside the CPML layers (h = 1e-2; the
    gradient there is ~1e-3 of the largest)."""
    w0, d = _tiny_inverse_problem()
    resid = d - oracle.forward(w0)["E_rec"]
    g = td.adjoint_gradient_td(w0, resid)["grad"]
    for c in [(4, 5, 6), (5, 5, 5), (6, 4, 8), (5, 7, 6)]:
        fd = _fd(w0, d, c, 1e-3)
        assert abs(fd - g[c]) / abs(fd) < 1e-5, (c, fd, g[c])
    for c in [(5, 7, 2), (7, 9, 3)]:                      # x index < npml = 3
        fd = _fd(w0, d, c, 1e-2)
        assert abs(fd - g[c]) / abs(fd) < 1e-4, (c, fd, g[c])


def test_td_gradient_matches_the_frequency_domain_gradient():
    """Two routes to the same derivative: the basis-function adjoint of
    Section 3 (eq. gradsigmaij with the discrete-time factor) and the
    time-domain adjoint of the Appendix agree on every cell outside the CPML
    layers.  Inside the layers eq. gradsigmaij (with the plain dual volume of
    the edge) is not the derivative of the stretched system; the time-domain
    gradient is, as the finite-difference test above shows."""
    w0, d = _tiny_inverse_problem()
    fwd = oracle.forward(w0, want_volume=True)
    resid = d - fwd["E_rec"]
    g_fd = oracle.adjoint_gradient(w0, fwd, resid)["grad"]
    g_td = td.adjoint_gradient_td(w0, resid)["grad"]
    m = w0.npml
    inner = (slice(m, -m),) * 3
    err = np.linalg.norm((g_td - g_fd)[inner]) / np.linalg.norm(g_fd[inner])
    assert err < 1e-9, err
