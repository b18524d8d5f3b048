"""Pins of the oracle's decimated volume transform (an option of this
implementation, not of the paper: the volume transform of eq. dft takes only
the samples E^m with m a multiple of D, each weighted by D, a coarser
Riemann sum of the integral of eq. dtft; receivers keep every sample).

  * D = 1 is the exact transform: the normalised volume equals E of the
    sparse solve of the frequency-domain identity on every edge (1e-9);
  * D > 1 is the stated sum: against D sum_{m = D, 2D, ...} E^m z^m formed
    from the state history of the time-domain adjoint's own step;
  * the error against D = 1 stays small while D dt is well inside the
    wavelet's width and grows by orders of magnitude once D dt nears it
    (aliasing), for the volume and for the gradient (decimated forward
    volume, exact adjoint transform);
  * planted mistakes (no weight D, samples at m = 1 mod D) break the pins.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint_td as td
from oracle import stepping
from oracle.discretization import make_setup
from tests.pins.fdsolve import solve as fd_solve
from workloads import tiny


def _w(seed=3, **kw):
    return tiny(seed=seed, n=(14, 12, 10), npml=3, contrast=1.0, nr=8, nfreq=2, ns=1, **kw)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_undecimated_volume_equals_sparse_solve():
    w = _w(moment_dirs=True)
    res = oracle.forward(w, want_volume=True, decimate=1)
    s = res["setup"]
    for kf, f in enumerate(w.freqs):
        _, fields = fd_solve(w.x, w.y, w.z, w.rho, w.npml, w.f0, f, s.dt,
                             list(zip(w.src_pos, w.src_mom)), w.rec_pos, w.rec_comp,
                             s.vref, alpha_max=0.5 * s.a.min(), full=True)
        for c in range(3):
            assert _rel(res["vol"][0][c][kf], fields[0][c]) < 1e-9, (f, c)


def _history_sum(w, D):
    s = make_setup(w)
    inj = stepping.source_injection(s, w.src_pos[0], w.src_mom[0])
    states = td.forward_states(s, inj, s.wavelet[None, :], s.nt)      # E^0 .. E^nt
    norm, _ = stepping.source_norms(s, s.nt)
    out = []
    for c in range(3):
        acc = np.zeros((len(s.freqs),) + states[0][c].shape, dtype=np.complex128)
        for m in range(D, s.nt + 1, D):
            z = np.exp(1j * s.wprime * m * s.dt)
            acc += D * z[:, None, None, None] * states[m][c][None]
        out.append(acc * norm[:, None, None, None])
    return out


@pytest.mark.parametrize("D", [3, 8])
def test_decimated_volume_is_the_stated_sum(D):
    w = _w()
    res = oracle.forward(w, want_volume=True, decimate=D)
    ref = _history_sum(w, D)
    for c in range(3):
        assert _rel(res["vol"][0][c], ref[c]) < 1e-12


def test_plant_sample_offset(monkeypatch):
    """Plant: samples m = 1 (mod D) instead of m = 0 (mod D)."""
    w = _w()
    D = 8
    orig = stepping.run_stepping

    def planted(s, inj, tfun, rec_nodes, want_volume, nt=None, decimate=1):
        if decimate == 1:
            return orig(s, inj, tfun, rec_nodes, want_volume, nt, 1)
        # every sample recorded, then those at m = 1 mod D kept
        nt_ = s.nt if nt is None else nt
        acc, _ = orig(s, inj, tfun, rec_nodes, False, nt_, 1)
        st = td.forward_states(s, inj, tfun, nt_)
        vol = []
        for c in range(3):
            v = np.zeros((len(s.freqs),) + st[0][c].shape, dtype=np.complex128)
            for m in range(1, nt_ + 1, decimate):
                v += decimate * np.exp(1j * s.wprime * m * s.dt)[:, None, None, None] * st[m][c][None]
            vol.append(v)
        return acc, vol
    monkeypatch.setattr(stepping, "run_stepping", planted)
    res = oracle.forward(w, want_volume=True, decimate=D)
    ref = _history_sum(w, D)
    # another valid Riemann sum, so the shift is of the size of the decimation
    # error, far above the 1e-12 of the stated-sum pin
    assert max(_rel(res["vol"][0][c], ref[c]) for c in range(3)) > 1e-8


def _vol_error(w, D, ref):
    r = oracle.forward(w, want_volume=True, decimate=D)
    return max(_rel(r["vol"][0][c], ref["vol"][0][c]) for c in range(3))


def test_decimation_error_against_wavelet_width():
    """On this grid the wavelet is about 11 steps wide (tau / dt).  Up to
    D = 8 the volume stays within 1e-5 of the exact transform; at D = 32 the
    samples no longer resolve the wavelet and the error is O(0.1)."""
    w = _w()
    s = make_setup(w)
    assert 10 < s.tau / s.dt < 12
    ref = oracle.forward(w, want_volume=True)
    errs = {D: _vol_error(w, D, ref) for D in (2, 8, 32)}
    assert errs[2] < 1e-6 and errs[8] < 1e-5 and errs[32] > 1e-2, errs
    assert errs[2] < errs[8] < errs[32]


def test_plant_missing_weight(monkeypatch):
    """Plant: decimated samples not weighted by D (the sum falls by D)."""
    w = _w()
    orig = stepping.run_stepping

    def planted(s, inj, tfun, rec_nodes, want_volume, nt=None, decimate=1):
        acc, vol = orig(s, inj, tfun, rec_nodes, want_volume, nt, decimate)
        return acc, (None if vol is None else [v / decimate for v in vol])
    ref = oracle.forward(w, want_volume=True)
    monkeypatch.setattr(stepping, "run_stepping", planted)
    assert _vol_error(w, 4, ref) > 0.5


def test_decimated_gradient_error():
    """The gradient from a decimated forward volume transform against the
    exact one (same basis functions, same residual, exact adjoint
    transform): 1e-5 up to D = 8 on this grid, O(0.1) at D = 32."""
    w_true = _w(seed=5)
    rng = np.random.default_rng(105)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    g = {}
    for D in (1, 8, 32):
        fwd = oracle.forward(w0, want_volume=True, decimate=D)
        g[D] = oracle.adjoint_gradient(w0, fwd, d - fwd["E_rec"])["grad"]
    e8 = np.linalg.norm(g[8] - g[1]) / np.linalg.norm(g[1])
    e32 = np.linalg.norm(g[32] - g[1]) / np.linalg.norm(g[1])
    assert e8 < 1e-5 and e32 > 1e-2, (e8, e32)
