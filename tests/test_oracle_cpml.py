"""Pin of the oracle's CPML (the absorbing layers of Section 2, K&M form) by
what it must do rather than by its formula: absorb.

A y-dipole in a uniform 1 S/m whole space, receivers on the +x axis up to 7
cells from the source and 7 from the layers' inner boundary (6-cell layers,
walls 6 cells further out).  Over a window of 140 steps the field travels
about 77 cells, so the walls' echo returns within the window.  The same run
on a grid 40 cells longer on each x side (its walls too far for an echo to
return) is the reference:
  * with the CPML the difference stays below 1e-3 of the field at every
    receiver (observed 2e-6 next to the source, 5e-4 next to the layer);
  * with the layers replaced by plain grid cells (PEC walls at the same
    place) it exceeds 1e-2, and the CPML cuts it by more than 30x at every
    receiver;
  * a planted sign error in the memory term breaks the first bound.
This pins that the layers absorb; the exact coefficients are pinned by the
sparse solve of tests/pins/fdsolve.py (rows assembled from the same K&M
definitions, written again there).  Changes of the damping's strength
(its time constant, the profile's scale) only move the echo within the
bound: they are readings of parameters the paper leaves open.
"""
import numpy as np
import pytest

import oracle
from oracle import discretization as disc
from oracle.discretization import make_setup
from workloads.configs import Workload

H = 100.0


def _axis(ncells):
    return (np.arange(ncells + 1) - ncells / 2) * H


def _workload(pad, npml=6, core=16, dt=None, vref=None):
    x = _axis(core + 2 * npml + 2 * pad)
    y = z = _axis(core + 2 * npml)
    rho = np.ones((len(z) - 1, len(y) - 1, len(x) - 1))
    recs = np.array([(m * H + 0.5 * H, 0.0, 0.0) for m in range(2, 8)])
    w = Workload(name="cpml_pin", x=x, y=y, z=z, rho=rho, freqs=np.array([0.5, 1.5]),
                 src_pos=np.array([[0.5 * H, 0.0, 0.0]]), src_mom=np.array([[0.0, 1.0, 0.0]]),
                 rec_pos=recs, rec_comp=(1,), npml=npml, nt=140, field_dtype="f64",
                 rho_air_cap=1e8)
    if dt is not None:
        w = w.replace(dt=dt)
    if vref is not None:
        w.cpml_vref = vref
    return w


def _echo(npml=6, core=16):
    """Largest |small - big| / |big| over frequencies, per receiver."""
    s = make_setup(_workload(0))
    small = oracle.forward(_workload(0, npml, core, s.dt, s.vref))["E_rec"]
    big = oracle.forward(_workload(40, npml, core, s.dt, s.vref))["E_rec"]
    return (np.abs(small - big) / np.abs(big))[0, :, 0, :].max(axis=1)


def test_cpml_absorbs_what_pec_walls_reflect():
    e_cpml = _echo()
    e_pec = _echo(npml=0, core=28)
    assert e_cpml.max() < 1e-3, e_cpml
    assert e_pec.max() > 1e-2, e_pec
    assert np.all(e_pec / e_cpml > 30.0), e_pec / e_cpml


def _planted(monkeypatch, change):
    orig = disc.cpml_profile

    def planted(nodes, npml, dt, vref, order, R, kappa_max, alpha_max):
        return change(orig, nodes, npml, dt, vref, order, R, kappa_max, alpha_max)
    monkeypatch.setattr(disc, "cpml_profile", planted)


def test_planted_sign_error_reflects(monkeypatch):
    def change(orig, nodes, npml, dt, vref, order, R, kmax, amax):
        out = orig(nodes, npml, dt, vref, order, R, kmax, amax)
        return tuple((k, b, -a) for (k, b, a) in out)
    _planted(monkeypatch, change)
    e = _echo()
    assert not np.all(np.isfinite(e)) or e.max() > 1e-3, e
