"""The reciprocity swap (Section 4, marine example) on the CPU oracle: the
swapped runs reproduce the data of the original survey, and the gradient of
the swapped formulation (transposed residual into the swapped adjoint) is
the gradient of the original misfit.  The index maps are also checked as an
adjoint pair."""
import numpy as np
import pytest

import oracle
from oracle.discretization import make_setup
from paper_2211_16665_amd.reciprocity import (data_from_swaps, fields_to_data,
                                              residual_to_swapped, swap_workload,
                                              swap_workloads)
from workloads import tiny


def _survey(seed=3):
    w = tiny(seed=seed, n=(14, 12, 10), npml=3, ns=3, nr=2, nfreq=2, rec_comp=(0, 2),
             moment_dirs=True)
    s0 = make_setup(w)
    w = w.replace(dt=s0.dt, nt=s0.nt)
    w.cpml_vref = s0.vref
    return w


def _swapped(w):
    ws = swap_workload(w)
    ws.cpml_vref = w.cpml_vref
    return ws


def test_swapped_runs_reproduce_the_data():
    """3 sources with random moments, 2 receivers with E_x and E_z: 4 swapped
    runs give the 3 x 2 x 2 data to 1e-9 (discrete reciprocity)."""
    w = _survey()
    d = oracle.forward(w)["E_rec"]
    ws = _swapped(w)
    assert len(ws.src_pos) == 4 and len(ws.rec_pos) == 3
    Esw = oracle.forward(ws)["E_rec"]
    got = fields_to_data(Esw, w.src_mom, len(w.rec_comp))
    assert np.abs(got - d).max() < 1e-9 * np.abs(d).max()


def test_maps_are_an_adjoint_pair():
    rng = np.random.default_rng(1)
    p = rng.standard_normal((3, 3))
    E = rng.standard_normal((4, 3, 3, 2)) + 1j * rng.standard_normal((4, 3, 3, 2))
    R = rng.standard_normal((3, 2, 2, 2)) + 1j * rng.standard_normal((3, 2, 2, 2))
    lhs = np.vdot(R, fields_to_data(E, p, 2))
    rhs = np.vdot(residual_to_swapped(R, p, 2), E)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_swapped_gradient_is_the_gradient():
    """The basis-function gradient of the swapped formulation equals that of
    the original survey (same misfit as a function of the model) to the
    accuracy of the basis fit."""
    w_true = _survey(seed=5)
    rng = np.random.default_rng(7)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    w0.cpml_vref = w_true.cpml_vref
    d = oracle.forward(w_true)["E_rec"]
    fwd = oracle.forward(w0, want_volume=True)
    g = oracle.adjoint_gradient(w0, fwd, d - fwd["E_rec"])["grad"]
    ws = _swapped(w0)
    fsw = oracle.forward(ws, want_volume=True)
    dsw = fields_to_data(fsw["E_rec"], w0.src_mom, len(w0.rec_comp))
    rsw = residual_to_swapped(d - dsw, w0.src_mom, len(w0.rec_comp))
    gs = oracle.adjoint_gradient(ws, fsw, rsw)["grad"]
    err = np.linalg.norm(gs - g) / np.linalg.norm(g)
    assert err < 1e-6, err


def test_mixed_components_need_the_list_form():
    with pytest.raises(ValueError):
        swap_workload(tiny(seed=0, rec_comp=(0, 3)))


@pytest.mark.parametrize("src_kind", [0, 1])
def test_swapped_runs_reproduce_magnetic_and_mixed_data(src_kind):
    """E and H receiver components (E_x, H_y, H_z) of electric or magnetic
    sources: the swapped runs (electric unit dipoles for E_x, magnetic ones
    for H_y and H_z; E recorded at electric sources, H at magnetic ones)
    give the data to 1e-9 (Lorentz reciprocity of eq. freq on the stepped
    system)."""
    w = tiny(seed=3, n=(14, 12, 10), npml=3, ns=3, nr=2, nfreq=2, rec_comp=(0, 4, 5),
             moment_dirs=True).replace(src_kind=src_kind)
    s0 = make_setup(w)
    w = w.replace(dt=s0.dt, nt=s0.nt)
    w.cpml_vref = s0.vref
    d = oracle.forward(w)["E_rec"]
    parts = []
    for ws, cis in swap_workloads(w):
        ws.cpml_vref = w.cpml_vref
        assert ws.src_kind == (1 if w.rec_comp[cis[0]] >= 3 else 0)
        parts.append((oracle.forward(ws)["E_rec"], cis))
    assert [cis for _, cis in parts] == [[0], [1, 2]]
    got = data_from_swaps(parts, w.src_mom, len(w.rec_comp))
    assert np.abs(got - d).max() < 1e-9 * np.abs(d).max()
