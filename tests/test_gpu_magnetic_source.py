"""Parity of magnetic dipole sources on the GPU with the oracle.

A plan of source kind 1 injects M'^n = m w_n into the H update at n dt
(Faraday row of eq. fictitiouswave, M' = M by eq. mittet) and normalises
by W^M_k = sum_n w_n z_k^n.  Bars as for electric sources: FP64 fields to
1e-11 (receivers and volume), basis-function gradient to 1e-7 and
time-domain gradient to 1e-9 (relative L2) against the FP64 oracle; FP32
fields to 1e-4 and 1e-3.  The three schedules, graph replay and batching
agree bit for bit, and the reciprocity swap gives magnetic data from
magnetic unit sources.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.discretization import make_setup
from workloads import tiny

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def mag_tiny(seed, npml=3, ns=2, order=2, rec_comp=(0, 1, 2, 3, 4, 5), **kw):
    return tiny(seed=seed, npml=npml, ns=ns, moment_dirs=True, contrast=1.5,
                rec_comp=rec_comp, **kw).replace(fd_order=order, src_kind=1)


@pytest.mark.parametrize("seed,npml,order,dtype,tol", [(0, 3, 2, "f64", 1e-11),
                                                       (1, 0, 2, "f64", 1e-11),
                                                       (2, 3, 4, "f64", 1e-11),
                                                       (2, 3, 2, "f32", 1e-4)])
def test_magnetic_source_receivers_and_volume_match_oracle(seed, npml, order, dtype, tol):
    w = mag_tiny(seed, npml, order=order)
    say(f"magnetic sources seed={seed} npml={npml} order={order} {dtype}")
    ref = oracle.forward(w, want_volume=True)
    p = fw.Plan.from_workload(w, field_dtype=dtype, acc_mode="f64")
    p.set_model(w.rho)
    E, vol = p.forward(want_volume=True)
    E = E.cpu().numpy()
    for ci, c in enumerate(w.rec_comp):
        err = rel(E[:, :, ci], ref["E_rec"][:, :, ci])
        say(f"  component {c}: {err:.2e}")
        assert err < tol, (c, err)
    V = p.volume_export(vol).cpu().numpy()            # [ns][nf][3][NZ][NY][PX]
    for s in range(w.ns):
        for c in range(3):
            r = ref["vol"][s][c]                          # [nf, ...] normalised
            nz, ny, nx = r.shape[1:]
            got = V[s, :, c, :nz, :ny, :nx]
            err = rel(got, r)
            assert err < tol, (s, c, err)


def test_magnetic_source_schedules_tilings_and_replay_bitwise():
    """Two-kernel, fused and persistent schedules, eager launches, another
    tiling and vector widths: the same bits for receivers, volume and
    gradient."""
    w0 = mag_tiny(3, ns=2, rec_comp=(0, 3, 5))
    d = oracle.forward(w0)["E_rec"] * 1.01
    out = []
    for opts in (dict(), dict(schedule=1, zchunk=4), dict(schedule=2, block_x=64, block_y=4),
                 dict(graph_steps=0), dict(block_x=16, block_y=16, tile_order=1, xcd_remap=0),
                 dict(vector=4, vector_h=4)):
        say(f"magnetic sources, options {opts}")
        p = fw.Plan.from_workload(w0, field_dtype="f32", acc_mode="kahan")
        for key, v in opts.items():
            p.set_option(getattr(fw, "FWD_OPT_" + key.upper()), v)
        p.set_model(w0.rho)
        p.basis_build(gamma_rel=1e-12)
        E, vol = p.forward(want_volume=True)
        g = p.adjoint(vol, torch.from_numpy(d).cuda() - E)
        out.append((E.cpu().numpy(), vol.cpu().numpy(), g.cpu().numpy()))
    for o in out[1:]:
        for a, b in zip(o, out[0]):
            assert np.array_equal(a, b)


def test_magnetic_source_batch_equals_single_sources():
    w = mag_tiny(5, ns=3, rec_comp=(1, 2, 3))
    say("magnetic sources: batch against single-source plans")
    p = fw.Plan.from_workload(w, field_dtype="f32", acc_mode="f64")
    p.set_model(w.rho)
    Eb = p.forward().cpu().numpy()
    for s in range(w.ns):
        q = fw.Plan.from_workload(w.replace(src_pos=w.src_pos[s:s + 1], src_mom=w.src_mom[s:s + 1]),
                                  field_dtype="f32", acc_mode="f64")
        q.set_model(w.rho)
        assert np.array_equal(q.forward().cpu().numpy()[0], Eb[s])


def _problem(rec_comp, seed=3, order=2):
    w_true = tiny(seed=seed, n=(14, 12, 10), npml=3, contrast=1.0, nr=8, nfreq=2, ns=2,
                  rec_comp=rec_comp, moment_dirs=True).replace(fd_order=order, src_kind=1)
    rng = np.random.default_rng(seed + 100)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    return w0, d


@pytest.mark.parametrize("rec_comp,order,dtype,tol", [((0, 1, 2), 2, "f64", 1e-7),
                                                      ((0, 4, 5), 2, "f64", 1e-7),
                                                      ((0, 4, 5), 4, "f64", 1e-7),
                                                      ((0, 1, 4), 2, "f32", 1e-3)])
def test_magnetic_source_gradient_matches_oracle(rec_comp, order, dtype, tol):
    w0, d = _problem(rec_comp, order=order)
    say(f"magnetic-source gradient, components {rec_comp}, order {order}, {dtype}")
    fwd = oracle.forward(w0, want_volume=True)
    resid = d - fwd["E_rec"]
    go = oracle.adjoint_gradient(w0, fwd, resid)["grad"]
    p = fw.Plan.from_workload(w0, field_dtype=dtype)
    p.set_model(w0.rho)
    p.basis_build(gamma_rel=1e-12)
    E, vol = p.forward(want_volume=True)
    assert rel(E.cpu().numpy(), fwd["E_rec"]) < (1e-11 if dtype == "f64" else 1e-4)
    g = p.adjoint(vol, torch.from_numpy(d).cuda() - E).cpu().numpy()
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    say(f"  relative L2 {err:.2e}")
    assert err < tol, err


@pytest.mark.parametrize("rec_comp,order,dtype,tol", [((0, 4, 5), 2, "f64", 1e-9),
                                                      ((0, 1, 2), 4, "f64", 1e-9),
                                                      ((0, 4, 5), 2, "f32", 1e-3)])
def test_magnetic_source_td_gradient_matches_oracle(rec_comp, order, dtype, tol):
    """The time-domain adjoint, whose forward replay injects M' into H,
    against the oracle's time-domain adjoint."""
    from oracle.adjoint_td import adjoint_gradient_td
    w0, d = _problem(rec_comp, order=order)
    say(f"magnetic-source time-domain gradient, components {rec_comp}, order {order}, {dtype}")
    resid = d - oracle.forward(w0)["E_rec"]
    go = adjoint_gradient_td(w0, resid)["grad"]
    p = fw.Plan.from_workload(w0, field_dtype=dtype)
    p.set_model(w0.rho)
    g = p.adjoint_td(torch.from_numpy(resid).cuda(), segment=37).cpu().numpy()
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    say(f"  relative L2 {err:.2e}")
    assert err < tol, err


def test_reciprocity_swap_with_magnetic_data_on_the_gpu():
    """Electric sources with E_x, H_y, H_z receivers: the swapped runs (an
    electric plan for E_x, a magnetic plan for H_y and H_z) give the data of
    the original survey (FP64, 1e-9)."""
    from paper_2211_16665_amd.reciprocity import data_from_swaps, swap_workloads
    w = tiny(seed=3, n=(14, 12, 10), npml=3, ns=3, nr=2, nfreq=2, rec_comp=(0, 4, 5),
             moment_dirs=True)
    s0 = make_setup(w)
    w = w.replace(dt=s0.dt, nt=s0.nt)
    w.cpml_vref = s0.vref
    say("reciprocity swap with magnetic data: 3 sources x 2 receivers (E_x, H_y, H_z)")
    p = fw.Plan.from_workload(w, field_dtype="f64")
    p.set_model(w.rho)
    d = p.forward().cpu().numpy()
    parts = []
    for ws, cis in swap_workloads(w):
        ws.cpml_vref = w.cpml_vref
        q = fw.Plan.from_workload(ws, field_dtype="f64")
        q.set_model(w.rho)
        parts.append((q.forward().cpu().numpy(), cis))
    got = data_from_swaps(parts, w.src_mom, len(w.rec_comp))
    err = rel(got, d)
    say(f"  data {err:.2e}")
    assert err < 1e-9
