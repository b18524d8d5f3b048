"""Parity of magnetic data on the GPU with the oracle.

Receiver components 3-5 (H_x, H_y, H_z): the forward H at the receivers
(H^{n+1/2} transformed with z^{n+1/2}, scaled by 1 / W_k), and the gradient
of a misfit over magnetic data (magnetic residual injected as M' into H at
n dt).  Bars as for electric data: FP64 fields to 1e-11 (fields) and 1e-7
(basis-function gradient) and 1e-9 (time-domain gradient, relative L2)
against the FP64 oracle; FP32 fields to 1e-4 and 1e-3.  The two schedules
and the tilings agree bit for bit.
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


@pytest.mark.parametrize("seed,npml,order,dtype,tol", [(0, 3, 2, "f64", 1e-11),
                                                       (1, 0, 2, "f64", 1e-11),
                                                       (2, 3, 4, "f64", 1e-11),
                                                       (2, 3, 2, "f32", 1e-4)])
def test_h_receivers_match_oracle(seed, npml, order, dtype, tol):
    w = tiny(seed=seed, npml=npml, ns=2, moment_dirs=True, contrast=1.5,
             rec_comp=(0, 3, 4, 5)).replace(fd_order=order)
    say(f"H receivers seed={seed} npml={npml} order={order} {dtype}")
    ref = oracle.forward(w)["E_rec"]
    p = fw.Plan.from_workload(w, field_dtype=dtype, acc_mode="f64")
    p.set_model(w.rho)
    E = p.forward().cpu().numpy()
    for ci, c in enumerate(w.rec_comp):
        err = rel(E[:, :, ci], ref[:, :, ci])
        say(f"  component {c}: {err:.2e}")
        assert err < tol, (c, err)


def test_h_receivers_schedules_and_replay_bitwise():
    """Two-kernel and fused schedules, eager launches and graph replay, and
    two tilings give the same bits for E and H rows."""
    w = tiny(seed=3, npml=3, ns=2, moment_dirs=True, rec_comp=(1, 3, 5))
    out = []
    for opts in (dict(), dict(schedule=1, zchunk=4), dict(graph_steps=0),
                 dict(block_x=16, block_y=16, tile_order=1, xcd_remap=0)):
        say(f"H receivers, options {opts}")
        p = fw.Plan.from_workload(w, field_dtype="f32", acc_mode="f64")
        for key, v in opts.items():
            p.set_option(getattr(fw, "FWD_OPT_" + key.upper()), v)
        p.set_model(w.rho)
        out.append(p.forward().cpu().numpy())
    for o in out[1:]:
        assert np.array_equal(o, out[0])


def _problem(rec_comp, seed=3, order=2):
    w_true = tiny(seed=seed, n=(14, 12, 10), npml=3, contrast=1.0, nr=8, nfreq=2, ns=2,
                  rec_comp=rec_comp).replace(fd_order=order)
    rng = np.random.default_rng(seed + 100)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    return w0, d


@pytest.mark.parametrize("rec_comp,order,dtype,tol", [((3, 4, 5), 2, "f64", 1e-7),
                                                      ((0, 4, 5), 2, "f64", 1e-7),
                                                      ((0, 4, 5), 4, "f64", 1e-7),
                                                      ((3, 4, 5), 2, "f32", 1e-3)])
def test_magnetic_gradient_matches_oracle(rec_comp, order, dtype, tol):
    w0, d = _problem(rec_comp, order=order)
    say(f"gradient with components {rec_comp}, order {order}, {dtype}")
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


def test_magnetic_gradient_schedules_bitwise():
    """The magnetic adjoint source and the gradient give the same bits with
    the fused schedule as with the two-kernel one."""
    w0, d = _problem((0, 3, 5), seed=5)
    out = []
    for sched in (0, 1):
        say(f"magnetic gradient, schedule {sched}")
        p = fw.Plan.from_workload(w0, field_dtype="f32", acc_mode="kahan")
        p.set_option(fw.FWD_OPT_SCHEDULE, sched)
        p.set_model(w0.rho)
        p.basis_build(gamma_rel=1e-12)
        E, vol = p.forward(want_volume=True)
        r = torch.from_numpy(d).cuda() - E
        out.append((E.cpu().numpy(), p.adjoint(vol, r).cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("rec_comp,order,dtype,tol", [((3, 4, 5), 2, "f64", 1e-9),
                                                      ((0, 4, 5), 2, "f64", 1e-9),
                                                      ((0, 4, 5), 4, "f64", 1e-9),
                                                      ((0, 4, 5), 2, "f32", 1e-3)])
def test_magnetic_td_gradient_matches_oracle(rec_comp, order, dtype, tol):
    """The time-domain adjoint with magnetic receivers (d phi / d H^{n+1/2}
    into the H multipliers between the two reverse kernels) against the
    oracle's time-domain adjoint, which is the exact derivative of the
    stepped misfit; FP64 to 1e-9 (relative L2), FP32 fields to 1e-3."""
    from oracle.adjoint_td import adjoint_gradient_td
    w0, d = _problem(rec_comp, order=order)
    say(f"time-domain gradient with components {rec_comp}, order {order}, {dtype}")
    resid = d - oracle.forward(w0)["E_rec"]
    go = adjoint_gradient_td(w0, resid)["grad"]
    p = fw.Plan.from_workload(w0, field_dtype=dtype)
    p.set_model(w0.rho)
    g = p.adjoint_td(torch.from_numpy(resid).cuda(), segment=37).cpu().numpy()
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    say(f"  relative L2 {err:.2e}")
    assert err < tol, err


def test_autograd_magnetic_data_matches_finite_differences():
    """FictitiousForward over magnetic receivers: both adjoints against
    central differences of the GPU misfit (FP64, h = 1e-3, 1e-4 relative:
    at cell (5, 5, 5) the gradient is 200x below the largest and the
    difference quotient, not the adjoint, sets the error; the two adjoints
    agree there to 7 digits)."""
    from paper_2211_16665_amd.autograd import FictitiousForward, misfit
    w0, d = _problem((3, 4, 5), seed=4)
    say("autograd with magnetic data vs finite differences (fp64)")
    p = fw.Plan.from_workload(w0, field_dtype="f64")
    dd = torch.from_numpy(d).cuda()
    grads = {}
    for method, snap in (("basis", 0), ("time", 64)):
        m = torch.tensor(np.log(w0.rho), dtype=torch.float64, device="cuda", requires_grad=True)
        misfit(FictitiousForward.apply(m, p, snap, 1e-12, method), dd).backward()
        grads[method] = m.grad.cpu().numpy()
    for c in [(4, 5, 6), (5, 5, 5)]:
        vals = []
        for sgn in (1, -1):
            mm = np.log(w0.rho).copy()
            mm[c] += sgn * 1e-3
            with torch.no_grad():
                E = FictitiousForward.apply(torch.from_numpy(mm).cuda(), p)
            vals.append(float(misfit(E, dd)))
        fd = (vals[0] - vals[1]) / 2e-3
        gb, gt = grads["basis"][c], grads["time"][c]
        say(f"  cell {c}: fd {fd:.6e} basis {gb:.6e} time {gt:.6e}")
        assert abs(fd - gb) < 1e-4 * abs(fd), (c, fd, gb)
        assert abs(fd - gt) < 1e-4 * abs(fd), (c, fd, gt)
        assert abs(gb - gt) < 1e-6 * abs(gt), (c, gb, gt)


def test_magnetic_adjoint_graph_replay_and_checkpoint_bitwise():
    """With magnetic receivers: the adjoint (magnetic sources in the H
    update) gives the same bits with graph replay as with eager launches,
    and a forward run interrupted, diverged and resumed from a checkpoint
    gives the same H (and E) rows as an uninterrupted one."""
    w0, d = _problem((0, 3, 4), seed=6)
    grads = []
    for graph_steps in (32, 0):
        say(f"magnetic adjoint, graph steps {graph_steps}")
        p = fw.Plan.from_workload(w0, field_dtype="f32", acc_mode="f64")
        p.set_option(fw.FWD_OPT_GRAPH_STEPS, graph_steps)
        p.set_model(w0.rho)
        p.basis_build(gamma_rel=1e-12)
        E, vol = p.forward(want_volume=True)
        grads.append(p.adjoint(vol, torch.from_numpy(d).cuda() - E).cpu().numpy())
    assert np.array_equal(grads[0], grads[1])
    say("magnetic receivers, checkpoint resume")
    p = fw.Plan.from_workload(w0, field_dtype="f32", acc_mode="f64")
    p.set_model(w0.rho)
    nt = p.info.nt
    E_full = p.forward().cpu().numpy()
    p.run_begin()
    k = nt // 3
    p.run_steps(k)
    snap = torch.empty(p.checkpoint_size(False), dtype=torch.uint8, device="cuda")
    p.checkpoint_save(snap)
    p.run_steps(nt // 2)                       # diverge
    p.checkpoint_restore(snap)
    p.run_steps(nt - k)
    assert np.array_equal(p.run_receivers().cpu().numpy(), E_full)

