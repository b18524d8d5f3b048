"""Inversion with the GPU gradient (Section 3.5 driver): the library's driver
on the GPU gradient takes the same iterates as the oracle's driver on the
oracle's gradient; a resistive block in a 1 ohm-m background is recovered
from two sources' data, with the basis-function and the time-domain adjoint;
and iteration timing on the marine grid."""
import time

import numpy as np
import pytest
import torch

from paper_2211_16665_amd import inversion as inv
from workloads import c2_marine1d, tiny

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")


def say(msg):
    print(msg, flush=True)


RHO_MAX = 30.0


def _block_problem():
    w = tiny(seed=11, n=(20, 18, 14), npml=3, contrast=0.0, nr=24, nfreq=2, ns=2,
             rec_comp=(0, 1))
    rho = np.ones(w.shape)
    blk = (slice(6, 9), slice(7, 11), slice(8, 12))
    rho[blk] = 10.0
    w_true = w.replace(rho=rho)
    p = fw.Plan.from_workload(w_true, field_dtype="f64")
    p.set_model(rho)
    d = p.forward().cpu().numpy()
    # fix dt, nt and the CPML velocity so that every model the bounds allow
    # (rho <= RHO_MAX) steps the same discrete system: dt from the most
    # resistive one
    w0 = w_true.replace(rho=np.ones(w.shape))
    p0 = fw.Plan.from_workload(w0, field_dtype="f64")
    p0.set_model(np.full(w.shape, RHO_MAX))
    i = p0.info
    w0 = w0.replace(dt=i.dt, nt=i.nt)
    w0.cpml_vref = i.vref
    W = 1.0 / (0.03 * np.abs(d) + 1e-3 * np.abs(d).max())     # uncertainty-model weights
    return w0, d, W, blk


@pytest.mark.parametrize("method", ["basis", "time"])
def test_inversion_recovers_a_block(method):
    w0, d, W, blk = _block_problem()
    say(f"inversion of a 10 ohm-m block, {method} adjoint")
    plan = fw.Plan.from_workload(w0, field_dtype="f64")
    term = inv.gpu_data_term(plan, d, W, method=method, snapshot_every=100)
    active = np.zeros(w0.shape, bool)
    n = w0.npml
    active[n:-n, n:-n, n:-n] = True
    obj = inv.Objective(term, np.zeros(w0.shape), active=active, alpha=(1.0, 1.0, 1.0),
                        beta=1e-3)
    t0 = time.perf_counter()
    res = inv.lbfgs(obj, np.zeros(int(active.sum())), max_iter=6, first_step=0.5,
                    m_min=np.log(0.1), m_max=np.log(RHO_MAX))
    t = time.perf_counter() - t0
    phis = [h["phi_d"] for h in res.history]
    say(f"  phi_d per iteration: {[f'{v:.3g}' for v in phis]}; {res.evaluations} gradient "
        f"evaluations in {t:.1f} s; restarts {res.restarts}")
    tot = [h["phi"] for h in res.history]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(tot, tot[1:]))
    assert phis[-1] < 0.3 * phis[0]
    mb = float(res.m[blk].mean())
    outside = active.copy()
    outside[blk] = False
    say(f"  mean ln rho in the block {mb:.3f} (true {np.log(10):.3f}), elsewhere "
        f"{float(res.m[outside].mean()):.3f}")
    assert mb > 0.1 and mb > float(res.m[outside].mean()) + 0.1


def _oracle_term(w0, d, W, method):
    import oracle

    def term(m):
        wm = w0.replace(rho=np.exp(m))
        wm.cpml_vref = w0.cpml_vref
        if method == "basis":
            f = oracle.forward(wm, want_volume=True)
            g = oracle.adjoint_gradient(wm, f, W ** 2 * (d - f["E_rec"]))["grad"]
        else:
            f = oracle.forward(wm)
            g = oracle.adjoint_gradient_td(wm, W ** 2 * (d - f["E_rec"]))["grad"]
        return oracle.misfit(f["E_rec"], d, W), g
    return term


@pytest.mark.parametrize("method", ["basis", "time"])
def test_inversion_iterates_match_the_oracle(method):
    """Two iterations on a 14x12x10 block problem (FP64 fields): the same
    line-search decisions, objective values to 1e-9 and models to 1e-8."""
    import oracle
    from oracle import inversion as oinv
    from oracle.discretization import make_setup
    w = tiny(seed=11, n=(14, 12, 10), npml=3, contrast=0.0, nr=16, nfreq=2, ns=2,
             rec_comp=(0, 1))
    rho = np.ones(w.shape)
    rho[4:6, 5:8, 5:9] = 10.0
    s = make_setup(w.replace(rho=np.full(w.shape, RHO_MAX)))
    w0 = w.replace(rho=np.ones(w.shape), dt=s.dt, nt=s.nt)
    w0.cpml_vref = s.vref
    wt = w0.replace(rho=rho)
    wt.cpml_vref = s.vref
    d = oracle.forward(wt)["E_rec"]
    W = 1.0 / (0.03 * np.abs(d) + 1e-3 * np.abs(d).max())
    active = np.zeros(w.shape, bool)
    active[3:-3, 3:-3, 3:-3] = True
    n = int(active.sum())
    kw = dict(max_iter=2, first_step=0.5, m_min=np.log(0.1), m_max=np.log(RHO_MAX))
    say(f"inversion parity, {method} adjoint, {n} active cells")
    plan = fw.Plan.from_workload(w0, field_dtype="f64")
    obj = inv.Objective(inv.gpu_data_term(plan, d, W, method=method, snapshot_every=100),
                        np.zeros(w.shape), active=active, alpha=(1.0, 1.0, 1.0), beta=1e-3)
    res = inv.lbfgs(obj, np.zeros(n), **kw)
    ref = oinv.invert(_oracle_term(w0, d, W, method), np.zeros(w.shape), active, np.zeros(n),
                      alpha=(1.0, 1.0, 1.0), beta=1e-3, **kw)
    lib_phi = ["%.9g" % h["phi"] for h in res.history]
    ora_phi = ["%.9g" % h["phi"] for h in ref["history"]]
    say(f"  phi: library {lib_phi}, oracle {ora_phi}")
    assert len(res.history) == len(ref["history"]) and res.evaluations == ref["evaluations"]
    for h, o in zip(res.history, ref["history"]):
        assert h["step"] == o["step"] and h["restart"] == o["restart"]
        assert abs(h["phi"] - o["phi"]) <= 1e-9 * o["phi"]
    assert ref["history"][-1]["phi"] < ref["history"][0]["phi"]
    err = np.abs(res.m - ref["m"]).max()
    say(f"  max |m_library - m_oracle| = {err:.2e}")
    assert err < 1e-8


def test_vti_inversion_iterates_match_the_oracle():
    """Two-parameter (ln rho_h, ln rho_v) inversion, two iterations on a
    14x12x10 VTI problem (FP64 fields, basis-function adjoint with the split
    gradient of Section 3.1): the library's driver on the GPU gradient takes
    the oracle driver's steps on the oracle gradient."""
    import oracle
    from oracle import inversion as oinv
    from oracle.discretization import make_setup
    from workloads import with_vti
    w = with_vti(tiny(seed=13, n=(14, 12, 10), npml=3, contrast=0.0, nr=16, nfreq=2, ns=2,
                      rec_comp=(0, 1)), ratio=1.0, seed=13, rho_min=0.0)
    rho_h = np.ones(w.shape)
    rho_v = np.ones(w.shape)
    rho_v[4:6, 5:8, 5:9] = 8.0                      # a vertically resistive block
    s = make_setup(w.replace(rho=np.full(w.shape, RHO_MAX), rho_v=np.full(w.shape, RHO_MAX)))
    w0 = w.replace(rho=np.ones(w.shape), rho_v=np.ones(w.shape), dt=s.dt, nt=s.nt)
    w0.cpml_vref = s.vref
    wt = w0.replace(rho=rho_h, rho_v=rho_v)
    wt.cpml_vref = s.vref
    d = oracle.forward(wt)["E_rec"]
    W = 1.0 / (0.03 * np.abs(d) + 1e-3 * np.abs(d).max())
    shape = (2,) + w.shape
    active = np.zeros(shape, bool)
    active[:, 3:-3, 3:-3, 3:-3] = True
    n = int(active.sum())

    def oracle_term(m):
        wm = w0.replace(rho=np.exp(m[0]), rho_v=np.exp(m[1]))
        wm.cpml_vref = w0.cpml_vref
        f = oracle.forward(wm, want_volume=True)
        g = oracle.adjoint_gradient(wm, f, W ** 2 * (d - f["E_rec"]))
        return oracle.misfit(f["E_rec"], d, W), np.stack([g["grad_h"], g["grad_v"]])
    kw = dict(max_iter=2, first_step=0.5, m_min=np.log(0.1), m_max=np.log(RHO_MAX))
    say(f"VTI inversion parity, {n} active parameters")
    plan = fw.Plan.from_workload(w0, field_dtype="f64")
    obj = inv.Objective(inv.gpu_data_term(plan, d, W), np.zeros(shape), active=active,
                        alpha=(1.0, 1.0, 1.0), beta=1e-3)
    res = inv.lbfgs(obj, np.zeros(n), **kw)
    ref = oinv.invert(oracle_term, np.zeros(shape), active, np.zeros(n), alpha=(1.0, 1.0, 1.0),
                      beta=1e-3, **kw)
    lib_phi = ["%.9g" % h["phi"] for h in res.history]
    ora_phi = ["%.9g" % h["phi"] for h in ref["history"]]
    say(f"  phi: library {lib_phi}, oracle {ora_phi}")
    assert len(res.history) == len(ref["history"]) and res.evaluations == ref["evaluations"]
    for h, o in zip(res.history, ref["history"]):
        assert h["step"] == o["step"] and h["restart"] == o["restart"]
        assert abs(h["phi"] - o["phi"]) <= 1e-9 * o["phi"]
    assert ref["history"][-1]["phi"] < ref["history"][0]["phi"]
    err = np.abs(res.m - ref["m"]).max()
    say(f"  max |m_library - m_oracle| = {err:.2e}")
    assert err < 1e-8


def test_inversion_iteration_time_on_the_marine_grid():
    """Two l-BFGS iterations on the marine workload (FP32 fields): the
    starting model without the reservoir; time per gradient evaluation."""
    w = c2_marine1d()
    p = fw.Plan.from_workload(w, field_dtype="f32")
    p.set_model(w.rho)
    d = p.forward().cpu().numpy()
    rho0 = w.rho.copy()
    rho0[rho0 == 100.0] = 1.0
    W = 1.0 / (0.03 * np.abs(d) + 1e-6 * np.abs(d).max())    # 3 % and a low noise floor
    # inline E_y vanishes by symmetry (x-dipole over a 1D model, receivers on
    # the tow line): its weights would only amplify rounding; use E_x alone
    W[:, :, 1, :] = 0.0
    zc = 0.5 * (w.z[:-1] + w.z[1:])
    active = np.broadcast_to((zc > 300.0)[:, None, None], w.shape).copy()   # below the sea floor
    n = w.npml
    active[:n] = active[-n:] = False
    active[:, :n] = active[:, -n:] = False
    active[:, :, :n] = active[:, :, -n:] = False
    obj = inv.Objective(inv.gpu_data_term(p, d, W), np.log(rho0), active=active,
                        alpha=(1.0, 1.0, 0.1), beta=1e-2)
    D = inv.depth_preconditioner(w.z, w.shape, depth0=500.0, z_top=300.0)[active]
    t0 = time.perf_counter()
    res = inv.lbfgs(obj, np.log(rho0)[active], max_iter=2, first_step=0.3, cooling=0.8,
                    precond=D)
    t = time.perf_counter() - t0
    phis = [h["phi_d"] for h in res.history]
    say(f"marine inversion: phi_d {[f'{v:.4g}' for v in phis]}, {res.evaluations} gradient "
        f"evaluations, {t / res.evaluations:.2f} s each")
    assert phis[-1] < phis[0]
