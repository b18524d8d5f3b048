"""Parity of the fourth-order HIP path with the oracle (FWD_OPT_FD_ORDER = 4).

Same bars as the second-order path: FP64 fields agree with the FP64 oracle
to rounding (1e-11 of the largest value for fields, 1e-7 / 1e-9 relative L2
for the basis-function / time-domain gradient); FP32 fields to 1e-4 (fields)
and 1e-3 (gradients).  Tilings are compared bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.adjoint_td import adjoint_gradient_td
from oracle.discretization import make_setup
from workloads import c1_wholespace, tiny, with_vti

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("seed,npml,ns,dtype,tol", [(0, 3, 1, "f64", 1e-11),
                                                    (1, 0, 1, "f64", 1e-11),
                                                    (2, 3, 3, "f64", 1e-11),
                                                    (2, 3, 3, "f32", 1e-4)])
def test_order4_forward_matches_oracle(seed, npml, ns, dtype, tol):
    w = tiny(seed=seed, npml=npml, ns=ns, moment_dirs=True, contrast=1.5).replace(fd_order=4)
    say(f"order-4 forward seed={seed} npml={npml} ns={ns} {dtype} shape={w.shape}")
    ref = oracle.forward(w, want_volume=True)
    p = fw.Plan.from_workload(w, field_dtype=dtype, acc_mode="f64")
    assert p.get_option(fw.FWD_OPT_FD_ORDER) == 4
    p.set_model(w.rho)
    assert np.isclose(p.info.dt, ref["setup"].dt, rtol=1e-13)
    E, vol = p.forward(want_volume=True)
    assert rel(E.cpu().numpy(), ref["E_rec"]) < tol
    V = p.volume_export(vol).cpu().numpy()
    nz, ny, nx = w.shape
    for s in range(ns):
        ox, oy, oz = ref["vol"][s]
        assert rel(V[s, :, 0, :, :, :nx], ox) < tol
        assert rel(V[s, :, 1, :, :ny, :], oy) < tol
        assert rel(V[s, :, 2, :nz, :, :], oz) < tol


def test_order4_wholespace_matches_oracle():
    w = c1_wholespace(n=32, h=100.0, nt=600).replace(rec_pos=c1_wholespace().rec_pos,
                                                     fd_order=4)
    say("order-4 whole space 32^3, 600 steps, fp64")
    ref = oracle.forward(w)["E_rec"]
    p = fw.Plan.from_workload(w, field_dtype="f64")
    p.set_model(w.rho)
    assert rel(p.forward().cpu().numpy(), ref) < 1e-11


def _problem(seed=3, ns=2, vti=False):
    w_true = tiny(seed=seed, n=(14, 12, 10), npml=3, contrast=1.0, nr=8, nfreq=2,
                  ns=ns).replace(fd_order=4)
    if vti:
        w_true = with_vti(w_true, ratio=3.0, seed=seed, rho_min=0.0)
    rng = np.random.default_rng(seed + 100)
    kw = dict(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    if vti:
        kw["rho_v"] = w_true.rho_v * np.exp(0.3 * rng.standard_normal(w_true.rho.shape))
    w0 = w_true.replace(**kw)
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    return w0, d


@pytest.mark.parametrize("dtype,tb,tt", [("f64", 1e-7, 1e-9), ("f32", 1e-3, 1e-3)])
def test_order4_gradients_match_oracle(dtype, tb, tt):
    w0, d = _problem()
    say(f"order-4 gradients (basis and time-domain), {dtype}")
    fwd = oracle.forward(w0, want_volume=True)
    resid = d - fwd["E_rec"]
    gb = oracle.adjoint_gradient(w0, fwd, resid)["grad"]
    gt = adjoint_gradient_td(w0, resid)["grad"]
    p = fw.Plan.from_workload(w0, field_dtype=dtype)
    p.set_model(w0.rho)
    p.basis_build(gamma_rel=1e-12)
    E, vol = p.forward(want_volume=True)
    r = torch.from_numpy(d).cuda() - E
    g = p.adjoint(vol, r).cpu().numpy()
    g2 = p.adjoint_td(torch.from_numpy(resid).cuda(), segment=37).cpu().numpy()
    eb = np.linalg.norm(g - gb) / np.linalg.norm(gb)
    et = np.linalg.norm(g2 - gt) / np.linalg.norm(gt)
    say(f"  relative L2: basis {eb:.2e}, time-domain {et:.2e}")
    assert eb < tb and et < tt


def test_order4_vti_gradients_match_oracle():
    w0, d = _problem(vti=True)
    say("order-4 VTI split gradients, fp64")
    fwd = oracle.forward(w0, want_volume=True)
    resid = d - fwd["E_rec"]
    gb = oracle.adjoint_gradient(w0, fwd, resid)
    gt = adjoint_gradient_td(w0, resid)
    p = fw.Plan.from_workload(w0, field_dtype="f64")
    p.set_model(w0.rho, w0.rho_v)
    p.set_option(fw.FWD_OPT_VTI_GRADIENT, 1)
    p.basis_build(gamma_rel=1e-12)
    E, vol = p.forward(want_volume=True)
    assert rel(E.cpu().numpy(), fwd["E_rec"]) < 1e-11
    r = torch.from_numpy(resid).cuda()
    g = p.adjoint(vol, r).cpu().numpy()
    g2 = p.adjoint_td(r, segment=50).cpu().numpy()
    for k, name in enumerate(("grad_h", "grad_v")):
        eb = np.linalg.norm(g[k] - gb[name]) / np.linalg.norm(gb[name])
        et = np.linalg.norm(g2[k] - gt[name]) / np.linalg.norm(gt[name])
        say(f"  {name}: basis {eb:.2e}, time-domain {et:.2e}")
        assert eb < 1e-7 and et < 1e-9


TILINGS4 = [
    dict(block_x=64, block_y=4),
    dict(block_x=16, block_y=16, xcd_remap=0, tile_order=1),
    dict(block_x=32, block_y=8, xcd_remap=1, tile_order=0, graph_steps=0),
]


def test_order4_tilings_are_bitwise_identical():
    w0, d = _problem(seed=6)
    out = []
    for opts in TILINGS4:
        say(f"order-4 tiling {opts}")
        p = fw.Plan.from_workload(w0, field_dtype="f32", acc_mode="kahan")
        for key, v in opts.items():
            p.set_option(getattr(fw, "FWD_OPT_" + key.upper()), v)
        p.set_model(w0.rho)
        p.basis_build(gamma_rel=1e-12)
        E, vol = p.forward(want_volume=True)
        r = torch.from_numpy(d).cuda() - E
        out.append([E.cpu().numpy(), p.volume_export(vol).cpu().numpy(),
                    p.adjoint(vol, r).cpu().numpy(), p.adjoint_td(r, segment=41).cpu().numpy()])
    for o in out[1:]:
        for a, b in zip(out[0], o):
            assert np.array_equal(a, b)


def test_order4_options_and_autotune():
    """Order 4 runs the two-kernel schedule with scalar threads: other
    schedules and vector widths are refused, changing the order drops the
    model, and the autotuner keeps the results bit for bit."""
    w0, d = _problem(seed=7, ns=1)
    p = fw.Plan.from_workload(w0, field_dtype="f32")
    for key, v in ((fw.FWD_OPT_SCHEDULE, 1), (fw.FWD_OPT_VECTOR, 4), (fw.FWD_OPT_VECTOR_H, 4)):
        with pytest.raises(fw.FwdError):
            p.set_option(key, v)
    p.set_model(w0.rho)
    E0 = p.forward().cpu().numpy()
    p.autotune(steps=8)
    assert p.get_option(fw.FWD_OPT_SCHEDULE) == 0 and p.get_option(fw.FWD_OPT_VECTOR) == 1
    assert np.array_equal(p.forward().cpu().numpy(), E0)
    p.set_option(fw.FWD_OPT_FD_ORDER, 2)
    with pytest.raises(fw.FwdError):
        p.forward()
    p.set_model(w0.rho)
    E2 = p.forward().cpu().numpy()
    assert rel(E2, E0) > 1e-4                    # the orders differ
