"""The decimated forward volume transform (FWD_OPT_DFT_DECIMATE = D: samples
E^m with m a multiple of D, weight D) on the GPU against the oracle's
decimated transform, and its error against the exact transform on the full
marine run.

  * tiny grids, FP64: the volume against the oracle to 1e-11 for several D
    and transform blocks (including blocks longer than the run's last
    partial block, and D * K longer than the graph chunk); order 4 too;
  * the basis-function gradient from a decimated forward volume against the
    oracle's (exact adjoint transform on both sides) to 1e-7;
  * graph replay against eager launches bit for bit, and a run flushed
    inside a block and continued to rounding;
  * schedules other than the two-kernel one refuse a decimated transform;
  * marine workload, full run, FP32 fields: volume and gradient against the
    undecimated run for D = 2 .. 64 (the error study).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.discretization import make_setup
from workloads import c2_marine1d, tiny

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def plan(w, dtype="f64", acc="f64", **opt):
    p = fw.Plan.from_workload(w, field_dtype=dtype, acc_mode=acc)
    for k, v in opt.items():
        p.set_option(getattr(fw, "FWD_OPT_" + k.upper()), v)
    p.set_model(w.rho)
    return p


def volume_rel(p, vol, ref_vols):
    V = p.volume_export(vol).cpu().numpy()
    err = 0.0
    for s in range(len(ref_vols)):
        for c in range(3):
            r = ref_vols[s][c]
            nz, ny, nx = r.shape[1:]
            err = max(err, rel(V[s, :, c, :nz, :ny, :nx], r))
    return err


@pytest.mark.parametrize("D,kb,order", [(2, 8, 2), (4, 16, 2), (8, 1, 2), (64, 8, 2), (4, 8, 4)])
def test_decimated_volume_matches_oracle(D, kb, order):
    w = tiny(seed=2, npml=3, ns=2, moment_dirs=True, contrast=1.5).replace(fd_order=order)
    say(f"decimated volume D={D} K={kb} order={order}")
    ref = oracle.forward(w, want_volume=True, decimate=D)
    p = plan(w, dft_decimate=D, dft_block=kb)
    E, vol = p.forward(want_volume=True)
    assert rel(E.cpu().numpy(), ref["E_rec"]) < 1e-11        # receivers keep every sample
    err = volume_rel(p, vol, ref["vol"])
    say(f"  volume {err:.2e} (nt = {p.info.nt})")
    assert err < 1e-11


@pytest.mark.parametrize("D,dtype,tol", [(4, "f64", 1e-7), (8, "f32", 1e-3)])
def test_decimated_gradient_matches_oracle(D, dtype, tol):
    w_true = tiny(seed=5, n=(14, 12, 10), npml=3, contrast=1.0, nr=8, nfreq=2, ns=2)
    rng = np.random.default_rng(105)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    say(f"decimated gradient D={D} {dtype}")
    fwd = oracle.forward(w0, want_volume=True, decimate=D)
    go = oracle.adjoint_gradient(w0, fwd, d - fwd["E_rec"])["grad"]
    p = plan(w0, dtype, dft_decimate=D)
    p.basis_build(gamma_rel=1e-12)
    E, vol = p.forward(want_volume=True)
    g = p.adjoint(vol, torch.from_numpy(d).cuda() - E).cpu().numpy()
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    say(f"  relative L2 {err:.2e}")
    assert err < tol


def test_decimated_graph_eager_bitwise_and_flush_midway():
    """Graph replay and eager launches give the same bits; a flush inside a
    block (between two samples) followed by the rest of the run splits that
    block's sum in two, so it agrees to rounding (FP64)."""
    w = tiny(seed=7, npml=3, ns=2)
    say("decimated transform: graph, eager, flush midway")
    outs = []
    for gs in (32, 0):
        p = plan(w, "f32", "kahan", dft_decimate=4, dft_block=8, graph_steps=gs)
        _, vol = p.forward(want_volume=True)
        outs.append(p.volume_export(vol).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    p = plan(w, "f64", "f64", dft_decimate=4, dft_block=8)
    nt = p.info.nt
    _, vol_full = p.forward(want_volume=True)
    ref = p.volume_export(vol_full).cpu().numpy()
    vol = p.volume_buffer()
    p.run_begin(vol)
    k = 4 * 8 * 3 + 13                       # inside a block, between samples
    p.run_steps(k, vol)
    p.run_flush(vol)
    p.run_flush(vol)                         # idempotent
    p.run_steps(nt - k, vol)
    p.run_flush(vol)
    assert rel(p.volume_export(vol).cpu().numpy(), ref) < 1e-13


def test_decimated_transform_refuses_other_schedules():
    w = tiny(seed=8, npml=3, ns=1)
    for sched in (1, 2):
        p = plan(w, "f32", dft_decimate=4, schedule=sched, block_x=64, block_y=4)
        with pytest.raises(fw.FwdError) as e:
            p.forward(want_volume=True)
        assert e.value.status == 7
        p.forward()                          # without a volume transform it runs


def test_marine_decimation_error_study():
    """Full marine run (45,758 steps, wavelet width tau / dt ~ 200), FP32
    fields, FP64 accumulators: the volume transform and the gradient for
    D = 2 .. 64 against D = 1."""
    w_true = c2_marine1d()
    rho0 = w_true.rho.copy()
    rho0[rho0 == 100.0] = 1.0
    p = plan(w_true, "f32", "f64")
    d = p.forward()
    p.set_model(rho0)
    p.basis_build(gamma_rel=1e-12)
    say(f"marine decimation study: tau/dt = {p.info.tau / p.info.dt:.0f}")
    out = {}
    for D in (1, 2, 4, 8, 16, 32, 64):
        p.set_option(fw.FWD_OPT_DFT_DECIMATE, D)
        E, vol = p.forward(want_volume=True)
        g = p.adjoint(vol, d - E).cpu().numpy()
        out[D] = (p.volume_export(vol).cpu().numpy(), g)
        del vol
    v1, g1 = out[1]
    errs = {}
    for D in (2, 4, 8, 16, 32, 64):
        ev = rel(out[D][0], v1)
        eg = np.linalg.norm(out[D][1] - g1) / np.linalg.norm(g1)
        errs[D] = (ev, eg)
        say(f"  D={D}: volume {ev:.2e} of the maximum, gradient {eg:.2e} (relative L2)")
    assert errs[8][1] < 1e-4
    assert errs[64][1] > errs[8][1]
