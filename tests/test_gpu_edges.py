"""Edge cases of the forward and adjoint path against the oracle (FP64 fields
and accumulators, so the bar is rounding):
  * the smallest grids the plan accepts (2 npml + 4 cells per axis);
  * grids ragged against the tiles (one node past a 64-wide tile, tiles
    taller than the grid), on every schedule;
  * absorbing layers that leave a four-cell interior;
  * one frequency, one receiver, one component, sources and receivers on
    grid nodes;
  * runs of one to five steps, where the first transform block is also the
    flushed last one (with and without decimation, blocks of 1, 2 and 8);
  * the gradient on a minimal grid;
  * adjoints of a zero residual and of residuals scaled by powers of two.
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
    """Largest difference over the largest reference value; where the
    reference is exactly zero (a component the first steps have not reached)
    the result must be too."""
    big = np.abs(b).max()
    return float(np.abs(a - b).max() / big) if big > 0 else float(np.abs(a).max())


def plan(w, **opt):
    p = fw.Plan.from_workload(w, field_dtype="f64", acc_mode="f64")
    for k, v in opt.items():
        p.set_option(getattr(fw, "FWD_OPT_" + k.upper()), v)
    p.set_model(w.rho)
    return p


def check_forward(w, decimate=1, tol=1e-11, **opt):
    ref = oracle.forward(w, want_volume=True, decimate=decimate)
    p = plan(w, dft_decimate=decimate, **opt)
    E, vol = p.forward(want_volume=True)
    assert rel(E.cpu().numpy(), ref["E_rec"]) < tol
    V = p.volume_export(vol).cpu().numpy()
    nz, ny, nx = w.shape
    for s in range(w.ns):
        ox, oy, oz = ref["vol"][s]
        assert rel(V[s, :, 0, :, :, :nx], ox) < 1e-11
        assert rel(V[s, :, 1, :, :ny, :], oy) < 1e-11
        assert rel(V[s, :, 2, :nz, :, :], oz) < 1e-11


# The 65-cell grid's receivers lie up to 30 cells from the sources, six
# orders of magnitude below the fields near them: FP64 rounding of those
# fields reaches 2e-11 of the receivers' largest value (the volume transform,
# which holds the near-source fields, still agrees to 1e-11).
@pytest.mark.parametrize("n,npml,opt,tol", [
    ((4, 4, 4), 0, {}, 1e-11),
    ((5, 4, 7), 0, {"vector": 4, "vector_h": 4}, 1e-11),
    ((65, 4, 4), 0, {"block_x": 64, "block_y": 1}, 1e-10),
    ((65, 4, 4), 0, {"block_x": 16, "block_y": 16, "vector": 4, "vector_h": 4}, 1e-10),
    ((12, 12, 12), 4, {}, 1e-11),
    ((20, 8, 8), 2, {"block_x": 16, "block_y": 16}, 1e-11),
    ((20, 8, 8), 2, {"schedule": 1, "block_x": 16, "block_y": 8, "zchunk": 64}, 1e-11),
    ((20, 8, 8), 2, {"schedule": 2, "block_x": 64, "block_y": 4}, 1e-11),
])
def test_small_and_ragged_grids(n, npml, opt, tol):
    w = tiny(seed=31, n=n, npml=npml, ns=2, moment_dirs=True, contrast=1.0)
    say(f"grid {n} npml {npml} {opt}")
    check_forward(w, tol=tol, **opt)


def test_one_frequency_receiver_and_component_on_nodes():
    w = tiny(seed=32, n=(9, 8, 8), npml=2, ns=1, nfreq=1, nr=1, rec_comp=(2,), off_grid=False)
    say("one frequency, one receiver, one component, on nodes")
    check_forward(w)


@pytest.mark.parametrize("nt,decimate,kb", [(1, 1, 8), (2, 1, 1), (3, 1, 2), (3, 2, 8), (5, 2, 2)])
def test_runs_of_a_few_steps(nt, decimate, kb):
    w = tiny(seed=33, n=(8, 9, 8), npml=2, ns=2)
    s = make_setup(w)
    w = w.replace(dt=s.dt, nt=nt)
    w.cpml_vref = s.vref
    say(f"{nt} steps, decimation {decimate}, block {kb}")
    check_forward(w, decimate=decimate, dft_block=kb)


def test_gradient_on_a_minimal_grid():
    w_true = tiny(seed=34, n=(4, 4, 5), npml=0, ns=2, nr=3, contrast=0.5)
    rng = np.random.default_rng(134)
    w0 = w_true.replace(rho=w_true.rho * np.exp(0.3 * rng.standard_normal(w_true.rho.shape)))
    d = oracle.forward(w_true)["E_rec"]
    s0 = make_setup(w0)
    w0 = w0.replace(dt=s0.dt, nt=s0.nt)
    w0.cpml_vref = s0.vref
    say("gradient on a 4x4x5 grid")
    fwd = oracle.forward(w0, want_volume=True)
    go = oracle.adjoint_gradient(w0, fwd, d - fwd["E_rec"])["grad"]
    p = plan(w0)
    p.basis_build(gamma_rel=1e-12)
    E, vol = p.forward(want_volume=True)
    g = p.adjoint(vol, torch.from_numpy(d).cuda() - E).cpu().numpy()
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    say(f"  relative L2 {err:.2e}")
    assert err < 1e-7


def test_adjoint_of_zero_and_scaled_residuals():
    """The adjoint sources are formed on the device with a power-of-two
    scale: a zero residual gives an exactly zero gradient (no 0/0), and a
    residual scaled by 2^k (k = -60, 90) gives the gradient scaled by 2^k
    bit for bit, with FP32 fields as with FP64."""
    w_true = tiny(seed=35, n=(8, 8, 8), npml=2, ns=2, nr=4)
    w0 = w_true.replace(rho=w_true.rho * 1.3)
    d = torch.from_numpy(oracle.forward(w_true)["E_rec"]).cuda()
    for dtype in ("f64", "f32"):
        say(f"zero and scaled residuals, {dtype}")
        p = fw.Plan.from_workload(w0, field_dtype=dtype, acc_mode="f64")
        p.set_model(w0.rho)
        p.basis_build(gamma_rel=1e-12)
        E, vol = p.forward(want_volume=True)
        g0 = p.adjoint(vol, torch.zeros_like(E))
        assert not torch.any(g0)
        r = d - E
        g = p.adjoint(vol, r)
        assert torch.isfinite(g).all() and torch.any(g)
        for k in (-60, 90):
            gk = p.adjoint(vol, r * 2.0 ** k)
            assert torch.equal(gk, g * 2.0 ** k), k
