"""Full-size GPU checks of the five workloads, by properties that hold at any
size (the CPU oracle cannot run them to completion; it is matched on windows
and small grids in test_gpu_parity.py).  Receiver transforms always
accumulate in FP64; the accumulator mode selects the type of the volume
transform, so accumulator checks compare exported volumes.

  * marine 1D (101x101x61, 45,758 steps): FP32 fields against FP64 fields at
    every receiver and frequency; over the whole run, the volume transform
    with compensated-FP32 and FP32 accumulators against FP64 accumulators
    (same FP32 fields);
  * three blocks (128x128x96): the FP64 basis-function gradient from
    FictitiousForward (its checkpoint is the forward volume transform)
    against central finite differences on 10 random interior cells, and the
    FP32 gradient against the FP64 one; the time-domain gradient (forward
    checkpoints every 200 steps) against central differences too;
  * batched (200x200x100, 16 sources): FP32 against FP64 per frequency on a
    window, batch against a single-source run;
  * large (400x400x200, ~32M cells, 8 frequencies): the volume transform with
    compensated-FP32 and FP32 accumulators against FP64 accumulators on a
    2000-step window of one source;
  * reciprocity on the full marine run in the benchmark's configuration
    (FP32 fields, FP64 accumulators, autotuned tiling): G_ab(r, s) =
    G_ba(s, r) for an off-grid source at the tow position and a seabed
    receiver 1.5 km away, all nine component pairs.
"""
import numpy as np
import pytest
import torch

from workloads import c2_marine1d, c3_blocks, c4_batched, c5_large, with_window

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")


def say(msg):
    print(msg, flush=True)


def forward(w, dtype, acc, volume=False):
    p = fw.Plan.from_workload(w, field_dtype=dtype, acc_mode=acc)
    p.set_model(w.rho)
    if volume:
        E, vol = p.forward(want_volume=True)
        return p, E.cpu().numpy(), vol
    return p, p.forward().cpu().numpy(), None


def receiver_errors(E, ref):
    """|E - ref| per receiver and frequency, relative to the receiver's
    largest component (components that vanish by symmetry do not count as
    their own scale)."""
    scale = np.abs(ref).max(axis=2, keepdims=True)          # [ns][nr][1][nf]
    return np.abs(E - ref) / scale


def volume_errors(v, ref):
    """Largest |v - ref| relative to the largest |ref| of the same source,
    frequency and component, and largest pointwise relative error over the
    nodes where |ref| is above 1e-3 of that maximum."""
    scale = ref.abs().amax(dim=(3, 4, 5), keepdim=True)
    d = (v - ref).abs()
    glob = float((d / scale).max())
    mask = ref.abs() > 1e-3 * scale
    point = float((d[mask] / ref.abs()[mask]).max())
    return glob, point


def test_marine_full_run_fp32_fields():
    w = c2_marine1d()
    say("marine full run: fp32 fields against fp64 at the receivers")
    _, E64, _ = forward(w, "f64", "f64")
    _, E32, _ = forward(w, "f32", "f64")
    err = receiver_errors(E32, E64)
    for k, f in enumerate(w.freqs):
        say(f"  {f:.2f} Hz: max {err[..., k].max():.2e}, median {np.median(err[..., k]):.2e}")
    assert err.max() < 1e-4


def accumulator_study(w, tol_kahan, tol_f32):
    vols = {}
    for acc in ("f64", "kahan", "f32"):
        p, _, vol = forward(w, "f32", acc, volume=True)
        vols[acc] = p.volume_export(vol)
        del p, vol
        torch.cuda.empty_cache()
    ref = vols.pop("f64")
    for acc, tol in (("kahan", tol_kahan), ("f32", tol_f32)):
        glob, point = volume_errors(vols[acc], ref)
        say(f"  {acc} against f64 accumulators: max {glob:.2e} of the maximum, "
            f"pointwise {point:.2e} above 1e-3 of it")
        assert glob < tol and point < 100 * tol


def test_marine_full_run_accumulators():
    say("marine full run: volume transform per accumulator mode, fp32 fields")
    accumulator_study(c2_marine1d(), 1e-7, 1e-5)


def _blocks_problem():
    """Data of the true three-block model; gradient at the 1 S/m background
    with dt, nt and the CPML reference velocity held at the background's
    values so that finite differences see one fixed discrete system."""
    w_true = c3_blocks()
    _, d, _ = forward(w_true, "f64", "f64")
    w0 = w_true.replace(rho=np.ones_like(w_true.rho))
    p = fw.Plan.from_workload(w0, field_dtype="f64")
    p.set_model(w0.rho)
    info = p.info
    w0 = w0.replace(dt=info.dt, nt=info.nt)
    w0.cpml_vref = info.vref
    return w0, torch.from_numpy(d).cuda()


def test_blocks_gradient_finite_differences():
    from paper_2211_16665_amd.autograd import FictitiousForward, misfit
    w0, d = _blocks_problem()
    say(f"three blocks: fp64 basis-function gradient, nt={w0.nt}")
    p = fw.Plan.from_workload(w0, field_dtype="f64")
    m0 = np.log(w0.rho)
    m = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = misfit(FictitiousForward.apply(m, p), d)
    L.backward()
    g = m.grad.cpu().numpy()
    rng = np.random.default_rng(1)
    nz, ny, nx = w0.shape
    cells = []
    while len(cells) < 10:
        c = (int(rng.integers(12, nz - 12)), int(rng.integers(12, ny - 12)), int(rng.integers(12, nx - 12)))
        if abs(g[c]) > 1e-3 * np.abs(g).max():      # cells where the gradient is not negligible
            cells.append(c)
    h = 1e-3
    errs = []
    for c in cells:
        vals = []
        for sgn in (1, -1):
            mm = m0.copy()
            mm[c] += sgn * h
            with torch.no_grad():
                E = FictitiousForward.apply(torch.from_numpy(mm).cuda(), p)
            vals.append(float(misfit(E, d)))
        fd = (vals[0] - vals[1]) / (2 * h)
        errs.append(abs(fd - g[c]) / abs(fd))
        say(f"  cell {c}: fd {fd:.6e} adjoint {g[c]:.6e} rel {errs[-1]:.2e}")
    assert max(errs) < 1e-3


def test_blocks_gradient_fp32_against_fp64():
    w0, d = _blocks_problem()
    say("three blocks: fp32 gradient against fp64")
    grads = {}
    for dtype, acc in (("f64", "f64"), ("f32", "f64"), ("f32", "kahan")):
        p = fw.Plan.from_workload(w0, field_dtype=dtype, acc_mode=acc)
        p.set_model(w0.rho)
        p.basis_build(gamma_rel=1e-12)
        E, vol = p.forward(want_volume=True)
        grads[(dtype, acc)] = p.adjoint(vol, d - E).cpu().numpy()
    ref = grads[("f64", "f64")]
    for key in (("f32", "f64"), ("f32", "kahan")):
        e = np.linalg.norm(grads[key] - ref) / np.linalg.norm(ref)
        say(f"  {key}: relative L2 {e:.2e}")
        assert e < 1e-3


def test_batched_window_fp32_and_single_source():
    w = with_window(c4_batched(), 400)
    say("batched 16 sources, 400-step window: fp32 against fp64, batch against one source")
    _, E64, _ = forward(w, "f64", "f64")
    _, E32, _ = forward(w, "f32", "f64")
    err = receiver_errors(E32, E64)
    for k, f in enumerate(w.freqs):
        say(f"  {f:.2f} Hz: max {err[..., k].max():.2e}")
    assert err.max() < 1e-4
    w1 = w.replace(src_pos=w.src_pos[5:6], src_mom=w.src_mom[5:6])
    _, E1, _ = forward(w1, "f32", "f64")
    assert bool(np.array_equal(E1[0], E32[5]))


def test_large_window_accumulators():
    w = c5_large()
    w = with_window(w.replace(src_pos=w.src_pos[:1], src_mom=w.src_mom[:1]), 2000)
    say("large grid (~32M cells), 1 source, 2000-step window: volume per accumulator mode")
    accumulator_study(w, 1e-7, 1e-5)


def test_blocks_td_gradient_finite_differences_and_basis():
    """Three blocks, FP64: the time-domain adjoint gradient (checkpoints every
    200 steps) against central differences on 6 interior cells and the 2
    largest-gradient cells of the CPML layers, and against the basis-function
    gradient outside the layers."""
    from paper_2211_16665_amd.autograd import FictitiousForward, misfit
    w0, d = _blocks_problem()
    say(f"three blocks: time-domain adjoint, nt={w0.nt}")
    p = fw.Plan.from_workload(w0, field_dtype="f64")
    m0 = np.log(w0.rho)
    m = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = misfit(FictitiousForward.apply(m, p, 200, 1e-12, "time"), d)
    L.backward()
    g = m.grad.cpu().numpy()
    p.basis_build(gamma_rel=1e-12)
    E, vol = p.forward(want_volume=True)
    gb = p.adjoint(vol, d - E).cpu().numpy()
    npml = w0.npml
    inner = (slice(npml, -npml),) * 3
    e = np.linalg.norm((g - gb)[inner]) / np.linalg.norm(gb[inner])
    say(f"  against the basis-function gradient outside the layers: {e:.2e}")
    assert e < 1e-6
    rng = np.random.default_rng(3)
    nz, ny, nx = w0.shape
    cells = []
    while len(cells) < 6:
        c = (int(rng.integers(12, nz - 12)), int(rng.integers(12, ny - 12)), int(rng.integers(12, nx - 12)))
        if abs(g[c]) > 1e-3 * np.abs(g).max():
            cells.append((c, 1e-3, 1e-3))
    layer = np.abs(g).copy()
    layer[inner] = 0.0                       # cells of the six CPML layers only
    for q in np.argsort(layer.ravel())[-2:]:
        cells.append((tuple(int(v) for v in np.unravel_index(q, layer.shape)), 1e-2, 1e-2))
    for c, h, tol in cells:
        vals = []
        for sgn in (1, -1):
            mm = m0.copy()
            mm[c] += sgn * h
            with torch.no_grad():
                Ec = FictitiousForward.apply(torch.from_numpy(mm).cuda(), p)
            vals.append(float(misfit(Ec, d)))
        fd = (vals[0] - vals[1]) / (2 * h)
        err = abs(fd - g[c]) / abs(fd)
        say(f"  cell {c}: fd {fd:.6e} time-domain adjoint {g[c]:.6e} rel {err:.2e}")
        assert err < tol


def test_marine_reciprocity_full_run():
    """The stepped operator is complex symmetric under the dual-volume
    pairing at any size: exchanging an off-grid source and receiver (with
    the same trilinear spreading and sampling) exchanges the components.
    FP32 fields over 45,758 steps: agreement to 1e-4 of the largest entry."""
    w = c2_marine1d()
    A = np.array([30.0, -20.0, 250.0])              # off-grid, 50 m above the seabed
    B = np.array([1530.0, 40.0, 330.0])             # off-grid, just below the seabed
    G = {}
    for (src, rec, key) in ((A, B, "ab"), (B, A, "ba")):
        p = fw.Plan.from_workload(w.replace(src_pos=np.array([src, src, src]),
                                            src_mom=np.eye(3), rec_pos=np.array([rec]),
                                            rec_comp=(0, 1, 2)),
                                  field_dtype="f32", acc_mode="f64")
        p.set_model(w.rho)
        p.autotune(fw.FWD_MODE_FORWARD, steps=16)
        say(f"marine reciprocity, source at {src}, {p.info.nt} steps")
        G[key] = p.forward().cpu().numpy()[:, 0]     # [source comp a][receiver comp b][nf]
    gab = G["ab"]                                    # E_b at B due to p_a at A
    gba = np.swapaxes(G["ba"], 0, 1)                 # E_a at A due to p_b at B, as [a][b]
    scale = np.abs(gab).max(axis=(0, 1))             # per frequency
    err = (np.abs(gab - gba).max(axis=(0, 1)) / scale)
    say(f"  max |G_ab - G_ba| / max |G| per frequency: {err}")
    assert np.all(err < 1e-4)

