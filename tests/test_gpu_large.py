"""The large workload (400x400x200 stretched grid, ~32M cells, 8
frequencies, 32 x-dipoles, 400 seabed receivers) on the GPU: the gradient of
a window of the run (forward + adjoint) for all 32 sources, which do not fit
in one plan (about 19 GB of workspace and volume transform per source), so
they run in groups sized from the plans' own memory figures and the
gradients are summed.

  * compensated-FP32 against FP64 volume accumulators (FP32 fields, both):
    receivers equal bit for bit (receiver transforms always accumulate in
    FP64), the summed gradient to 1e-6 in relative L2 (the transform sums
    and the gradient product, eq. dft and eq. gradsigmaij), and the volume
    transform per frequency;
  * one group against its single-source runs: receivers and volume bit for
    bit (batching changes no arithmetic per source), gradient to rounding;
  * FP32 against FP64 fields: the gradient to 1e-3 in relative L2.

The window is short next to the full run (73k steps), so the basis
functions fit poorly; both sides of each comparison use the same ones.
"""
import numpy as np
import pytest
import torch

from workloads import c5_large, with_window

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")

WINDOW = 128


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def large():
    w = with_window(c5_large(), WINDOW)
    rho0 = w.rho.copy()
    rho0[rho0 == 100.0] = 1.0                 # start model: the reservoir removed
    return w, rho0


def sub(w, a, b):
    return w.replace(src_pos=w.src_pos[a:b], src_mom=w.src_mom[a:b])


def plan_for(w, rho, dtype="f32", acc="kahan"):
    p = fw.Plan.from_workload(w, field_dtype=dtype, acc_mode=acc)
    p.set_model(rho)
    p.basis_build(gamma_rel=1e-12)
    return p


def group_size(w, rho, dtype, acc, frac=0.7):
    """Sources per plan whose workspace and volume transform fit in ``frac``
    of the free device memory."""
    one = fw.Plan.from_workload(sub(w, 0, 1), field_dtype=dtype, acc_mode=acc)
    one.set_model(rho)
    per = one.workspace_size(fw.FWD_MODE_ADJOINT) + one.volume_size()
    del one
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    return max(1, min(w.ns, int(frac * free // per))), per


def gradient(p, grad, accumulate):
    """Forward with the volume transform, then the adjoint of the misfit
    1/2 ||E||^2 (residual -E) added to ``grad``; returns E (host)."""
    E, vol = p.forward(want_volume=True)
    p.adjoint(vol, -E, grad=grad, accumulate=accumulate)
    del vol
    return E.cpu().numpy()


def volume_values(p, vol, acc, kf):
    """The raw volume transform of frequency kf as complex128 [ns][3][F] (FP64
    pairs, or compensated FP32 hi - lo)."""
    ns, nf = p.ns, p.nf
    if acc == "f64":
        v = vol.view(torch.float64).view(ns, nf, 3, -1, 2)[:, kf]
        return torch.complex(v[..., 0], v[..., 1])
    v = vol.view(torch.float32).view(ns, nf, 3, -1, 4)[:, kf]
    return torch.complex(v[..., 0].double() - v[..., 2].double(),
                         v[..., 1].double() - v[..., 3].double())


def test_large_gradient_all_sources_kahan_vs_f64(large):
    w, rho0 = large
    g, per = group_size(w, rho0, "f32", "f64")
    ng = -(-w.ns // g)
    say(f"large grid, {w.ns} sources, {WINDOW}+{WINDOW}-step window: groups of <= {g} "
        f"({ng} groups, {per / 1e9:.1f} GB per source)")
    assert ng >= 2                             # 32 sources do not fit in one plan
    grads = {}
    for acc in ("kahan", "f64"):
        grad = torch.zeros(w.shape, dtype=torch.float64, device="cuda")
        Es = []
        for gi, a in enumerate(range(0, w.ns, g)):
            p = plan_for(sub(w, a, min(a + g, w.ns)), rho0, "f32", acc)
            Es.append(gradient(p, grad, gi > 0))
            del p
            torch.cuda.empty_cache()
        grads[acc] = (grad.cpu().numpy(), np.concatenate(Es))
        say(f"  {acc}: |grad| max {np.abs(grads[acc][0]).max():.3e}")
    gk, Ek = grads["kahan"]
    gf, Ef = grads["f64"]
    assert np.isfinite(gf).all() and np.abs(gf).max() > 0
    assert bool(np.array_equal(Ek, Ef))        # receivers: FP64 sums in both runs
    err = np.linalg.norm(gk - gf) / np.linalg.norm(gf)
    say(f"  gradient, compensated FP32 against FP64 accumulators: relative L2 {err:.2e}")
    assert err < 1e-6


def test_large_volume_per_frequency_kahan_vs_f64(large):
    w, rho0 = large
    ws = sub(w, 0, 4)
    vols = {}
    for acc in ("kahan", "f64"):
        p = plan_for(ws, rho0, "f32", acc)
        _, vol = p.forward(want_volume=True)
        vols[acc] = (p, vol)
    pk, vk = vols["kahan"]
    pf, vf = vols["f64"]
    say("large grid, 4 sources: volume transform per frequency, compensated FP32 against FP64")
    for kf, f in enumerate(w.freqs):
        ref = volume_values(pf, vf, "f64", kf)
        err = float((volume_values(pk, vk, "kahan", kf) - ref).abs().max() / ref.abs().max())
        say(f"  {f:.3f} Hz: {err:.2e}")
        assert err < 1e-6


def test_large_group_equals_single_source_runs(large):
    w, rho0 = large
    ns = 4
    say(f"large grid: a group of {ns} sources against {ns} single-source plans")
    p = plan_for(sub(w, 0, ns), rho0, "f32", "kahan")
    grad = torch.zeros(w.shape, dtype=torch.float64, device="cuda")
    E, vol = p.forward(want_volume=True)
    p.adjoint(vol, -E, grad=grad)
    Eg, vb = E.cpu().numpy(), vol.view(ns, -1)
    g1 = torch.zeros_like(grad)
    for s in range(ns):
        q = plan_for(sub(w, s, s + 1), rho0, "f32", "kahan")
        E1, v1 = q.forward(want_volume=True)
        q.adjoint(v1, -E1, grad=g1, accumulate=s > 0)
        assert bool(np.array_equal(E1.cpu().numpy()[0], Eg[s]))
        assert torch.equal(v1.view(-1), vb[s])
        del q, v1
        torch.cuda.empty_cache()
    err = float((grad - g1).norm() / grad.norm())
    say(f"  receivers and volumes bit for bit; gradient {err:.1e}")
    assert err < 1e-12


def test_large_gradient_fp32_vs_fp64_fields(large):
    w, rho0 = large
    ws = sub(w, 14, 16)
    g = {}
    for dtype in ("f32", "f64"):
        p = plan_for(ws, rho0, dtype, "f64")
        grad = torch.zeros(w.shape, dtype=torch.float64, device="cuda")
        gradient(p, grad, False)
        g[dtype] = grad.cpu().numpy()
        del p
        torch.cuda.empty_cache()
    err = np.linalg.norm(g["f32"] - g["f64"]) / np.linalg.norm(g["f64"])
    say(f"large grid, 2 sources: gradient with FP32 against FP64 fields: relative L2 {err:.2e}")
    assert err < 1e-3
