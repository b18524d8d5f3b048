"""Non-temporal stores (FWD_OPT_STREAM_STORES) change only the cache hint of
the field and history stores: receivers, the volume transform
and the gradient are the same bit for bit with the hint on and off, on every
schedule, precision and transform block, and the automatic choice follows
the working set (off on grids whose streamed bytes fit the 256 MB Infinity
Cache, on above).
"""
import pytest
import torch

from workloads import tiny

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")


def say(msg):
    print(msg, flush=True)


def run(w, dtype, acc, nts, **opt):
    p = fw.Plan.from_workload(w, field_dtype=dtype, acc_mode=acc)
    for k, v in opt.items():
        p.set_option(getattr(fw, "FWD_OPT_" + k.upper()), v)
    p.set_option(fw.FWD_OPT_STREAM_STORES, nts)
    p.set_model(w.rho)
    p.basis_build(gamma_rel=1e-12)
    E, vol = p.forward(want_volume=True)
    g = p.adjoint(vol, -E)
    return E, vol, g


@pytest.mark.parametrize("dtype,acc,opt", [
    ("f64", "f64", {}),
    ("f32", "kahan", {"dft_block": 16}),
    ("f32", "f32", {"vector": 4, "vector_h": 4}),
    ("f32", "kahan", {"dft_decimate": 4}),
    ("f32", "kahan", {"schedule": 1, "block_x": 64, "block_y": 4}),
    ("f32", "kahan", {"schedule": 2, "block_x": 64, "block_y": 4}),
])
def test_hint_does_not_change_results(dtype, acc, opt):
    w = tiny(seed=21, npml=3, ns=2, moment_dirs=True)
    say(f"stream stores on/off: {dtype} {acc} {opt}")
    E0, v0, g0 = run(w, dtype, acc, 0, **opt)
    E1, v1, g1 = run(w, dtype, acc, 1, **opt)
    assert torch.equal(E0, E1)
    assert torch.equal(v0, v1)
    assert torch.equal(g0, g1)


def test_automatic_choice_follows_the_working_set():
    """Automatic (-1) is off on a grid whose streamed bytes fit the 256 MB
    Infinity Cache and on above it: its results equal the run with the
    matching fixed setting bit for bit, and the autotuner leaves the option
    at -1."""
    w = tiny(seed=22, npml=3, ns=1)
    E_auto, v_auto, _ = run(w, "f32", "kahan", -1)
    E_off, v_off, _ = run(w, "f32", "kahan", 0)
    assert torch.equal(E_auto, E_off) and torch.equal(v_auto, v_off)
    p = fw.Plan.from_workload(w, field_dtype="f32", acc_mode="kahan")
    p.set_model(w.rho)
    p.autotune(fw.FWD_MODE_FORWARD, vol=p.volume_buffer(), steps=8)
    assert p.get_option(fw.FWD_OPT_STREAM_STORES) == -1
