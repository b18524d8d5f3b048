"""A run does not clear the volume buffer: the first transform block of the
run writes every accumulator (zeros off the components' lattices), and a
run flushed before its first sample clears the buffer at the flush.  The
buffer's bytes after a run must therefore not depend on what it held
before: a buffer filled with NaN bytes ends bit for bit equal to one filled
with zeros, for every accumulator type, transform block (including K = 1,
one block per step), decimation, schedule, and for runs split and flushed
inside the first block.
"""
import numpy as np
import pytest
import torch

from workloads import tiny

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")


def say(msg):
    print(msg, flush=True)


def plan(w, dtype, acc, **opt):
    p = fw.Plan.from_workload(w, field_dtype=dtype, acc_mode=acc)
    for k, v in opt.items():
        p.set_option(getattr(fw, "FWD_OPT_" + k.upper()), v)
    p.set_model(w.rho)
    return p


def buffers(p):
    nan = p.volume_buffer()
    nan.fill_(0xFF)                        # every accumulator NaN
    zero = p.volume_buffer()
    zero.zero_()
    return nan, zero


@pytest.mark.parametrize("dtype,acc,opt", [
    ("f64", "f64", {}),
    ("f32", "kahan", {}),
    ("f32", "f32", {"dft_block": 1}),
    ("f32", "kahan", {"dft_block": 16, "dft_decimate": 4}),
    ("f32", "kahan", {"schedule": 1, "block_x": 64, "block_y": 4}),
    ("f32", "kahan", {"schedule": 2, "block_x": 64, "block_y": 4}),
])
def test_prior_contents_do_not_matter(dtype, acc, opt):
    w = tiny(seed=11, npml=3, ns=2, moment_dirs=True)
    p = plan(w, dtype, acc, **opt)
    say(f"full run over NaN and zero buffers: {dtype} {acc} {opt}")
    nan, zero = buffers(p)
    E1, _ = p.forward(vol=nan, want_volume=True)
    E0, _ = p.forward(vol=zero, want_volume=True)
    assert torch.equal(nan, zero)
    assert torch.equal(E1, E0)
    assert torch.isfinite(p.volume_export(nan)).all()


def test_split_run_flushed_inside_the_first_block():
    w = tiny(seed=12, npml=3, ns=2)
    p = plan(w, "f32", "kahan", dft_block=16)
    say("split run: flush at step 5, inside the first block")
    ref, _ = buffers(p)
    p.forward(vol=ref, want_volume=True)
    nan, _ = buffers(p)
    p.run_begin(nan)
    p.run_steps(5, nan)
    p.run_flush(nan)
    p.run_steps(p.info.nt - 5, nan)
    p.run_flush(nan)
    a = p.volume_export(nan).cpu().numpy()
    b = p.volume_export(ref).cpu().numpy()
    assert np.isfinite(a).all()
    assert np.abs(a - b).max() <= 1e-6 * np.abs(b).max()


def test_flushed_before_the_first_sample():
    """No sample yet (no step, or fewer steps than the decimation D): the
    flush clears the buffer, and the run continues from it as usual."""
    w = tiny(seed=13, npml=3, ns=1)
    say("flush before any sample")
    p = plan(w, "f64", "f64")
    nan, _ = buffers(p)
    p.run_begin(nan)
    p.run_flush(nan)
    assert not torch.any(nan)
    p = plan(w, "f64", "f64", dft_decimate=8)
    ref, _ = buffers(p)
    p.forward(vol=ref, want_volume=True)
    nan, _ = buffers(p)
    p.run_begin(nan)
    p.run_steps(5, nan)
    p.run_flush(nan)
    assert not torch.any(nan)
    p.run_steps(p.info.nt - 5, nan)
    p.run_flush(nan)
    assert torch.equal(nan, ref)
