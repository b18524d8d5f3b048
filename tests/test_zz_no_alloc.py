"""fwd_forward_static, the forward run for callers that cannot allocate (its
workspace is the library's static device array): through the C ABI, against
fwd_forward on the same plan, on two calls in a row -- the second with a
smaller grid.  Same kernels launched one by one instead of from a graph:
receivers and volume transform equal bit for bit.  The call makes no device
allocation (the device's free memory is unchanged across it), refuses a
plan whose tables are not on the device yet, and refuses a workspace
larger than the static array."""
import numpy as np
import pytest
import torch

from workloads import c2_marine1d, tiny

pytestmark = pytest.mark.gpu

fw = pytest.importorskip("paper_2211_16665_amd.fwdem")


def say(msg):
    print(msg, flush=True)


def check_against_forward(w):
    p = fw.Plan.from_workload(w, field_dtype="f32", acc_mode="kahan")
    p.set_model(w.rho)
    E_ref, vol_ref = p.forward(want_volume=True)
    V_ref = p.volume_export(vol_ref).cpu().numpy()
    vol = p.volume_buffer()
    out = p.rec_buffer()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    E = p.forward_static(vol=vol, out=out)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    assert np.array_equal(E.cpu().numpy(), E_ref.cpu().numpy())
    assert np.array_equal(p.volume_export(vol).cpu().numpy(), V_ref)
    return p.workspace_size(fw.FWD_MODE_FORWARD)


def test_static_forward_two_calls_second_smaller():
    w1 = tiny(seed=21, n=(18, 16, 14), npml=3, ns=2, nr=5, nfreq=3)
    w2 = tiny(seed=22, n=(12, 10, 10), npml=2, ns=1, nr=3, nfreq=2)
    b1 = check_against_forward(w1)
    b2 = check_against_forward(w2)
    say(f"static forward equals fwd_forward: workspaces {b1} then {b2} bytes")
    assert b2 < b1 < fw.FWD_STATIC_SCRATCH_BYTES


def test_static_forward_refusals():
    w = tiny(seed=23, n=(12, 10, 10), npml=2, ns=1, nr=3, nfreq=2)
    p = fw.Plan.from_workload(w, field_dtype="f32", acc_mode="f64")
    p.set_model(w.rho)
    with pytest.raises(fw.FwdError) as e:          # tables not on the device yet
        p.forward_static()
    assert e.value.status == 8
    big = c2_marine1d().replace(nt=4)              # workspace above the static array
    q = fw.Plan.from_workload(big, field_dtype="f32", acc_mode="f64")
    q.set_model(big.rho)
    assert q.workspace_size(fw.FWD_MODE_FORWARD) > fw.FWD_STATIC_SCRATCH_BYTES
    q.forward()
    with pytest.raises(fw.FwdError) as e:
        q.forward_static()
    assert e.value.status == 1
