"""The product path works in a fresh process that creates a Plan before it
touches torch itself (the binding loads torch's HIP runtime before the
library)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
from paper_2211_16665_amd import Plan
from workloads import tiny
w = tiny(seed=1, npml=3, ns=1)
p = Plan.from_workload(w, field_dtype="f64")
p.set_model(w.rho)
E = p.forward().cpu().numpy()
assert np.isfinite(E).all() and np.abs(E).max() > 0
print("ok", E.shape, flush=True)
"""


def test_plan_before_torch_in_a_fresh_process():
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
