"""Writes marine_window.json: the oracle's receiver fields of the marine
workload (101x101x61 stretched grid, x-dipole 50 m above the seabed, 50
seabed receivers at offsets 0.1 to 2.5 km) after a window of its first
WINDOW steps, long enough for the field to cross the whole tow line through
the sediment (about 4,500 steps for 2.5 km at 1 ohm-m).  Calls only the
oracle; takes about ten minutes on one core.

    python tests/golden/make_marine_window.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                                            # noqa: E402
from workloads import c2_marine1d, with_window           # noqa: E402

WINDOW = 6000


def main():
    w = with_window(c2_marine1d(), WINDOW)
    t0 = time.time()
    r = oracle.forward(w)
    E = r["E_rec"]                                       # [1][50][2][3]
    out = {
        "what": "oracle receiver fields E(omega_k) of the marine workload after its first "
                f"{WINDOW} steps (partial sums of eq. dft, normalised as the full run)",
        "workload": "c2_marine1d", "steps": WINDOW, "dt": float(r["setup"].dt),
        "freqs": [float(f) for f in w.freqs], "rec_comp": list(w.rec_comp),
        "rec_x": [float(p[0]) for p in w.rec_pos], "src_x": float(w.src_pos[0][0]),
        "re": E.real.tolist(), "im": E.imag.tolist(),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "marine_window.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} in {out['oracle_seconds']} s")


if __name__ == "__main__":
    main()
