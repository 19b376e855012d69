"""Writes tests/golden/fstar_40pow5_r16.json: the target fit of the
time-to-fit study, i.e. the explicit fit the float64 oracle's plain
ALS-QR-BR (restructured order, no extrapolation) reaches after 200 sweeps on
the 40^5 rank-16 workload (planted congruence 0.85, noise 1e-3; the float32
tensor promoted exactly to float64).  Calls only the oracle and the seeded
generators.  Run from the repository root:  python tests/golden/make_fstar.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synthgen as G  # noqa: E402

SWEEPS = 200


def main():
    prob = G.workload("fp32_40pow5_r16")
    X = prob.X.astype(np.float64)
    t0 = time.time()
    r = O.cp_als_qr(X, prob.rank, prob.init, SWEEPS, tree="restructured", extrap="off",
                    sweep_callback=lambda k, f: print(f"sweep {k} fit {f:.10f} "
                                                      f"({time.time() - t0:.0f} s)", flush=True))
    out = {
        "workload": "fp32_40pow5_r16",
        "what": "explicit fit of the float64 oracle's plain ALS-QR-BR after 200 sweeps "
                "(restructured order), the time-to-fit target f*",
        "sweeps": SWEEPS,
        "fstar": float(r["fitx"]),
        "fits": [float(f) for f in r["fits"]],
        "script": "tests/golden/make_fstar.py",
    }
    with open(os.path.join(ROOT, "tests", "golden", "fstar_40pow5_r16.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("fstar", out["fstar"])


if __name__ == "__main__":
    main()
