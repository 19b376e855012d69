"""Writes tests/golden/full_runs/*.npz: full-length float64 oracle runs of the
benchmark workloads, the reference of the GPU parity tests at the workloads'
own sweep counts.  Calls only the oracle and the seeded generators (the
float32 tensors are promoted exactly to float64).

Runs (name: workload, tree, extrapolation, sweeps):
  256cube_r32_restructured   256^3 rank 32, congruence 0.9, noise 1e-3;
                             restructured tree, no extrapolation, 100 sweeps
  256cube_r32_standard       same, standard dimension tree, 100 sweeps
  96pow4_r20_paper           96^4 rank 20, congruence 0.8, noise 1e-2;
                             restructured tree with the paper's extrapolation
                             (eq. (19), Section 4.3 rule), 200 sweeps
  40pow5_r16_plain           40^5 rank 16, congruence 0.85, noise 1e-3;
                             restructured tree, no extrapolation, 200 sweeps
  40pow5_r16_paper           same with the paper's extrapolation, 200 sweeps
  batch64                    the 64 independent order-3 problems (dims
                             U{32..160}, ranks U{4..24}, 1% noise),
                             restructured tree, 50 sweeps each

Each file holds the per-sweep fits (Section 4.1 formula), the final explicit
fit, lambda, the factors, the update orders and the activation sweep / beta.
Run from the repository root:
    python tests/golden/make_full_runs.py [name ...]
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

OUT = os.path.join(ROOT, "tests", "golden", "full_runs")

RUNS = {
    "256cube_r32_restructured": dict(workload="fp32_256cube_r32", tree="restructured", extrap="off",
                                     sweeps=100),
    "256cube_r32_standard": dict(workload="fp32_256cube_r32", tree="standard", extrap="off", sweeps=100),
    "96pow4_r20_paper": dict(workload="fp32_96pow4_r20", tree="restructured", extrap="paper", sweeps=200),
    "40pow5_r16_plain": dict(workload="fp32_40pow5_r16", tree="restructured", extrap="off", sweeps=200),
    "40pow5_r16_paper": dict(workload="fp32_40pow5_r16", tree="restructured", extrap="paper", sweeps=200),
    "batch64": dict(workload="batch64", tree="restructured", extrap="off", sweeps=50),
}


def run_one(prob, spec, log):
    t0 = time.time()
    every = max(1, spec["sweeps"] // 10)
    r = O.cp_als_qr(prob.X.astype(np.float64), prob.rank, prob.init, spec["sweeps"],
                    tree=spec["tree"], extrap=spec["extrap"],
                    sweep_callback=lambda k, f: log(f"  sweep {k} fit {f:.10f} ({time.time() - t0:.0f} s)")
                    if k % every == 0 else None)
    return r


def main(names):
    os.makedirs(OUT, exist_ok=True)
    manifest_path = os.path.join(OUT, "manifest.json")
    manifest = {}
    if os.path.exists(manifest_path):
        with open(manifest_path) as f:
            manifest = json.load(f)
    for name in names:
        spec = RUNS[name]

        def log(msg):
            print(f"[{name}] {msg}", flush=True)

        t0 = time.time()
        if spec["workload"] == "batch64":
            probs = G.batched_workload(64)
            arrays = {}
            for t, p in enumerate(probs):
                r = run_one(p, spec, lambda m: None)
                arrays[f"p{t}_fits"] = r["fits"]
                arrays[f"p{t}_fitx"] = np.array(r["fitx"])
                arrays[f"p{t}_lam"] = r["lam"]
                for n, a in enumerate(r["factors"]):
                    # float32 copies: the GPU comparison of the factors is by
                    # column cosines at float32 level
                    arrays[f"p{t}_A{n}"] = a.astype(np.float32)
                arrays[f"p{t}_orders"] = np.array(r["orders"], dtype=np.int32)
                log(f"problem {t}: dims {list(p.X.shape)} rank {p.rank} fitx {r['fitx']:.10f}")
        else:
            prob = G.workload(spec["workload"])
            r = run_one(prob, spec, log)
            arrays = {"fits": r["fits"], "fitx": np.array(r["fitx"]), "lam": r["lam"],
                      "orders": np.array(r["orders"], dtype=np.int32),
                      "beta": np.array(r["beta"]), "beta_sweep": np.array(r["beta_sweep"])}
            for n, a in enumerate(r["factors"]):
                arrays[f"A{n}"] = a
            log(f"fitx {r['fitx']:.12f} beta {r['beta']} at sweep {r['beta_sweep']}")
        np.savez_compressed(os.path.join(OUT, name + ".npz"), **arrays)
        manifest[name] = dict(spec, seconds=round(time.time() - t0, 1),
                              script="tests/golden/make_full_runs.py")
        with open(manifest_path, "w") as f:
            json.dump(manifest, f, indent=1, sort_keys=True)
        log(f"written in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1:] or list(RUNS))
