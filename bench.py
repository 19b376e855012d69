#!/usr/bin/env python
"""Benchmark: ALS-QR sweeps per second on one MI355X.

A step is one full ALS-QR sweep (every TTM of the restructured dimension
tree, and for every mode: Khatri-Rao of the R factors and its Householder
TSQR, Y_(n) Q0, the triangular solve, normalisation, factor QR, fit) over the
256 x 256 x 256 float32 rank-32 workload (planted factors with pairwise
congruence 0.9, noise 1e-3 relative), inputs resident in HBM.

Prints one JSON line.  ``value`` comes from the timed region (HIP graph
replay, K sweeps, synchronised on both sides).  ``roofline`` describes the
level-1 TTM (the TTM that streams X, the dominant streaming kernel): its
average duration comes from HIP events on the library's stream during a
second pass of the same K sweeps launched kernel by kernel, in which every
level-1 TTM runs as a graph of 8 back-to-back launches (it is idempotent)
between two events.  ``cpu_baseline`` times the FP64 oracle on a bounded
sample of sweeps of the same workload on the host cores.

Extra keys on the same line (skipped with --no-extras): ``orders`` holds the
sweep rates of the order-4 (96^4, rank 20) and order-5 (40^5, rank 16)
workloads, measured the same way with their own level-1 TTM roofline;
``time_to_fit`` holds the wall time of plain ALS-QR-BR, the paper's
ALS-QR-BRE and the learned extrapolation to reach the float64 oracle's fit
minus 1e-6 on the order-5 workload (time_to_fit_study).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ALS-QR sweeps/s + TTM %MFMA peak; time-to-fit learned vs plain extrapolation"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
WORKLOAD = "fp32_256cube_r32"


def _traffic_from_profile(kernel_src: str):
    """HBM bytes per level-1 TTM launch from the committed rocprofv3 counter
    summary, if it was taken on the current TTM source; else None."""
    path = os.path.join(ROOT, "profiles", "ttm_l1_256cube_r32_counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        with open(kernel_src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if d.get("ttm_source_sha256") != sha:
            return None
        return float(d["hbm_bytes_per_launch"])
    except Exception:
        return None


def _cpu_model() -> str:
    """Host CPU model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, budget_s: float):
    """Oracle sweeps/s on a bounded sample (first sweep excluded)."""
    import numpy as np
    import oracle as O
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    X = np.asarray(prob.X, dtype=np.float64)
    stamps = []

    class _Stop(Exception):
        pass

    def cb(k, fit):
        stamps.append(time.perf_counter())
        if stamps[-1] - stamps[0] > budget_s and len(stamps) >= 3:
            raise _Stop()

    try:
        O.cp_als_qr(X, prob.rank, prob.init, 10_000, tree="restructured",
                    explicit_final=False, sweep_callback=cb)
    except _Stop:
        pass
    n = len(stamps) - 1
    sec = stamps[-1] - stamps[0]
    return {"value": n / sec, "unit": "sweeps/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count() or 1,
            "sample": f"sweeps 2..{n + 1} of the same workload (restructured order, direct "
                      f"multi-TTM from X, float64 numpy), {sec:.1f} s"}


def time_to_fit_study(max_sweeps: int = 200, reps: int = 2):
    """Wall time on the GPU until the explicit fit reaches f* - 1e-6 on the
    40^5 rank-16 workload, for plain ALS-QR-BR, the paper's ALS-QR-BRE and
    the learned extrapolation with its fallback.  f* is the explicit fit of
    the float64 oracle's plain BR after 200 sweeps (tests/golden, written by
    a script that calls only the oracle).

    Every run of k sweeps ends with a plain sweep (beta = 0): while beta is
    on, eq. (19) scales lambda by about 1 + (1 - alpha) beta, and a plain
    sweep gives the extrapolated factors their own lambda (for plain BR it
    changes nothing).  For each variant k is the smallest number of sweeps
    whose run ends at or above the target, found by bisection on
    [2, max_sweeps] (the final fit grows with k; the fit at k - 1 is reported
    as well).  The time is that of sweeps 2..k of the k-sweep run, host clock
    around the sweeps and their synchronisation, best of ``reps`` runs; it
    holds all the method does, the learned mode's acceptance fits and
    rejected sweeps included.  Sweep 1 (graph capture) and the final
    explicit fit that checks the target are not timed."""
    import torch

    import paper_2503_18759_amd as P
    from paper_2503_18759_amd import learned_beta as LB
    import synthgen as G

    with open(os.path.join(ROOT, "tests", "golden", "fstar_40pow5_r16.json")) as f:
        fstar = float(json.load(f)["fstar"])
    target = fstar - 1e-6
    prob = G.workload("fp32_40pow5_r16")
    x, dims = P.to_device(prob.X)
    weights = LB.load_weights()
    variants = {"plain_br": dict(extrapolate="off"), "paper_bre": dict(extrapolate="paper"),
                "learned": dict(extrapolate="learned", mlp_weights=weights)}

    def run(kw, k):
        sess = P.Session(x, prob.rank, prob.init, k, dims=dims, tree="restructured",
                         explicit_fit=True, closing_plain=True, **kw)
        sess.sweeps(1)
        sess.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sess.sweeps(k - 1)
        sess.sync()
        sec = time.perf_counter() - t0
        r = sess.result()
        sess.close()
        return sec, r

    out = {}
    for name, kw in variants.items():
        cache = {}

        def fit_at(k):
            if k not in cache:
                cache[k] = run(kw, k)
            return cache[k][1]["fit_explicit"]

        lo, hi = 1, max_sweeps          # fit_at(lo) < target (lo = 1: nothing run yet)
        reached = fit_at(hi) >= target
        if reached:
            while hi - lo > 1:
                mid = (lo + hi) // 2
                if fit_at(mid) >= target:
                    hi = mid
                else:
                    lo = mid
        k = hi
        sec = min([cache[k][0]] + [run(kw, k)[0] for _ in range(reps - 1)])
        r = cache[k][1]
        out[name] = {"sweeps": k, "seconds": sec, "reached": reached,
                     "fit_explicit": r["fit_explicit"],
                     "fit_explicit_at_k_minus_1": cache[k - 1][1]["fit_explicit"] if k - 1 in cache else None,
                     "beta": r["beta"], "beta_sweep": r["beta_sweep"],
                     "beta_learned": r["beta_learned"],
                     "learned_fallback_sweep": r["learned_fallback_sweep"],
                     "runs": len(cache) + reps - 1}
        print(json.dumps({"variant": name, **out[name]}), file=sys.stderr, flush=True)
    del x
    torch.cuda.empty_cache()
    res = {"workload": "order-5 dense 40^5 float32, rank 16, planted congruence 0.85, noise 1e-3; "
                       "restructured tree", "fstar": fstar, "target": target,
           "max_sweeps": max_sweeps,
           "timing": "sweeps 2..k of a k-sweep run ending with a plain sweep, host clock, best of %d"
                     % reps,
           "variants": out}
    if out["plain_br"]["reached"] and out["learned"]["reached"]:
        res["learned_over_plain_time"] = out["learned"]["seconds"] / out["plain_br"]["seconds"]
    return res


def measure_workload(name: str, K: int, W: int, tree: str = "restructured", prec: str = "fp32"):
    """Sweeps/s of one workload (graph replay of K sweeps after W warmup
    sweeps, synchronised on both sides) and the level-1 TTM's roofline from
    a second pass of the same sweeps launched kernel by kernel, every
    level-1 TTM timed with HIP events on the library's stream."""
    import torch

    import paper_2503_18759_amd as P
    import synthgen as G

    prob = G.workload(name)
    x, dims = P.to_device(prob.X)
    del prob.X
    R = prob.rank
    torch.cuda.synchronize()
    sess = P.Session(x, R, prob.init, W + K, dims=dims, tree=tree, prec=prec)
    sess.sweeps(W)
    sess.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sess.sweeps(K)
    sess.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    res = sess.result()
    sess.close()

    tsess = P.Session(x, R, prob.init, W + K, dims=dims, tree=tree, prec=prec, time_kernels=True)
    tsess.sweeps(W)
    r0 = tsess.result()
    te0 = time.perf_counter()
    tsess.sweeps(K)
    tsess.sync()
    te1 = time.perf_counter()
    r1 = tsess.result()
    tsess.close()
    del x
    torch.cuda.empty_cache()
    n_l1 = r1["l1_ttm_launches"] - r0["l1_ttm_launches"]
    avg = (r1["l1_ttm_seconds"] - r0["l1_ttm_seconds"]) / max(n_l1, 1)
    l1_bytes = r1["l1_ttm_bytes"]
    l1_flops = r1["l1_ttm_flops"]
    achieved = l1_bytes / avg / 1e9
    return {
        "dims": dims, "rank": R, "sweeps_per_s": K / elapsed, "ms_per_sweep": elapsed / K * 1e3,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "kernel": "level-1 TTM (X x_m Q_m^T, reads X once)",
                     "avg_launch_us": avg * 1e6, "launches_timed": n_l1,
                     "algorithmic_bytes_per_launch": l1_bytes},
        "ttm_pct_mfma_peak": 100.0 * l1_flops / avg / (FP32_MFMA_PEAK_TFLOPS * 1e12),
        "ttm_flops_per_sweep": res["ttm_flops"] / max(res["sweeps"], 1),
        "fit_after_steps": float(res["fit"]),
        "timing_pass_ms_per_step": (te1 - te0) / K * 1e3,
    }


def orders_4_5_study(steps: int, warmup: int):
    """Sweeps/s of the order-4 (96^4, rank 20) and order-5 (40^5, rank 16)
    workloads: ``warmup`` untimed sweeps, then ``steps`` sweeps replayed from
    the per-sweep graphs between two synchronisations (restructured tree,
    float32 TTMs, no extrapolation)."""
    import torch

    import paper_2503_18759_amd as P
    import synthgen as G

    out = {}
    for name in ("fp32_96pow4_r20", "fp32_40pow5_r16"):
        prob = G.workload(name)
        x, dims = P.to_device(prob.X)
        sess = P.Session(x, prob.rank, prob.init, warmup + steps, dims=dims, tree="restructured")
        sess.sweeps(warmup)
        sess.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sess.sweeps(steps)
        sess.sync()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        fit = float(sess.result()["fit"])
        sess.close()
        del x
        out[name] = {"dims": dims, "rank": prob.rank, "sweeps_per_s": steps / sec,
                     "ms_per_sweep": sec / steps * 1e3, "fit_after": fit}
        print(json.dumps({"workload": name, **out[name]}), file=sys.stderr, flush=True)
    return {"study": "orders_4_5", "steps": steps, "warmup": warmup,
            "timing": "graph replay of the timed sweeps, synchronised on both sides",
            "workloads": out}


def paper_shapes_study(sweeps: int = 20, real_rank: int = 16):
    """Sweep rates at the sizes of the paper's synthetic suite (Table 8, the
    rows within this build's limits) and of its real-world tensors (stand-ins
    of the same shapes; the data are not available): ``sweeps`` ALS-QR-BRE
    sweeps (the paper runs 20 iterations per method), restructured tree,
    float32 TTMs.  Sweep 1 (a standard sweep plus graph capture) is not
    timed; the rest are timed as one replay between two synchronisations."""
    import torch

    import paper_2503_18759_amd as P
    import synthgen as G

    cases = [("table8_row%d" % r, lambda r=r: G.table8_problem(r)) for r in (1, 4, 7, 8, 9, 10, 11, 12)]
    cases += [(name + "_standin", lambda name=name: G.real_shape_problem(name, real_rank))
              for name in G.REAL_SHAPES]
    out = {}
    for name, make in cases:
        t0 = time.perf_counter()
        prob = make()
        gen = time.perf_counter() - t0
        x, dims = P.to_device(prob.X)
        del prob.X
        sess = P.Session(x, prob.rank, prob.init, sweeps, dims=dims, tree="restructured",
                         extrapolate="paper", explicit_fit=True)
        sess.sweeps(1)
        sess.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sess.sweeps(sweeps - 1)
        sess.sync()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        r = sess.result()
        sess.close()
        del x
        torch.cuda.empty_cache()
        out[name] = {"dims": dims, "rank": prob.rank, "true_rank": prob.meta.get("true_rank"),
                     "ms_per_sweep": sec / (sweeps - 1) * 1e3, "fit": float(r["fit"]),
                     "fit_explicit": float(r["fit_explicit"]),
                     "beta": r["beta"], "beta_sweep": r["beta_sweep"], "host_generation_s": gen}
        print(json.dumps({"case": name, **out[name]}), file=sys.stderr, flush=True)
    return {"study": "paper_shapes", "sweeps": sweeps,
            "timing": "sweeps 2..%d replayed between two synchronisations" % sweeps,
            "cases": out}


def batched_study(count: int = 64, short: int = 10, long: int = 60, single_sweeps: int = 20):
    """Throughput of the batched sweep (every kernel covers all problems, one
    graph per sweep) on the 64-problem order-3 workload (dims U{32..160}^3,
    ranks U{4..24}, float32 TTMs, restructured tree).  Each batched call
    includes set-up, the TTM autotuning of its first sweep and graph capture,
    so the time per batch sweep is the difference of a ``long`` and a
    ``short`` run (best of two each, after an untimed call) divided by the
    extra sweeps.  For comparison the same
    problems run one after another as single-problem sessions (sweep 1 not
    timed, then ``single_sweeps`` replayed sweeps each)."""
    import torch

    import paper_2503_18759_amd as P
    import synthgen as G

    probs = G.batched_workload(count)
    xs, dims = [], []
    for p in probs:
        x, d = P.to_device(p.X)
        xs.append(x)
        dims.append(d)
    ranks = [p.rank for p in probs]
    inits = [p.init for p in probs]
    # an untimed call first (the handle's workspace is allocated once), then
    # the best of two calls at each length
    P.cp_als_qr_batched(xs, ranks, inits, short, dims=dims)
    wall = {}
    for it in (short, long):
        best = float("inf")
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.cp_als_qr_batched(xs, ranks, inits, it, dims=dims)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        wall[it] = best
        print(json.dumps({"batched_sweeps": it, "seconds": wall[it]}), file=sys.stderr, flush=True)
    per_batch_sweep = (wall[long] - wall[short]) / (long - short)
    single = 0.0
    for x, d, p in zip(xs, dims, probs):
        sess = P.Session(x, p.rank, p.init, 1 + single_sweeps, dims=d, tree="restructured")
        sess.sweeps(1)
        sess.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sess.sweeps(single_sweeps)
        sess.sync()
        torch.cuda.synchronize()
        single += (time.perf_counter() - t0) / single_sweeps
        sess.close()
    print(json.dumps({"single_sum_ms": single * 1e3}), file=sys.stderr, flush=True)
    return {"study": "batched", "problems": count, "ranks": [min(ranks), max(ranks)],
            "batch_sweep_ms": per_batch_sweep * 1e3,
            "problem_sweeps_per_s": count / per_batch_sweep,
            "one_by_one_sweep_ms": single * 1e3,
            "speedup_over_one_by_one": single / per_batch_sweep,
            "timing": "batched: (wall(%d sweeps) - wall(%d sweeps)) / %d; one by one: sum over problems "
                      "of the mean replayed sweep" % (long, short, long - short)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--tree", default="restructured", choices=["none", "standard", "restructured"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the order-4/5 sweep rates and the time-to-fit comparison")
    ap.add_argument("--study", choices=["time-to-fit", "orders-4-5", "paper-shapes", "batched"], default=None,
                    help="run a study instead of the benchmark (prints its own JSON line)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the measurement, copy a MIB-MiB device buffer once (a plain copy "
                         "kernel of known size, used to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2503_18759_amd as P
    import synthgen as G

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    P.load_library()
    if args.study == "time-to-fit":
        print(json.dumps(time_to_fit_study()), flush=True)
        return
    if args.study == "batched":
        print(json.dumps(batched_study()), flush=True)
        return
    if args.study == "paper-shapes":
        print(json.dumps(paper_shapes_study()), flush=True)
        return
    if args.study == "orders-4-5":
        print(json.dumps(orders_4_5_study(args.steps, args.warmup)), flush=True)
        return
    K, W = args.steps, args.warmup
    m = measure_workload(WORKLOAD, K, W, tree=args.tree, prec=args.prec)
    traffic = _traffic_from_profile(os.path.join(ROOT, "paper_2503_18759_amd", "csrc", "ttm.hip"))
    roof = dict(m["roofline"])
    roof["traffic"] = traffic
    out = {
        "metric": METRIC,
        "value": m["sweeps_per_s"],
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": m["ms_per_sweep"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {
            "workload": "order-3 dense 256x256x256 float32, rank 32, planted factors with "
                        "pairwise congruence 0.9, noise 1e-3 relative; ALS-QR sweeps with the "
                        f"{args.tree} dimension tree, no extrapolation; QR, solves, Y*Q0 and fit in float64",
            "dims": m["dims"], "rank": m["rank"], "tree": args.tree, "ttm_precision": args.prec,
        },
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                          "kernel", "avg_launch_us", "launches_timed",
                                          "algorithmic_bytes_per_launch")},
        "ttm_pct_mfma_peak": m["ttm_pct_mfma_peak"],
        "ttm_flops_per_sweep": m["ttm_flops_per_sweep"],
        "fit_after_steps": m["fit_after_steps"],
        "timing_pass_ms_per_step": m["timing_pass_ms_per_step"],
    }
    if not args.no_extras:
        # the order-4 and order-5 workloads (restructured tree, float32 TTMs,
        # no extrapolation), each with its own level-1 TTM roofline
        out["orders"] = {}
        for name, label in (("fp32_96pow4_r20", "order-4 96^4 rank 20"),
                            ("fp32_40pow5_r16", "order-5 40^5 rank 16")):
            e = measure_workload(name, K, W)
            out["orders"][label] = e
            print(json.dumps({"workload": label, "sweeps_per_s": e["sweeps_per_s"],
                              "frac": e["roofline"]["frac"]}), file=sys.stderr, flush=True)
        t = time_to_fit_study()
        out["time_to_fit"] = {
            "workload": t["workload"], "target": t["target"], "timing": t["timing"],
            **{n: {k: v[k] for k in ("sweeps", "seconds", "reached", "fit_explicit", "beta_learned",
                                     "learned_fallback_sweep")}
               for n, v in t["variants"].items()},
            "learned_over_plain_time": t.get("learned_over_plain_time"),
        }
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 4 * n
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(G.workload(WORKLOAD), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
