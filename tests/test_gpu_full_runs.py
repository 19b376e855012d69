"""Full-length GPU parity on the benchmark workloads against stored float64
oracle runs (tests/golden/full_runs, written by make_full_runs.py, which calls
only the oracle), at each workload's own sweep count.

Errors are stated per result:
  * fit: the explicit fit 1 - ||X - K|| / ||X|| at the end (float64
    accumulation on both sides): within 1e-6 for float32 TTMs and 1e-4 for
    bf16x3;
  * per-sweep fit (Section 4.1 formula): within 1e-6 + 5e-7 / (1 - fit) for
    float32 (the formula subtracts ||Vu||^2, accurate to ~1e-7 relative from
    float32 leaves, from ||X||^2) and 1e-4 + 5e-5 / (1 - fit) for bf16x3 at
    every sweep where the oracle's run has settled (its fit moved less than
    1e-6 over the five sweeps before).  While the fit still climbs through a
    flat stretch, ALS amplifies the float32 rounding of the TTMs and the two
    trajectories may part by up to ~1e-4 before they meet again at the same
    fit; there (and for the final fit of a run that has not settled by its
    last sweep) only a sanity bound of 1e-3 is asserted, and the largest
    difference is reported;  * factor congruence: min over modes and columns of |cos(a_gpu, a_oracle)|;
  * lambda: largest relative difference;
  * orthonormality of the float32 Q_n the TTMs use: ||Q_n^T Q_n - I||_F.
With CPQR_PARITY_REPORT=<path> every test appends its measured errors to that
file as one JSON line (the per-result error table).
"""
import json
import os

import numpy as np
import pytest

import synthgen as G

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_runs")


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2503_18759_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.load_library()
    return P


def _golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"golden run {name} not written (python tests/golden/make_full_runs.py {name})")
    return dict(np.load(path))


def errors(g, fits_o, fitx_o, lam_o, facs_o):
    """Per-result errors of a GPU run against an oracle run."""
    cos = [np.abs(np.sum(a * b, axis=0) / (np.linalg.norm(a, axis=0) * np.linalg.norm(b, axis=0)))
           for a, b in zip(g["factors"], facs_o)]
    orth = []
    for q in g["Q"]:
        k = min(q.shape)
        qq = q[:, :k]
        orth.append(float(np.linalg.norm(qq.T @ qq - np.eye(k))))
    n = min(len(g["fits"]), len(fits_o))
    return {
        "settled": bool(_settled(fits_o[:n])[-1]),
        "d_fit_explicit": float(abs(g["fit_explicit"] - fitx_o)),
        "d_fit_sweep_max": float(np.max(np.abs(g["fits"][:n] - fits_o[:n]))),
        "fit_explicit": float(g["fit_explicit"]), "fit_explicit_oracle": float(fitx_o),
        "congruence_min": float(min(c.min() for c in cos)),
        "lambda_rel_max": float(np.max(np.abs(g["lam"] - lam_o) / np.abs(lam_o))),
        "orth_max": float(max(orth)),
        "sweeps": int(g["sweeps"]),
    }


def _report(name, prec, tree, err):
    path = os.environ.get("CPQR_PARITY_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"run": name, "prec": prec, "tree": tree, **err}) + "\n")


def _settled(fits_o):
    """Per sweep: has the oracle's fit moved less than 1e-6 over the five
    sweeps before (a settled run, where float32 rounding is not amplified)."""
    f = np.asarray(fits_o)
    return np.array([k >= 5 and np.max(np.abs(np.diff(f[k - 5:k + 1]))) < 1e-6 for k in range(len(f))])


def _check(err, g, fits_o, prec, cong_min, strict_final=False):
    """strict_final: hold the final explicit fit to the float32 / bf16x3
    target even though the run has not settled (the 256^3 rank-32 runs are
    still in their flat stretch at sweep 100; the target is stated for that
    workload's 100 sweeps)."""
    tol = 1e-6 if prec == "fp32" else 1e-4
    n = min(len(g["fits"]), len(fits_o))
    settled = _settled(fits_o[:n])
    assert err["d_fit_explicit"] <= (tol if (settled[-1] or strict_final) else max(1e-3, tol)), err
    for k, (fg, fo) in enumerate(zip(g["fits"][:n], fits_o[:n])):
        bound = tol + (tol / 2) / max(1e-12, 1 - fo) if settled[k] else max(1e-3, tol)
        assert abs(fg - fo) <= bound, (k, fg, fo)
    assert err["congruence_min"] >= cong_min, err
    assert err["orth_max"] <= (2e-6 if prec == "fp32" else 2e-6), err


# 256^3 rank 32 (congruence 0.9), 100 sweeps: both trees, both TTM precisions.
@pytest.mark.parametrize("tree", ["restructured", "standard"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_256cube_r32_100_sweeps(P, tree, prec):
    name = f"256cube_r32_{tree}"
    o = _golden(name)
    prob = G.workload("fp32_256cube_r32")
    x, dims = P.to_device(prob.X)
    g = P.cp_als_qr(x, 32, prob.init, 100, dims=dims, tree=tree, prec=prec, explicit_fit=True)
    assert g["orders"] == o["orders"].tolist()
    err = errors(g, o["fits"], float(o["fitx"]), o["lam"], [o[f"A{n}"] for n in range(3)])
    _report(name, prec, tree, err)
    _check(err, g, o["fits"], prec, 1 - 1e-3 if prec == "fp32" else 0.9, strict_final=True)


# 96^4 rank 20 with the paper's extrapolation, 200 sweeps.
def test_96pow4_r20_paper_200_sweeps(P):
    o = _golden("96pow4_r20_paper")
    prob = G.workload("fp32_96pow4_r20")
    x, dims = P.to_device(prob.X)
    g = P.cp_als_qr(x, 20, prob.init, 200, dims=dims, tree="restructured", extrapolate="paper",
                    explicit_fit=True)
    assert g["orders"] == o["orders"].tolist()
    assert g["beta_sweep"] == int(o["beta_sweep"]) and g["beta"] == float(o["beta"])
    err = errors(g, o["fits"], float(o["fitx"]), o["lam"], [o[f"A{n}"] for n in range(4)])
    _report("96pow4_r20_paper", "fp32", "restructured", err)
    _check(err, g, o["fits"], "fp32", 1 - 1e-4)


# 40^5 rank 16, 200 sweeps, without and with the paper's extrapolation.
@pytest.mark.parametrize("extrap", ["plain", "paper"])
def test_40pow5_r16_200_sweeps(P, extrap):
    name = f"40pow5_r16_{extrap}"
    o = _golden(name)
    prob = G.workload("fp32_40pow5_r16")
    x, dims = P.to_device(prob.X)
    g = P.cp_als_qr(x, 16, prob.init, 200, dims=dims, tree="restructured",
                    extrapolate="off" if extrap == "plain" else "paper", explicit_fit=True)
    assert g["orders"] == o["orders"].tolist()
    if extrap == "paper":
        assert g["beta_sweep"] == int(o["beta_sweep"]) and g["beta"] == float(o["beta"])
    err = errors(g, o["fits"], float(o["fitx"]), o["lam"], [o[f"A{n}"] for n in range(5)])
    _report(name, "fp32", "restructured", err)
    _check(err, g, o["fits"], "fp32", 1 - 1e-4)


# The 64-problem batch, 50 sweeps, every problem.
def test_batch64_50_sweeps(P):
    o = _golden("batch64")
    probs = G.batched_workload(64)
    xs, dims = [], []
    for p in probs:
        x, d = P.to_device(p.X)
        xs.append(x)
        dims.append(d)
    res = P.cp_als_qr_batched(xs, [p.rank for p in probs], [p.init for p in probs], 50, dims=dims,
                              explicit_fit=True)
    worst = {}
    for t, (g, p) in enumerate(zip(res, probs)):
        assert g["orders"] == o[f"p{t}_orders"].tolist()
        err = errors(g, o[f"p{t}_fits"], float(o[f"p{t}_fitx"]), o[f"p{t}_lam"],
                     [o[f"p{t}_A{n}"].astype(np.float64) for n in range(3)])
        _check(err, g, o[f"p{t}_fits"], "fp32", 1 - 1e-3)
        worst["unsettled"] = worst.get("unsettled", 0) + (0 if err["settled"] else 1)
        for k, v in err.items():
            if k.startswith("d_") or k in ("lambda_rel_max", "orth_max"):
                worst[k] = max(worst.get(k, 0.0), v)
            elif k == "congruence_min":
                worst[k] = min(worst.get(k, 1.0), v)
    _report("batch64", "fp32", "restructured", dict(worst, problems=len(probs)))
