"""Training of the learned extrapolation MLP (a feature of this library, not
part of the paper: the paper picks beta from a fixed table of fit levels,
Section 4.3).

Training set: 2,000 seeded problems (seeds 10000..11999), order 3 for even
and 4 for odd indices, mode sizes U{24..64}, rank U{4..16}, planted
congruence U[0, 0.9], noise 10^U[-4, -1.5] (relative).  For every problem
the GPU runs HORIZON float32 sweeps of ALS-QR-BRE for each beta of GRID with
the schedule: beta = 0 in sweeps 1-2, the candidate beta in sweeps 3 to
HORIZON-2, and beta = 0 in the last two sweeps (one batched launch sequence
per group of problems).  The final plain sweeps matter: at a fixed point eq.
(19) scales the update by 1 + (1 - alpha) beta, which the weights lambda
carry, so a fit read while beta is still on mixes the acceleration with that
offset; two plain sweeps remove it.  The label is the beta whose explicit fit
after HORIZON sweeps is highest (ties: the smallest beta).  The features are those of the
learned mode (include/cpqr.h), computed from the fits of sweeps 1 and 2 of
the beta = 0 run.  The MLP (8 -> 64 tanh -> 1) regresses the momentum share
u = g beta / (1 + g beta), g = 1 - alpha = 0.9 (include/cpqr.h): eq. (19)
equals (1 + g beta) (Q0^k + (alpha / g) u (Q0^k - Q0^{k-1})), so u is the
momentum of the normalised update up to a constant, and where problems with
alike features have different labels the regression averages momenta, not
orders of magnitude of beta.  It is trained with the library's Adam kernels.
The labelled set (features, labels and the explicit fit of every grid value)
is written beside the weights.

Run on a GPU host from the repository root:
    python -m paper_2503_18759_amd.learned_beta [--count 2000]
It writes paper_2503_18759_amd/data/learned_beta_mlp.json.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time
from typing import List, Sequence

import numpy as np

from . import cpqr as C

# Beta enters eq. (19) as (1 + beta) Q0^k - alpha beta Q0^{k-1}: the part that
# moves the factors is the difference term, alpha beta (Q0^k - Q0^{k-1})
# against (1 + (1 - alpha) beta) Q0^k, whose weight grows towards
# alpha / (1 - alpha) only for beta of order one and more, so the grid
# reaches well past the paper's table (at most 1/250).
GRID = [0.0, 1e-3, 1e-2, 5e-2, 0.1, 0.3, 1.0, 3.0, 10.0, 30.0]
HORIZON = 30
BASE_SEED = 10000
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "learned_beta_mlp.json")
DATASET_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "learned_beta_dataset.npz")


SHARE_G = 0.9
BETA_MAX = 30.0


def share_of_beta(beta: float) -> float:
    """The network output u for ``beta`` (the library maps u back)."""
    return SHARE_G * beta / (1.0 + SHARE_G * beta)


def features(f1: float, f2: float, N: int, R: int, dims: Sequence[int]) -> np.ndarray:
    """Learned-mode inputs (the same formula the library evaluates after sweep 2)."""
    d = [float(v) for v in dims]
    return np.array([f1, f2, 10.0 * (f2 - f1), math.log10(max(1.0 - f2, 1e-12)) / 4.0, N / 5.0,
                     R / 16.0, math.log2(sum(d) / len(d)) / 8.0, R / min(d)], dtype=np.float32)


def schedule(beta: float) -> List[float]:
    """Per-sweep beta (entry k is the beta of sweep k + 1)."""
    return [0.0, 0.0] + [beta] * (HORIZON - 4) + [0.0, 0.0]


def problem(t: int):
    import synthgen as G
    seed = BASE_SEED + t
    rng = np.random.default_rng(seed)
    N = 3 if t % 2 == 0 else 4
    dims = [int(v) for v in rng.integers(24, 65, size=N)]
    R = int(rng.integers(4, 17))
    c = float(rng.uniform(0.0, 0.9))
    rho = float(10.0 ** rng.uniform(-4.0, -1.5))
    return G.make_problem(dims, R, seed=seed, congruence=c, rho=rho, dtype=np.float32,
                          name=f"train{t}")


def label_group(probs) -> List[tuple]:
    """(features, best beta, explicit fits per grid value) for problems of one order."""
    xs, dims, ranks, inits, scheds = [], [], [], [], []
    for p in probs:
        x, d = C.to_device(p.X)
        for b in GRID:
            xs.append(x)
            dims.append(d)
            ranks.append(p.rank)
            inits.append(p.init)
            scheds.append(schedule(b))
    res = C.cp_als_qr_batched(xs, ranks, inits, HORIZON, dims=dims, extrapolate="paper",
                              beta_schedules=scheds, explicit_fit=True)
    out = []
    G = len(GRID)
    for i, p in enumerate(probs):
        rs = res[i * G:(i + 1) * G]
        fx = np.array([r["fit_explicit"] for r in rs])
        best = int(np.argmax(fx))
        beta = GRID[best]
        f = features(rs[0]["fits"][0], rs[0]["fits"][1], p.X.ndim, p.rank, p.X.shape)
        out.append((f, beta, fx))
    return out


def build_dataset(count: int, group: int = 5, log=print):
    X, y, fits = [], [], []
    t0 = time.time()
    for order_parity in (0, 1):
        ids = [t for t in range(count) if t % 2 == order_parity]
        for g0 in range(0, len(ids), group):
            probs = [problem(t) for t in ids[g0:g0 + group]]
            for f, beta, fx in label_group(probs):
                X.append(f)
                y.append(share_of_beta(beta))
                fits.append(fx)
            log(f"labelled {len(y)}/{count} ({time.time() - t0:.0f} s)")
    return np.array(X, np.float32), np.array(y, np.float32), np.array(fits)


def train(X, y, *, epochs: int = 300, lr: float = 3e-3, seed: int = 0, val_frac: float = 0.1):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(y))
    nv = max(1, int(len(y) * val_frac))
    va, tr = perm[:nv], perm[nv:]
    w0 = np.concatenate([rng.standard_normal(C.MLP_HIDDEN * C.MLP_FEATURES) * 0.3,
                         np.zeros(C.MLP_HIDDEN), rng.standard_normal(C.MLP_HIDDEN) * 0.1,
                         [float(np.mean(y[tr]))]]).astype(np.float32)
    w, hist = C.mlp_train(w0, X[tr], y[tr], epochs=epochs, batch=64, lr=lr, seed=seed)
    val_loss, _ = C.mlp_grad(w, X[va], y[va])
    const_loss = 0.5 * float(np.mean((y[va] - np.mean(y[tr])) ** 2))
    return w, hist, val_loss, const_loss


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--out", default=WEIGHTS_PATH)
    ap.add_argument("--dataset", default=DATASET_PATH,
                    help="labelled set: read if it exists and --relabel is not given, else written")
    ap.add_argument("--relabel", action="store_true")
    args = ap.parse_args()
    C.load_library()
    if os.path.exists(args.dataset) and not args.relabel:
        d = np.load(args.dataset)
        X, betas, fits = d["features"], d["labels"], d["fits"]
        if len(betas) != args.count or list(d["grid"]) != GRID:
            raise SystemExit(f"{args.dataset} holds another set: run with --relabel")
        y = np.array([share_of_beta(b) for b in betas], np.float32)
        print(f"read {len(y)} labelled problems from {args.dataset}", flush=True)
    else:
        X, y, fits = build_dataset(args.count, log=lambda m: print(m, flush=True))
        betas = np.array([GRID[int(np.argmax(f))] for f in fits])
        os.makedirs(os.path.dirname(args.dataset), exist_ok=True)
        np.savez_compressed(args.dataset, features=X, labels=betas, fits=fits, grid=np.array(GRID))
        print("wrote", args.dataset, flush=True)
    w, hist, val_loss, const_loss = train(X, y, epochs=args.epochs)
    print(f"train loss {hist[0]:.4f} -> {hist[-1]:.4f}; validation {val_loss:.4f} "
          f"(constant predictor {const_loss:.4f})", flush=True)
    labels = {f"{b:g}": int(np.sum(betas == b)) for b in GRID}
    doc = {
        "what": "weights of the learned extrapolation MLP (8 -> 64 tanh -> 1, output the momentum "
                "share u = 0.9 beta / (1 + 0.9 beta))",
        "layout": "W1 (64 x 8 row-major), b1 (64), w2 (64), b2 (1)",
        "training_set": {"count": args.count, "seeds": [BASE_SEED, BASE_SEED + args.count - 1],
                         "orders": "3 (even index), 4 (odd index)", "dims": "U{24..64}",
                         "rank": "U{4..16}", "congruence": "U[0, 0.9]", "noise": "10^U[-4, -1.5]",
                         "grid": GRID, "horizon_sweeps": HORIZON, "label_counts": labels},
        "train_loss_first_last": [float(hist[0]), float(hist[-1])],
        "validation_loss": val_loss, "constant_predictor_validation_loss": const_loss,
        "epochs": args.epochs, "script": "python -m paper_2503_18759_amd.learned_beta",
        "weights": [float(v) for v in w],
    }
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", args.out, flush=True)


def load_weights(path: str = WEIGHTS_PATH) -> np.ndarray:
    with open(path) as f:
        return np.asarray(json.load(f)["weights"], dtype=np.float32)


if __name__ == "__main__":
    main()
