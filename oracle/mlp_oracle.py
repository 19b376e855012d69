"""Plain float64 CPU reference of the learned-extrapolation MLP.

TEST INFRASTRUCTURE ONLY (same rules as cpqr_oracle: only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it; it shares no
code with the HIP library).

The learned extrapolation is a feature of this library, not of the paper,
so nothing here has a paper citation ("parity unpinned" with respect to the
paper).  It is pinned mathematically instead: the backpropagated gradient
against central finite differences of the loss, and the Adam step against
its closed form on the first step.

Model: x (8 features) -> h = tanh(W1 x + b1) (64 units) -> y = w2 . h + b2.
Parameter vector layout: W1 (64 x 8, row-major), b1 (64), w2 (64), b2 (1).
Loss over n rows: (1/2n) sum_i (y_i - t_i)^2.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

FEATURES = 8
HIDDEN = 64
PARAMS = HIDDEN * FEATURES + 2 * HIDDEN + 1
BETA_MAX = 30.0
# The output is u = g beta / (1 + g beta) with g = 1 - alpha, alpha = 0.1 (the
# value of the training runs): eq. (19) equals
# (1 + g beta) (Q0^k + (alpha / g) u (Q0^k - Q0^{k-1})), so u is the momentum
# of the normalised update up to the constant alpha / g, and lies in [0, 1).
SHARE_G = 0.9
U_MAX = SHARE_G * BETA_MAX / (1.0 + SHARE_G * BETA_MAX)


def unpack(w: np.ndarray):
    w = np.asarray(w, np.float64).reshape(-1)
    assert w.size == PARAMS
    W1 = w[:HIDDEN * FEATURES].reshape(HIDDEN, FEATURES)
    b1 = w[HIDDEN * FEATURES:HIDDEN * FEATURES + HIDDEN]
    w2 = w[HIDDEN * FEATURES + HIDDEN:HIDDEN * FEATURES + 2 * HIDDEN]
    b2 = w[-1]
    return W1, b1, w2, b2


def pack(W1, b1, w2, b2) -> np.ndarray:
    return np.concatenate([np.asarray(W1, np.float64).reshape(-1), np.asarray(b1, np.float64),
                           np.asarray(w2, np.float64), [float(b2)]])


def forward(w, X) -> np.ndarray:
    W1, b1, w2, b2 = unpack(w)
    X = np.asarray(X, np.float64).reshape(-1, FEATURES)
    H = np.tanh(X @ W1.T + b1)
    return H @ w2 + b2


def loss_and_grad(w, X, t) -> Tuple[float, np.ndarray]:
    """Mean-squared loss and its gradient by backpropagation."""
    W1, b1, w2, b2 = unpack(w)
    X = np.asarray(X, np.float64).reshape(-1, FEATURES)
    t = np.asarray(t, np.float64).reshape(-1)
    n = X.shape[0]
    H = np.tanh(X @ W1.T + b1)
    y = H @ w2 + b2
    e = y - t
    loss = 0.5 * float(e @ e) / n
    dy = e / n
    gw2 = H.T @ dy
    gb2 = dy.sum()
    dz = np.outer(dy, w2) * (1.0 - H * H)
    gW1 = dz.T @ X
    gb1 = dz.sum(axis=0)
    return loss, pack(gW1, gb1, gw2, gb2)


def adam_step(w, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba, bias-corrected); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def features(f1: float, f2: float, N: int, R: int, dims: Sequence[int]) -> np.ndarray:
    """Inputs after sweep 2: fits of sweeps 1 and 2, order, rank, mode sizes."""
    dims = [float(d) for d in dims]
    return np.array([f1, f2, 10.0 * (f2 - f1), math.log10(max(1.0 - f2, 1e-12)) / 4.0, N / 5.0,
                     R / 16.0, math.log2(sum(dims) / len(dims)) / 8.0, R / min(dims)])


def beta_from_output(y: float) -> float:
    """u = clamp(y, 0, U_MAX); beta = u / (g (1 - u)), at most BETA_MAX."""
    u = min(max(float(y), 0.0), U_MAX)
    return min(u / (SHARE_G * (1.0 - u)), BETA_MAX)


def share_of_beta(beta: float) -> float:
    """The output u that maps to ``beta``."""
    return SHARE_G * beta / (1.0 + SHARE_G * beta)


def constant_weights(beta: float) -> np.ndarray:
    """Weights whose output is the constant share_of_beta(beta)."""
    w = np.zeros(PARAMS)
    w[-1] = share_of_beta(beta)
    return w
