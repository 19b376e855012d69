"""Pins of the float64 reference MLP and of the oracle's learned mode.

The learned extrapolation has no basis in the paper, so these pins are
mathematical: backpropagation against central finite differences, Adam
against its closed form, and the learned mode with beta = 0 reducing exactly
to ALS-QR-BR (eq. 19 with beta = 0 is the plain update).
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import mlp_oracle as M
import synthgen as G


def _rand_case(seed=0, n=37):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(M.PARAMS) * 0.3
    X = rng.standard_normal((n, M.FEATURES))
    t = rng.standard_normal(n)
    return w, X, t


def test_gradient_matches_central_differences():
    w, X, t = _rand_case()
    _, g = M.loss_and_grad(w, X, t)
    h = 1e-6
    fd = np.empty_like(w)
    for p in range(w.size):
        wp, wm = w.copy(), w.copy()
        wp[p] += h
        wm[p] -= h
        fd[p] = (M.loss_and_grad(wp, X, t)[0] - M.loss_and_grad(wm, X, t)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_loss_is_half_mean_square_of_forward_error():
    w, X, t = _rand_case(1)
    loss, _ = M.loss_and_grad(w, X, t)
    y = np.array([M.forward(w, x)[0] for x in X])     # row by row
    assert abs(loss - 0.5 * np.mean((y - t) ** 2)) <= 1e-14 * max(1.0, loss)


def test_adam_first_two_steps_closed_form():
    rng = np.random.default_rng(3)
    w0 = rng.standard_normal(5)
    g1, g2 = rng.standard_normal(5), rng.standard_normal(5)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    m, v = np.zeros(5), np.zeros(5)
    w1, m, v = M.adam_step(w0, g1, m, v, 1, lr, b1, b2, eps)
    # first step: mhat = g, vhat = g^2 -> w0 - lr g / (|g| + eps)
    assert np.allclose(w1, w0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    w2, m, v = M.adam_step(w1, g2, m, v, 2, lr, b1, b2, eps)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    assert np.allclose(w2, w1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)


def test_constant_weights_round_trip():
    for beta in [0.0, 5e-5, 2e-3, 0.04]:
        w = M.constant_weights(beta)
        y = M.forward(w, np.zeros(M.FEATURES))[0]
        assert abs(M.beta_from_output(y) - beta) <= 1e-15 + 1e-12 * beta
    assert M.beta_from_output(5.0) == M.BETA_MAX
    assert M.beta_from_output(-20.0) == 0.0


def test_features_by_hand():
    x = M.features(0.5, 0.75, 3, 8, [16, 32, 64])
    expect = [0.5, 0.75, 2.5, math.log10(0.25) / 4, 0.6, 0.5, math.log2(112 / 3) / 8, 0.5]
    assert np.allclose(x, expect, rtol=0, atol=1e-15)


def test_learned_beta_zero_equals_plain_br():
    prob = G.make_problem([9, 8, 10], 3, seed=41, congruence=0.5, rho=0.05, dtype=np.float64)
    a = O.cp_als_qr(prob.X, 3, prob.init, 8, tree="restructured", extrap="off")
    b = O.cp_als_qr(prob.X, 3, prob.init, 8, tree="restructured", extrap="learned",
                    mlp_weights=M.constant_weights(0.0))
    assert b["fallback_sweep"] == 0 and b["beta_learned"] == 0.0
    assert np.array_equal(a["fits"], b["fits"])
    for u, v in zip(a["factors"], b["factors"]):
        assert np.array_equal(u, v)


def test_learned_rejection_falls_back_to_paper_beta():
    """A beta far too large lowers the fit; the sweep is redone with the
    paper's table value for the previous fit, after which the fit keeps
    rising."""
    prob = G.make_problem([10, 9, 11], 3, seed=42, congruence=0.8, rho=0.01, dtype=np.float64)
    r = O.cp_als_qr(prob.X, 3, prob.init, 10, tree="restructured", extrap="learned",
                    mlp_weights=M.constant_weights(M.BETA_MAX))
    assert r["fallback_sweep"] >= 3
    k = r["fallback_sweep"]
    assert r["beta"] == O.beta_from_fit(r["fits"][k - 2])
    assert np.all(np.diff(r["fits"][k - 2:]) > -1e-12)


def test_zero_schedule_equals_plain_br():
    """beta_schedule of zeros is exactly ALS-QR-BR (eq. 19 with beta = 0)."""
    prob = G.make_problem([9, 8, 10], 3, seed=43, congruence=0.5, rho=0.05, dtype=np.float64)
    a = O.cp_als_qr(prob.X, 3, prob.init, 7, tree="restructured", extrap="off")
    b = O.cp_als_qr(prob.X, 3, prob.init, 7, tree="restructured", extrap="paper",
                    beta_schedule=[0.0] * 7)
    assert np.array_equal(a["fits"], b["fits"])


def test_committed_weights_load_and_give_a_beta():
    """The trained weights shipped with the package have the documented
    layout and map a 40^5 rank-16 start to a beta inside the clamp."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2503_18759_amd", "data", "learned_beta_mlp.json")
    with open(path) as f:
        doc = json.load(f)
    w = np.asarray(doc["weights"], dtype=np.float64)
    assert w.size == M.PARAMS and np.all(np.isfinite(w))
    x = M.features(0.8553, 0.8961, 5, 16, [40] * 5)
    b = M.beta_from_output(M.forward(w, x)[0])
    assert 0.0 <= b <= M.BETA_MAX
