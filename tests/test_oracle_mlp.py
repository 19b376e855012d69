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
    for beta in [0.0, 5e-5, 2e-3, 0.04, 3.0, 29.0]:
        w = M.constant_weights(beta)
        y = M.forward(w, np.zeros(M.FEATURES))[0]
        assert abs(M.beta_from_output(y) - beta) <= 1e-15 + 1e-12 * beta
    assert M.beta_from_output(5.0) == M.BETA_MAX == 30.0
    assert M.beta_from_output(M.U_MAX) == M.BETA_MAX


def test_output_share_is_the_momentum_of_eq19():
    """The output u maps to beta such that eq. (19), divided by its
    rescaling 1 + (1 - alpha) beta, is Q0^k + (alpha / (1 - alpha)) u
    (Q0^k - Q0^{k-1}) at alpha = 0.1."""
    rng = np.random.default_rng(3)
    q, qp = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    for u in [0.0, 0.01, 0.3, 0.8, 0.95]:
        b = M.beta_from_output(u)
        eq19 = (1 + b) * q - 0.1 * b * qp
        assert np.allclose(eq19 / (1 + 0.9 * b), q + (0.1 / 0.9) * u * (q - qp), rtol=0, atol=1e-13)
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
    """A beta far too large lowers the fit at the first check; the sweeps
    since the checkpoint (sweep 2) run again with the paper's table value
    for the checkpoint's fit, exactly as a run with that beta from sweep 3."""
    # collinear components (congruence 0.95), noise-free: with the largest
    # beta the lambda-corrected explicit fit at the first check (sweep 6)
    # stays below that of sweep 2 (0.9774 against 0.9787)
    prob = G.make_problem([5, 10, 9], 4, seed=77, congruence=0.95, rho=0.0, dtype=np.float64)
    r = O.cp_als_qr(prob.X, 4, prob.init, 10, tree="restructured", extrap="learned",
                    mlp_weights=M.constant_weights(M.BETA_MAX))
    assert r["fallback_sweep"] == 3 and r["beta_sweep"] == 2
    assert r["beta"] == O.beta_from_fit(r["fit_accept"])
    # sweeps 3..10 ran again with the paper's beta: the fit rises throughout
    assert np.all(np.diff(r["fits"][1:]) > -1e-12)
    p = O.cp_als_qr(prob.X, 4, prob.init, 10, tree="restructured", extrap="paper",
                    beta_schedule=[0.0, 0.0] + [r["beta"]] * 8)
    assert np.array_equal(p["fits"], r["fits"])


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


def test_extrapolation_scales_lambda_at_a_fixed_point():
    """Eq. (19) at a fixed point: when Q0 of the sweep equals Q0 of the
    previous sweep, the extrapolated Q0 is (1 + beta - alpha beta) Q0, so
    lambda grows by that factor while the normalised factors stay put.  This
    is the factor the learned mode divides out of lambda before it compares
    fits.  Start from the planted factors of a noise-free tensor (a fixed
    point of ALS) and apply beta from sweep 2."""
    prob = G.make_problem([8, 9, 7], 3, seed=5, congruence=0.3, rho=0.0, dtype=np.float64)
    a = O.cp_als_qr(prob.X, 3, prob.truth, 1, tree="restructured", extrap="off")
    for beta in [0.5, 3.0, 30.0]:
        b = O.cp_als_qr(prob.X, 3, prob.truth, 2, tree="restructured", extrap="paper",
                        fix_beta=beta)
        assert np.allclose(b["lam"], (1.0 + (1.0 - 0.1) * beta) * a["lam"], rtol=1e-9, atol=0)
        for u, v in zip(a["factors"], b["factors"]):
            un = u / np.linalg.norm(u, axis=0)
            vn = v / np.linalg.norm(v, axis=0)
            assert np.max(np.abs(un - vn)) <= 1e-9


def test_closing_plain_sweep_removes_the_lambda_factor():
    """With the closing plain sweep the last lambda carries no extrapolation
    factor: at a fixed point the final explicit fit is the exact one (1 for
    a noise-free tensor) although every earlier sweep applied beta."""
    prob = G.make_problem([8, 9, 7], 3, seed=5, congruence=0.3, rho=0.0, dtype=np.float64)
    r = O.cp_als_qr(prob.X, 3, prob.truth, 6, tree="restructured", extrap="paper",
                    fix_beta=10.0, closing_plain=True)
    assert r["fitx"] > 1.0 - 1e-9
    s = O.cp_als_qr(prob.X, 3, prob.truth, 6, tree="restructured", extrap="paper",
                    fix_beta=10.0)
    assert s["fitx"] < 0.0          # lambda 10 times too large


def test_learned_checks_double_their_gap():
    """Checks at sweeps 6 (gap 4), 14 (gap 8) and the last sweep: here the
    first two pass and the last fails, so the run is the learned beta up to
    sweep 14 followed by the paper's beta for the fit of sweep 14."""
    prob = G.make_problem([7, 8, 5, 5], 4, seed=10, congruence=0.98, rho=0.01, dtype=np.float64)
    r = O.cp_als_qr(prob.X, 4, prob.init, 16, tree="restructured", extrap="learned",
                    mlp_weights=M.constant_weights(M.BETA_MAX))
    assert r["fallback_sweep"] == 15 and r["beta_sweep"] == 14
    b = r["beta_learned"]
    p = O.cp_als_qr(prob.X, 4, prob.init, 16, tree="restructured", extrap="paper",
                    beta_schedule=[0.0, 0.0] + [b] * 12 + [r["beta"]] * 2)
    assert np.array_equal(p["fits"], r["fits"])
