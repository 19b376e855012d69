"""GPU MLP kernels (forward, gradient, Adam training) against the float64
reference MLP, and the learned extrapolation mode against the oracle's.

Tolerances: float32 forward within 1e-5 relative to the output scale;
float32 gradients within 2e-5 of the largest gradient entry; the learned
mode on float64 problems within 1e-10 in the fits (the MLP runs in float32
on the device, so beta carries ~1e-7 relative error, which moves the fits by
far less than that bound on these sizes).
"""
import numpy as np
import pytest

import oracle as O
from oracle import mlp_oracle as M
import synthgen as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2503_18759_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.load_library()
    return P


def _case(seed, n):
    rng = np.random.default_rng(seed)
    w = (rng.standard_normal(M.PARAMS) * 0.3).astype(np.float32)
    X = rng.standard_normal((n, M.FEATURES)).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    return w, X, t


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000])
def test_forward_matches_reference(P, n):
    w, X, _ = _case(n, n)
    y = P.mlp_forward(w, X)
    ref = M.forward(w.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(y - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [1, 16, 33, 2000])
def test_gradient_matches_reference(P, n):
    w, X, t = _case(100 + n, n)
    loss, g = P.mlp_grad(w, X, t)
    rl, rg = M.loss_and_grad(w.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert abs(loss - rl) <= 1e-5 * max(1.0, rl)
    assert np.max(np.abs(g - rg)) <= 2e-5 * max(1.0, np.max(np.abs(rg)))


def test_one_full_batch_epoch_is_one_adam_step(P):
    w, X, t = _case(7, 64)
    w1, hist = P.mlp_train(w, X, t, epochs=1, batch=64, lr=1e-3, seed=5)
    _, g = M.loss_and_grad(w.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    ref, _, _ = M.adam_step(w.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    # a first Adam step moves each weight by lr * g / (|g| + eps): entries
    # with |g| near eps (float32 rounding decides their sign) are excluded
    ok = np.abs(g) > 1e-5
    assert np.max(np.abs(w1[ok] - ref[ok])) <= 1e-6
    assert abs(hist[0] - M.loss_and_grad(w1.astype(np.float64), X.astype(np.float64),
                                         t.astype(np.float64))[0]) <= 1e-5


def test_training_fits_a_teacher(P):
    rng = np.random.default_rng(11)
    teacher = rng.standard_normal(M.PARAMS) * 0.4
    X = rng.standard_normal((1500, M.FEATURES))
    t = M.forward(teacher, X)
    w0 = (rng.standard_normal(M.PARAMS) * 0.1).astype(np.float32)
    w, hist = P.mlp_train(w0, X, t, epochs=150, batch=64, lr=3e-3, seed=1)
    assert hist[-1] < 0.1 * hist[0]
    assert hist[-1] < 0.02 * np.var(t)
    # the reported loss is the reference loss of the returned weights
    rl = M.loss_and_grad(w.astype(np.float64), X, t)[0]
    assert abs(hist[-1] - rl) <= 1e-4 * max(1.0, rl)


def _learned(P, prob, iters, w, prec, closing_plain=False):
    dt = np.float64 if prec == "fp64" else np.float32
    x, dims = P.to_device(prob.X.astype(dt))
    g = P.cp_als_qr(x, prob.rank, prob.init, iters, dims=dims, tree="restructured",
                    extrapolate="learned", prec=prec, mlp_weights=w, explicit_fit=True,
                    closing_plain=closing_plain)
    o = O.cp_als_qr(np.asarray(prob.X, dtype=dt).astype(np.float64), prob.rank, prob.init, iters,
                    tree="restructured", extrap="learned", mlp_weights=np.asarray(w, np.float64),
                    closing_plain=closing_plain)
    return g, o


def test_learned_constant_beta_fp64(P):
    prob = G.workload("small_o4", dtype=np.float64)
    w = M.constant_weights(2e-3).astype(np.float32)
    g, o = _learned(P, prob, 15, w, "fp64")
    assert o["fallback_sweep"] == g["learned_fallback_sweep"]
    assert abs(g["beta_learned"] - o["beta_learned"]) <= 1e-9
    assert np.max(np.abs(g["fits"] - o["fits"])) <= 1e-10
    for a, b in zip(g["factors"], o["factors"]):
        assert np.max(np.abs(a - b)) <= 1e-8


def test_learned_rejection_and_fallback_fp64(P):
    # collinear components (congruence 0.95), noise-free: with the largest
    # beta the lambda-corrected explicit fit at the first check (sweep 6)
    # stays below that of sweep 2 (0.9774 against 0.9787)
    prob = G.make_problem([5, 10, 9], 4, seed=77, congruence=0.95, rho=0.0, dtype=np.float64)
    w = M.constant_weights(M.BETA_MAX).astype(np.float32)
    g, o = _learned(P, prob, 10, w, "fp64")
    assert o["fallback_sweep"] == 3
    assert g["learned_fallback_sweep"] == o["fallback_sweep"]
    assert g["beta"] == o["beta"] and g["beta_sweep"] == o["beta_sweep"]
    assert np.max(np.abs(g["fits"] - o["fits"])) <= 1e-10


def test_learned_random_mlp_fp32(P):
    """A random MLP (features -> beta through the float32 kernel) on a
    float32 problem: same beta to float32 accuracy, fits to float32 parity."""
    rng = np.random.default_rng(13)
    w = (rng.standard_normal(M.PARAMS) * 0.2).astype(np.float32)
    w[M.HIDDEN * M.FEATURES + M.HIDDEN:-1] *= 0.01
    w[-1] = 0.008     # beta around 9e-3
    prob = G.make_problem([30, 26, 34], 5, seed=22, congruence=0.7, rho=0.02, dtype=np.float32)
    g, o = _learned(P, prob, 25, w, "fp32")
    assert abs(g["beta_learned"] - o["beta_learned"]) <= 1e-5 * o["beta_learned"] + 1e-9
    assert g["learned_fallback_sweep"] == o["fallback_sweep"]
    for fg, fo in zip(g["fits"], o["fits"]):
        assert abs(fg - fo) <= 1e-6 + 5e-7 / (1 - fo)
    assert abs(g["fit_explicit"] - o["fitx"]) <= 1e-6


def test_learned_large_beta_closing_plain_fp64(P):
    """A large learned beta (3) accepted on the lambda-corrected explicit fit,
    then the closing plain sweep: same decisions, fits and factors as the
    oracle."""
    prob = G.workload("small_o4", dtype=np.float64)
    w = M.constant_weights(3.0).astype(np.float32)
    g, o = _learned(P, prob, 14, w, "fp64", closing_plain=True)
    assert o["fallback_sweep"] == g["learned_fallback_sweep"]
    assert abs(g["beta_learned"] - o["beta_learned"]) <= 1e-6 * o["beta_learned"]
    assert np.max(np.abs(g["fits"] - o["fits"])) <= 1e-9
    assert abs(g["fit_explicit"] - o["fitx"]) <= 1e-9
    for a, b in zip(g["factors"], o["factors"]):
        assert np.max(np.abs(a - b)) <= 1e-7


def test_learned_late_rejection_order4_fp64(P):
    """Checks at sweeps 6 and 14 pass, the one at the last sweep (16) fails:
    the checkpoint of sweep 14 (factors, the Q0 halves of sweep 14 and the
    intermediates live across that boundary of the restructured order-4
    tree) is restored and sweeps 15-16 run again with the paper's beta."""
    prob = G.make_problem([7, 8, 5, 5], 4, seed=10, congruence=0.98, rho=0.01, dtype=np.float64)
    w = M.constant_weights(M.BETA_MAX).astype(np.float32)
    g, o = _learned(P, prob, 16, w, "fp64")
    assert o["fallback_sweep"] == 15 and o["beta_sweep"] == 14
    assert g["learned_fallback_sweep"] == 15
    assert g["beta"] == o["beta"] and g["beta_sweep"] == o["beta_sweep"]
    assert np.max(np.abs(g["fits"] - o["fits"])) <= 1e-9
    for a, b in zip(g["factors"], o["factors"]):
        assert np.max(np.abs(a - b)) <= 1e-7
