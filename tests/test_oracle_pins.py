"""Pins for the FP64 oracle: each check compares the oracle against something
other than itself -- the definitions of Section 2.1 evaluated by brute force,
library routines for special cases, identities the paper states (eqs. 1, 3,
11, 14), the least-squares subproblem of eq. (6), and the structure of Q0
stated in Section 3.2."""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import synthgen as G


def rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- Section 2.1
def test_ttm_matches_definition_by_loops():
    r = rng(1)
    X = r.standard_normal((3, 4, 5))
    for n in range(3):
        B = r.standard_normal((2, X.shape[n]))
        Y = O.ttm(X, B, n)
        dims = list(X.shape)
        dims[n] = 2
        assert Y.shape == tuple(dims)
        for idx in itertools.product(*[range(d) for d in dims]):
            s = 0.0
            for i in range(X.shape[n]):
                src = list(idx)
                src[n] = i
                s += X[tuple(src)] * B[idx[n], i]
            assert abs(Y[idx] - s) < 1e-12


def test_unfold_column_order_by_loops():
    X = rng(2).standard_normal((3, 4, 5, 2))
    for n in range(4):
        U = O.unfold(X, n)
        others = [k for k in range(4) if k != n]
        for idx in itertools.product(*[range(d) for d in X.shape]):
            col, stride = 0, 1
            for k in others:               # smallest remaining mode fastest
                col += idx[k] * stride
                stride *= X.shape[k]
            assert U[idx[n], col] == X[idx]
        assert np.array_equal(O.fold(U, n, X.shape), X)


def test_kron_matches_numpy():
    r = rng(3)
    A, B = r.standard_normal((3, 2)), r.standard_normal((4, 5))
    assert np.array_equal(O.kron(A, B), np.kron(A, B))


def test_khatri_rao_columns_are_kroneckers():
    r = rng(4)
    mats = [r.standard_normal((d, 3)) for d in (2, 4, 3)]
    KR = O.khatri_rao(mats)
    for c in range(3):
        ref = np.kron(np.kron(mats[0][:, c], mats[1][:, c]), mats[2][:, c])
        assert np.allclose(KR[:, c], ref, rtol=0, atol=1e-14)


def test_mixed_product_identity_eq1():
    r = rng(5)
    A, B = r.standard_normal((3, 4)), r.standard_normal((5, 4))
    C, D = r.standard_normal((2, 3)), r.standard_normal((6, 5))
    lhs = np.kron(C, D) @ O.khatri_rao([A, B])
    rhs = O.khatri_rao([C @ A, D @ B])
    assert np.allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("N", [3, 4])
def test_multi_ttm_unfolding_identity_eq3(N):
    r = rng(6 + N)
    dims = [3, 4, 2, 5][:N]
    X = r.standard_normal(dims)
    Bs = [r.standard_normal((2 + k % 2, dims[k])) for k in range(N)]
    for n in range(N):
        Y = X
        for k in range(N):
            if k != n:
                Y = O.ttm(Y, Bs[k], k)
        K = None
        for k in reversed(range(N)):       # B_N kron ... kron B_1, skipping n
            if k == n:
                continue
            K = Bs[k] if K is None else np.kron(K, Bs[k])
        assert np.allclose(O.unfold(Y, n), O.unfold(X, n) @ K.T, atol=1e-12)


# ---------------------------------------------------------------- Section 2.4
@pytest.mark.parametrize("shape", [(7, 3), (40, 5), (64, 16), (5, 5), (130, 33),
                                   (3, 5), (1, 4), (6, 13), (2, 2)])
def test_householder_matches_library_qr(shape):
    """Thin QR for tall matrices; for wide ones (a mode smaller than the
    rank) the compact Q is square and R upper trapezoidal, as numpy's
    reduced QR."""
    A = rng(sum(shape)).standard_normal(shape)
    Q, R = O.householder_qr(A)
    k = min(shape)
    assert Q.shape == (shape[0], k) and R.shape == (k, shape[1])
    Ql, Rl = np.linalg.qr(A, mode="reduced")
    s = np.sign(np.diag(Rl))
    Ql, Rl = Ql * s, s[:, None] * Rl
    assert np.all(np.diag(R) >= 0)
    assert np.allclose(Q, Ql, atol=1e-12)
    assert np.allclose(R, Rl, atol=1e-12)
    assert np.linalg.norm(Q.T @ Q - np.eye(k)) < 1e-13
    assert np.allclose(Q @ R, A, atol=1e-12)
    assert np.array_equal(R, np.triu(R))


def test_householder_exact_e1_column():
    A = rng(9).standard_normal((20, 4))
    A[:, 0] = 0.0
    A[0, 0] = 2.5
    Q, R = O.householder_qr(A)
    e1 = np.zeros(20)
    e1[0] = 1.0
    assert np.array_equal(Q[:, 0], e1)
    assert np.all(Q[0, 1:] == 0.0)
    assert R[0, 0] == 2.5


def test_back_substitution_matches_library():
    r = rng(10)
    U = np.triu(r.standard_normal((6, 6))) + 4 * np.eye(6)
    B = r.standard_normal((6, 9))
    assert np.allclose(O.back_substitution(U, B),
                       scipy.linalg.solve_triangular(U, B, lower=False), atol=1e-12)


def _state(N=3, dims=(5, 6, 4), R=3, seed=11):
    r = rng(seed)
    A = [r.standard_normal((d, R)) for d in dims[:N]]
    A = [a / np.linalg.norm(a, axis=0) for a in A]
    QR = [O.householder_qr(a) for a in A]
    return A, [q for q, _ in QR], [rr for _, rr in QR]


@pytest.mark.parametrize("N,dims", [(3, (5, 6, 4)), (4, (4, 3, 5, 4))])
def test_P_equals_kron_Q_times_Q0_R0_eq11(N, dims):
    A, Qs, Rs = _state(N, dims, 3)
    for n in range(N):
        P = O.khatri_rao([A[k] for k in reversed(range(N)) if k != n])
        Z = O.khatri_rao([Rs[k] for k in reversed(range(N)) if k != n])
        Q0, R0 = O.householder_qr(Z)
        K = None
        for k in reversed(range(N)):
            if k != n:
                K = Qs[k] if K is None else np.kron(K, Qs[k])
        assert np.allclose(P, K @ Q0 @ R0, atol=1e-13)
        W = K @ Q0
        assert np.linalg.norm(W.T @ W - np.eye(3)) < 1e-13


@pytest.mark.parametrize("N,R", [(3, 4), (4, 3), (5, 3)])
def test_Q0_first_row_and_column_structure(N, R):
    """Section 3.2: Q0(1,1) = 1, the rest of row 1 and column 1 vanish; and
    column r of Q0 lives on rows whose indices are all <= r."""
    dims = [6, 5, 7, 4, 5][:N]
    A, Qs, Rs = _state(N, dims, R, seed=20 + N)
    for n in range(N):
        Z = O.khatri_rao([Rs[k] for k in reversed(range(N)) if k != n])
        Q0, R0 = O.householder_qr(Z)
        assert Q0[0, 0] == 1.0
        assert np.all(Q0[0, 1:] == 0.0) and np.all(Q0[1:, 0] == 0.0)
        idx = np.array(list(itertools.product(*[range(R)] * (N - 1))))[:, ::-1]
        rowmax = idx.max(axis=1)             # rows in Kolda order
        for c in range(R):
            assert np.all(Q0[rowmax > c, c] == 0.0)
        # R0^T R0 equals the Hadamard product of the other Gram matrices
        G_ = np.ones((R, R))
        for k in range(N):
            if k != n:
                G_ *= A[k].T @ A[k]
        assert np.allclose(R0.T @ R0, G_, atol=1e-12)


def test_mode_update_solves_least_squares_eq6():
    """With beta = 0 the update is the minimiser of ||X_(n) - Ahat P^T||."""
    r = rng(30)
    dims, R = (6, 5, 7), 3
    X = r.standard_normal(dims)
    A, Qs, Rs = _state(3, dims, R, seed=31)
    for n in range(3):
        Yn = O.unfold(O.multi_ttm_except(X, Qs, n), n)
        An, lam, Q0, R0, Vp, Vu = O.mode_update(Yn, Rs, n, None, 0.0, 0.1)
        P = O.khatri_rao([A[k] for k in reversed(range(3)) if k != n])
        sol = np.linalg.lstsq(P, O.unfold(X, n).T, rcond=None)[0].T
        assert np.allclose(An * lam, sol, atol=1e-11)
        # well-conditioned: also the normal-equation update of Algorithm 1
        Gam = np.ones((R, R))
        for k in range(3):
            if k != n:
                Gam *= A[k].T @ A[k]
        ne = np.linalg.solve(Gam.T, (O.unfold(X, n) @ P).T).T
        assert np.allclose(An * lam, ne, atol=1e-9)


def test_cheap_fit_matches_explicit_fit():
    p = G.make_problem([9, 8, 7], 3, seed=40, rho=0.05)
    res = O.cp_als_qr(p.X, 3, p.init, iters=6, explicit_every_sweep=True)
    assert np.allclose(res["fits"], res["fitxs"], atol=1e-12)


def test_fit_with_extrapolation_uses_plain_and_extrapolated_V():
    """<X,K> = <Vp,Vu>, ||K||^2 = ||Vu||^2 matches the explicit residual; the
    formula that uses Vu for both terms does not."""
    p = G.make_problem([9, 8, 7], 3, seed=41, rho=0.05)
    res = O.cp_als_qr(p.X, 3, p.init, iters=5, fix_beta=0.05, explicit_every_sweep=True)
    assert np.allclose(res["fits"][1:], res["fitxs"][1:], atol=1e-12)
    X = np.asarray(p.X, np.float64)
    A, Qs, Rs = _state(3, (9, 8, 7), 3, seed=42)
    Yn = O.unfold(O.multi_ttm_except(X, Qs, 2), 2)
    Q0prev = O.householder_qr(O.khatri_rao([Rs[1], Rs[0]]) + 0.01)[0]
    An, lam, Q0, R0, Vp, Vu = O.mode_update(Yn, Rs, 2, Q0prev, 0.05, 0.1)
    facs = [A[0], A[1], An]
    fx = O.explicit_fit(X, lam, facs)
    nx2 = O.sum_squares(X)
    assert abs(O.cheap_fit(nx2, Vp, Vu) - fx) < 1e-12
    assert abs(O.cheap_fit(nx2, Vu, Vu) - fx) > 1e-6


def test_beta_zero_is_bitwise_BR():
    p = G.make_problem([8, 9, 10], 3, seed=43, rho=0.02)
    a = O.cp_als_qr(p.X, 3, p.init, iters=6, tree="restructured", extrap="off")
    b = O.cp_als_qr(p.X, 3, p.init, iters=6, tree="restructured", fix_beta=0.0)
    for x, y in zip(a["factors"], b["factors"]):
        assert np.array_equal(x, y)
    assert np.array_equal(a["fits"], b["fits"])


def test_classical_extrapolation_keeps_first_row_and_column():
    """eq. (18) (alpha = 1) keeps Q0's first row/column; eq. (19) scales the
    (1,1) entry to 1 + beta (1 - alpha) and keeps the zeros."""
    A, Qs, Rs = _state(3, (5, 6, 4), 3, seed=44)
    Z1 = O.khatri_rao([Rs[2], Rs[1]])
    A2 = [a + 0.1 * rng(45).standard_normal(a.shape) for a in A]
    Rs2 = [O.householder_qr(a / np.linalg.norm(a, axis=0))[1] for a in A2]
    Q0a = O.householder_qr(Z1)[0]
    Q0b = O.householder_qr(O.khatri_rao([Rs2[2], Rs2[1]]))[0]
    beta = 0.3
    classical = Q0b + beta * (Q0b - Q0a)
    assert classical[0, 0] == 1.0 and np.all(classical[0, 1:] == 0) and np.all(classical[1:, 0] == 0)
    custom = Q0b + beta * (Q0b - 0.1 * Q0a)
    assert abs(custom[0, 0] - (1 + beta * 0.9)) < 1e-15
    assert np.all(custom[0, 1:] == 0) and np.all(custom[1:, 0] == 0)


@pytest.mark.parametrize("N,dims", [(3, (6, 5, 7)), (4, (4, 5, 3, 4))])
@pytest.mark.parametrize("alpha,beta", [(0.1, 0.05), (0.1, 1 / 500), (1.0, 0.3), (0.5, 0.02)])
def test_mode_update_eq19_first_column(N, dims, alpha, beta):
    """eq. (19) through the oracle's own mode update: Q0 and Q0prev both have
    e1 as their first column (Section 3.2), so the extrapolated Q0hat has
    (1 + beta (1 - alpha)) e1 there, and the first column of Vu = Y Q0hat is
    that multiple of the first column of Vp = Y Q0.  With alpha = 1 (the
    classical eq. (18)) the first column is unchanged."""
    r = rng(60 + N)
    X = r.standard_normal(dims)
    R = 3
    A, Qs, Rs = _state(N, dims, R, seed=61 + N)
    A2 = [a + 0.2 * r.standard_normal(a.shape) for a in A]
    Rs_prev = [O.householder_qr(a / np.linalg.norm(a, axis=0))[1] for a in A2]
    for n in range(N):
        Yn = O.unfold(O.multi_ttm_except(X, Qs, n), n)
        Q0prev = O.mode_update(Yn, Rs_prev, n, None, 0.0, alpha)[2]
        _, _, Q0, _, Vp, Vu = O.mode_update(Yn, Rs, n, Q0prev, beta, alpha)
        scale = 1.0 + beta * (1.0 - alpha)
        assert np.allclose(Vu[:, 0], scale * Vp[:, 0], rtol=1e-14, atol=1e-14)
        # the other columns move: Q0prev differs from Q0 beyond column 0
        assert np.abs(Vu[:, 1:] - scale * Vp[:, 1:]).max() > 1e-6
        if alpha == 1.0:
            assert np.array_equal(Vu[:, 0], Vp[:, 0]) or np.allclose(Vu[:, 0], Vp[:, 0], rtol=1e-15)


@pytest.mark.parametrize("tree", ["standard", "restructured"])
@pytest.mark.parametrize("alpha,beta", [(0.1, 0.05), (1.0, 0.2), (0.3, 0.01)])
def test_eq19_at_a_fixed_point_scales_lambda_only(tree, alpha, beta):
    """A noiseless rank-R tensor started at its exact factors is a fixed point
    of the plain update (the least-squares subproblem, eq. (6), is solved
    exactly).  There every mode's Q0 equals the previous sweep's Q0, so
    eq. (19) with Q0^{k-1} taken as the same mode's un-extrapolated Q0 of the
    previous sweep gives Q0hat = (1 + beta (1 - alpha)) Q0: the normalised
    factors stay exactly where they are and lambda carries the factor
    1 + beta (1 - alpha) after every sweep from sweep 2 on.  The cheap and the
    explicit fit both read 1 - beta (1 - alpha) (Section 4.1 with <Vp, Vu>).
    Taking Q0^{k-1} from another mode, or the previous extrapolated Q0hat,
    breaks one of these."""
    dims, R = (7, 6, 8), 3
    truth = G.gaussian_factors(rng(70), dims, R)
    unit = [a / np.linalg.norm(a, axis=0) for a in truth]
    lam_true = np.prod([np.linalg.norm(a, axis=0) for a in truth], axis=0)
    X = G.tensor_from_factors(truth)
    res = O.cp_als_qr(X, R, unit, iters=6, tree=tree, fix_beta=beta, alpha=alpha,
                      explicit_every_sweep=True)
    scale = 1.0 + beta * (1.0 - alpha)
    for a, u in zip(res["factors"], unit):
        assert np.allclose(a, u, atol=1e-12)
    assert np.allclose(res["lam"], scale * lam_true, rtol=1e-12)
    assert np.allclose(res["fits"][1:], 1.0 - beta * (1.0 - alpha), atol=1e-12)
    assert np.allclose(res["fitxs"][1:], 1.0 - beta * (1.0 - alpha), atol=1e-12)


@pytest.mark.parametrize("fit,beta", [(0.99, 1 / 20000), (0.9500001, 1 / 20000), (0.95, 1 / 2000),
                                      (0.91, 1 / 2000), (0.90, 1 / 500), (0.7000001, 1 / 500),
                                      (0.70, 1 / 250), (0.3, 1 / 250)])
def test_beta_table(fit, beta):
    assert O.beta_from_fit(fit) == beta


def test_extrapolation_activation_rule():
    p = G.make_problem([10, 11, 12], 3, seed=46, congruence=0.5, rho=0.05)
    res = O.cp_als_qr(p.X, 3, p.init, iters=25, tree="restructured", extrap="paper")
    f = res["fits"]
    k = res["beta_sweep"]
    assert k >= 2
    assert abs(f[k - 1] - f[k - 2]) < 0.03
    for j in range(2, k):
        assert abs(f[j - 1] - f[j - 2]) >= 0.03
    assert res["beta"] == O.beta_from_fit(f[k - 1])


@pytest.mark.parametrize("dims,R", [((3, 6, 7), 4), ((2, 5, 3, 4), 3), ((4, 3, 9), 5)])
def test_mode_update_least_squares_with_a_mode_below_the_rank(dims, R):
    """A mode smaller than the rank: its compact QR has min(I, R) columns, Z_n
    has prod_k min(I_k, R) rows, and the update is still the least-squares
    minimiser of eq. (6) whenever P^(n) has full column rank."""
    r = rng(33 + len(dims))
    N = len(dims)
    X = r.standard_normal(dims)
    A, Qs, Rs = _state(N, dims, R, seed=34 + N)
    assert any(q.shape[1] < R for q in Qs)
    for n in range(N):
        P = O.khatri_rao([A[k] for k in reversed(range(N)) if k != n])
        if np.prod([min(d, R) for k, d in enumerate(dims) if k != n]) < R:
            Yn = O.unfold(O.multi_ttm_except(X, Qs, n), n)
            with pytest.raises(ValueError):
                O.mode_update(Yn, Rs, n, None, 0.0, 0.1)
            continue
        Yn = O.unfold(O.multi_ttm_except(X, Qs, n), n)
        assert Yn.shape == (dims[n], int(np.prod([min(d, R) for k, d in enumerate(dims) if k != n])))
        An, lam, Q0, R0, Vp, Vu = O.mode_update(Yn, Rs, n, None, 0.0, 0.1)
        sol = np.linalg.lstsq(P, O.unfold(X, n).T, rcond=None)[0].T
        assert np.allclose(An * lam, sol, atol=1e-10)


def test_zero_padding_a_small_mode_leaves_the_update_unchanged():
    """Padding the compact Q_m (I x min(I,R)) with zero columns to I x R and
    R_m with zero rows to R x R gives Y_(n) and Z_n extra zero columns/rows;
    the QR of Z_n has the same R0 (unique with a positive diagonal), Q0 is
    zero on the extra rows, and Y_(n) Q0 is unchanged."""
    dims, R = (3, 6, 7), 5
    r = rng(36)
    X = r.standard_normal(dims)
    A, Qs, Rs = _state(3, dims, R, seed=37)
    Qp = [np.hstack([q, np.zeros((q.shape[0], R - q.shape[1]))]) for q in Qs]
    Rp = [np.vstack([rr, np.zeros((R - rr.shape[0], R))]) for rr in Rs]
    for n in range(3):
        Yn = O.unfold(O.multi_ttm_except(X, Qs, n), n)
        Ypn = O.unfold(O.multi_ttm_except(X, Qp, n), n)
        a1, l1, Q0, R0, Vp1, _ = O.mode_update(Yn, Rs, n, None, 0.0, 0.1)
        a2, l2, Q0p, R0p, Vp2, _ = O.mode_update(Ypn, Rp, n, None, 0.0, 0.1)
        assert np.allclose(R0, R0p, atol=1e-12)
        assert np.allclose(Vp1, Vp2, atol=1e-12)
        assert np.allclose(a1, a2, atol=1e-11) and np.allclose(l1, l2, rtol=1e-12)
        Zp = O.khatri_rao([Rp[k] for k in reversed(range(3)) if k != n])
        zero_rows = np.all(Zp == 0.0, axis=1)
        assert zero_rows.any() == (n != 0)
        assert np.abs(Q0p[zero_rows]).max(initial=0.0) < 1e-14


# ------------------------------------------------------- whole-method pins
def test_planted_noiseless_recovery():
    p = G.make_problem([12, 13, 14], 3, seed=50, rho=0.0)
    res = O.cp_als_qr(p.X, 3, p.init, iters=150)
    assert 1.0 - res["fitx"] < 1e-10
    # components match the planted ones up to permutation and sign
    for n in range(3):
        C = np.abs(res["factors"][n].T @ (p.truth[n] / np.linalg.norm(p.truth[n], axis=0)))
        assert np.all(C.max(axis=1) > 1 - 1e-8)
    for q in res["Q"]:
        assert np.linalg.norm(q.T @ q - np.eye(3)) < 1e-13


def test_planted_noiseless_recovery_with_a_mode_below_the_rank():
    """Rank 4 planted in 3 x 12 x 13 (generic factors: Kruskal's condition
    3 + 4 + 4 >= 2*4 + 2 holds, so the decomposition is unique)."""
    p = G.make_problem([3, 12, 13], 4, seed=53, rho=0.0)
    res = O.cp_als_qr(p.X, 4, p.init, iters=400)
    assert 1.0 - res["fitx"] < 1e-10
    assert res["Q"][0].shape == (3, 3) and res["R"][0].shape == (3, 4)
    for n in range(3):
        C = np.abs(res["factors"][n].T @ (p.truth[n] / np.linalg.norm(p.truth[n], axis=0)))
        assert np.all(C.max(axis=1) > 1 - 1e-7)


def test_noisy_fit_matches_first_order_closed_form():
    dims, R, rho = [30, 30, 30], 3, 0.05
    p = G.make_problem(dims, R, seed=51, rho=rho)
    res = O.cp_als_qr(p.X, R, p.init, iters=200, tol=1e-13)
    X = p.X
    X0 = G.tensor_from_factors(p.truth)
    rho_eff = np.linalg.norm((X - X0).ravel()) / np.linalg.norm(X.ravel())
    M = np.prod(dims)
    d = R * (sum(dims) - len(dims) + 1)
    pred = 1 - rho_eff * math.sqrt(1 - d / M)
    assert abs(res["fitx"] - pred) < 3e-4


def test_generator_congruence_and_noise_level():
    r = np.random.default_rng(52)
    B = G.congruent_factors(r, [50, 60], 5, 0.9)
    K = 0.1 * np.eye(5) + 0.9
    for b in B:
        assert np.allclose(b.T @ b, K, atol=1e-14)
    p = G.make_problem([10, 12, 9], 4, seed=53, rho=0.01)
    X0 = G.tensor_from_factors(p.truth)
    ratio = np.linalg.norm((p.X - X0).ravel()) / np.linalg.norm(X0.ravel())
    assert abs(ratio - 0.01) < 1e-14
    assert abs(G.rho_from_l1(50.0) - 1.0) < 1e-15


def test_generator_second_noise_term_and_per_mode_congruence():
    """Section 4.3: the second noise term is rho2 ||X'|| relative to the
    tensor after the first; each mode has its own congruence (Table 8)."""
    r = np.random.default_rng(54)
    B = G.congruent_factors(r, [40, 50, 30], 6, [0.5, 0.09, 0.9])
    for b, c in zip(B, [0.5, 0.09, 0.9]):
        assert np.allclose(b.T @ b, (1 - c) * np.eye(6) + c, atol=1e-14)
    with pytest.raises(ValueError):
        G.congruent_factors(r, [4, 50], 6, 0.5)
    dims, R = [11, 9, 10], 3
    p1 = G.make_problem(dims, R, seed=55, rho=0.05, congruence=[0.5, 0.09, 0.09])
    p2 = G.make_problem(dims, R, seed=55, rho=0.05, rho2=0.2, congruence=[0.5, 0.09, 0.09])
    # same draws up to the first noise term; the second is 0.2 of ||X'||
    ratio = np.linalg.norm((p2.X - p1.X).ravel()) / np.linalg.norm(p1.X.ravel())
    assert abs(ratio - 0.2) < 1e-14
    # l2 in percent maps like l1: 0.1 % -> 1 / sqrt(999)
    assert abs(G.rho_from_l1(0.1) - 1 / math.sqrt(999.0)) < 1e-16
    t = G.table8_problem(10, dims=[24, 22, 21, 20], dtype=np.float64)
    assert t.rank == 10 and t.meta["true_rank"] == 20 and t.X.shape == (24, 22, 21, 20)


# ------------------------------------------- seeded initial factors, rank test
def test_splitmix64_reference_outputs():
    """SplitMix64 seeded with 0: the first outputs of the published reference
    implementation (splitmix64.c, Vigna) are e220a8397b1dcdaf,
    6e789e6aa1b965f4, 06c45d188009454f; output j is the state after j + 1
    golden-ratio steps through the finaliser, so it is independent of how the
    outputs are requested."""
    z = O.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # counter form: output 1000 on its own equals the 1001st of a run
    run = O.splitmix64(12345, np.arange(1001, dtype=np.uint64))
    assert int(O.splitmix64(12345, np.array([1000], dtype=np.uint64))[0]) == int(run[-1])


def test_seeded_normal_factors_are_standard_normal():
    import scipy.stats
    f = O.seeded_normal_factors(7, [400, 300, 250], 64)
    assert [a.shape for a in f] == [(400, 64), (300, 64), (250, 64)]
    z = np.concatenate([a.ravel(order="F") for a in f])
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / math.sqrt(z.size) and abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    # consecutive entries are uncorrelated; another seed gives other values
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 5 / math.sqrt(z.size)
    g = O.seeded_normal_factors(8, [400], 64)[0]
    assert not np.allclose(g, f[0])
    # the counter runs across modes: mode 2 continues where mode 1 ended
    h = O.seeded_normal_factors(7, [400 + 300], 64)[0]
    assert np.array_equal(np.concatenate([f[0].ravel(order="F"), f[1].ravel(order="F")]),
                          h.ravel(order="F")[:(400 + 300) * 64])


def test_rank_test_flags_duplicate_initial_columns_and_passes_ill_conditioned_ones():
    p = G.make_problem([12, 10, 9], 3, seed=30, rho=0.01)
    init = [a.copy() for a in p.init]
    init[1][:, 2] = init[1][:, 0]
    with pytest.raises(O.RankDeficient):
        O.cp_als_qr(p.X, 3, init, 3)
    # near-collinear but resolvable columns (an independent perturbation of
    # relative size 1e-6) still run
    init = [a.copy() for a in p.init]
    init[1][:, 2] = init[1][:, 0] + 1e-6 * rng(31).standard_normal(init[1].shape[0])
    res = O.cp_als_qr(p.X, 3, init, 3)
    assert np.isfinite(res["fitx"])
