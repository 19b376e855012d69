"""The nested QR of the Khatri-Rao product Z_n (orders 4 and up), emulated in
float64 numpy in the order the library runs it: with the remaining modes
m_1 < ... < m_{N-1} (m_1 fastest in the Kolda row order),
W_1 = R_{m_2} (.) R_{m_1} = Q_1 T_1 and W_k = R_{m_{k+1}} (.) T_{k-1} = Q_k T_k,
each a QR of R^2 rows with a non-negative diagonal; then
Z_n = (I (x) Q_1)(I (x) Q_2) ... Q_L T_L.  Row r + R^2 t of Q0 is
Q_1[r, :] B_2(t_0) ... B_L(t_{L-2}), B_k(d) the rows dR .. dR + R - 1 of Q_k
(the formula of the kernel that writes Q0).  The result must be the QR of the
explicit Z_n: Q0 with orthonormal columns, Q0 R0 = Z_n, and, R0's diagonal
being non-negative, the same Q0 and R0 as numpy's QR after the sign fix.
Upper trapezoidal factors (modes below the rank) are covered too.
"""
import numpy as np
import pytest


def _krp(A, B):
    # columns a_c (x) b_c: B's index fastest
    return np.einsum("ic,jc->ijc", A, B).reshape(A.shape[0] * B.shape[0], A.shape[1])


def _qr_pos(W):
    Q, T = np.linalg.qr(W)
    d = np.where(np.diag(T) < 0, -1.0, 1.0)
    return Q * d, T * d[:, None]


def _nested(Rs, n):
    N, R = len(Rs), Rs[0].shape[0]
    m = [k for k in range(N) if k != n]
    L = N - 2
    Qs, T = [], None
    for k in range(L):
        W = _krp(Rs[m[1]], Rs[m[0]]) if k == 0 else _krp(Rs[m[k + 1]], T)
        Q, T = _qr_pos(W)
        Qs.append(Q)
    M = R ** (N - 1)
    Q0 = np.zeros((M, R))
    for t in range(R ** (L - 1)):
        digits = [(t // R ** i) % R for i in range(L - 1)]
        P = np.eye(R)
        for k in range(1, L):
            d = digits[k - 1]
            P = P @ Qs[k][d * R:(d + 1) * R]
        Q0[t * R * R:(t + 1) * R * R] = Qs[0] @ P
    return Q0, T


def _z(Rs, n):
    m = [k for k in range(len(Rs)) if k != n]
    Z = Rs[m[0]]
    for k in m[1:]:
        Z = _krp(Rs[k], Z)
    return Z


@pytest.mark.parametrize("N,R,seed", [(4, 3, 1), (4, 5, 2), (5, 3, 3), (5, 4, 4), (6, 2, 5), (6, 3, 6)])
def test_nested_qr_equals_the_qr_of_z(N, R, seed):
    rng = np.random.default_rng(seed)
    Rs = [np.triu(rng.standard_normal((R, R))) + 2.0 * np.eye(R) for _ in range(N)]
    for n in range(N):
        Z = _z(Rs, n)
        Q0, R0 = _nested(Rs, n)
        assert np.allclose(Q0.T @ Q0, np.eye(R), atol=1e-13)
        assert np.allclose(Q0 @ R0, Z, atol=1e-12 * np.abs(Z).max())
        assert np.all(np.diag(R0) >= 0) and np.allclose(np.tril(R0, -1), 0.0)
        Qd, Rd = _qr_pos(Z)
        assert np.allclose(Q0, Qd, atol=1e-12)
        assert np.allclose(R0, Rd, atol=1e-12 * np.abs(Rd).max())


def test_nested_qr_with_trapezoidal_factors():
    """Modes smaller than the rank: R factors with zero rows beyond I_k."""
    rng = np.random.default_rng(7)
    N, R, dims = 5, 4, [3, 5, 2, 6, 4]
    Rs = []
    for I in dims:
        Rk = np.triu(rng.standard_normal((R, R))) + 2.0 * np.eye(R)
        Rk[min(I, R):] = 0.0
        Rs.append(Rk)
    for n in range(N):
        Z = _z(Rs, n)
        if np.linalg.matrix_rank(Z) < R:
            continue
        Q0, R0 = _nested(Rs, n)
        Qd, Rd = _qr_pos(Z)
        assert np.allclose(Q0 @ R0, Z, atol=1e-12 * np.abs(Z).max())
        assert np.allclose(Q0, Qd, atol=1e-11)


def test_a_wrong_nesting_order_fails():
    """The Kronecker order matters: nesting the slow factor as if it were
    the fast one does not reproduce Z_n (so the test above can fail)."""
    rng = np.random.default_rng(8)
    N, R = 4, 3
    Rs = [np.triu(rng.standard_normal((R, R))) + 2.0 * np.eye(R) for _ in range(N)]
    Z = _z(Rs, 0)
    m = [1, 2, 3]
    Q1, T1 = _qr_pos(_krp(Rs[m[0]], Rs[m[1]]))   # fast and slow swapped
    Q2, T2 = _qr_pos(_krp(Rs[m[2]], T1))
    Q0 = np.zeros((R ** 3, R))
    for t in range(R):
        Q0[t * R * R:(t + 1) * R * R] = Q1 @ Q2[t * R:(t + 1) * R]
    assert not np.allclose(Q0 @ T2, Z, atol=1e-8)
