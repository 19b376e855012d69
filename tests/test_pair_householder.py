"""The two-columns-per-step Householder scheme of the column-distributed QR
kernels (col_qr_pair, col_qr_stair_pair), emulated in float64 numpy step by
step as the kernels order it: the owner of columns (j, j+1) forms reflector
j, applies it to column j+1 and forms reflector j+1; every later column then
takes H_{j+1} H_j in the compact WY form from its two dot products with the
published columns; finished columns form their U entries from the same dots.
The result must be a Householder QR: Q^T A = R with Q = H_0 ... H_{R-1},
zeros below R's rows, U = strict upper part of V^T V (what T is built from),
and the same R as sequential Householder (the factorisation is unique with
the kernels' sign convention).
"""
import numpy as np
import pytest


def _scalars(x0, st):
    # beta = -sign(x0) ||x||, tau = (|x0| + nrm) / nrm, scale = 1 / (x0 - beta)
    if st == 0.0:
        return 0.0, x0, 0.0
    nrm = np.sqrt(x0 * x0 + st)
    ax = abs(x0)
    beta = nrm if x0 < 0 else -nrm
    return (ax + nrm) / nrm, beta, (-1.0 if x0 < 0 else 1.0) / (ax + nrm)


def _pair_qr(A0, R):
    A = A0.copy()
    m = A.shape[0]
    tau, beta, scl = np.zeros(R), np.zeros(R), np.zeros(R)
    U = np.zeros((R, R))

    def owner(j):
        j1 = j + 1
        x = A[:, j]
        y = A[:, j1] if j1 < R else np.zeros(m)
        t1, b1, s1 = _scalars(x[j], np.sum(x[j + 1:] ** 2))
        w1y = y[j] + s1 * np.sum(x[j + 1:] * y[j + 1:])
        coef = np.zeros(m)
        coef[j + 1:] = t1 * s1 * x[j + 1:]
        coef[j] = t1
        y = y - coef * w1y
        tau[j], beta[j], scl[j] = t1, b1, s1
        if j1 < R:
            A[:, j1] = y
            t2, b2, s2 = _scalars(y[j1], np.sum(y[j1 + 1:] ** 2))
            tau[j1], beta[j1], scl[j1] = t2, b2, s2
            U[j, j1] = x[j1] + s2 * np.sum(x[j1 + 1:] * y[j1 + 1:])

    owner(0)
    for j in range(0, R, 2):
        j1 = j + 1
        two = j1 < R
        x = A[:, j].copy()
        x[:j + 1] = 0
        y = A[:, j1].copy() if two else np.zeros(m)
        y[:j1 + 1] = 0
        t2, s2c = (tau[j1], scl[j1]) if two else (0.0, 0.0)
        u12 = scl[j] * U[j, j1] if two else 0.0
        for c in range(R):
            if c in (j, j1):
                continue
            a = A[:, c]
            s1 = a[j] + scl[j] * (x @ a)
            s2 = a[j1] + s2c * (y @ a)
            if c > j1:
                c1 = tau[j] * s1
                c2 = t2 * (s2 - u12 * c1)
                v1 = scl[j] * x
                v1[j] = 1.0
                v2 = s2c * y
                v2[j1] = 1.0
                A[:, c] = a - v1 * c1 - v2 * c2
            else:
                U[c, j] = s1
                if two:
                    U[c, j1] = s2
        if j + 2 < R:
            owner(j + 2)
    for r in range(R):
        U[r, r + 1:] *= scl[r]
    Rm = np.triu(A[:R, :R], 1) + np.diag(beta)
    V = np.tril(A, -1) * scl[None, :] + np.eye(m, R)
    return Rm, V, tau, U


def _sequential_r(A):
    A = A.copy()
    m, R = A.shape
    for j in range(R):
        x = A[j:, j].copy()
        t, b, s = _scalars(x[0], np.sum(x[1:] ** 2))
        v = np.concatenate([[1.0], s * x[1:]])
        A[j:, j:] -= t * np.outer(v, v @ A[j:, j:])
    return np.triu(A[:R])


@pytest.mark.parametrize("m,R", [(64, 8), (100, 32), (256, 31), (40, 17), (256, 32), (9, 3)])
def test_two_column_steps_are_a_householder_qr(m, R):
    rng = np.random.default_rng(m * 100 + R)
    A = rng.standard_normal((m, R))
    A[:, 1] += 3 * A[:, 0]                 # nearly dependent columns
    Rm, V, tau, U = _pair_qr(A, R)
    Qt = np.eye(m)
    for k in range(R):
        Qt = (np.eye(m) - tau[k] * np.outer(V[:, k], V[:, k])) @ Qt
    QA = Qt @ A
    scale = np.abs(Rm).max()
    assert np.abs(QA[:R] - Rm).max() <= 1e-13 * scale
    assert np.abs(QA[R:]).max() <= 1e-13 * scale * np.sqrt(m)
    assert np.abs(U - np.triu(V.T @ V, 1)).max() <= 1e-13
    assert np.abs(Rm - _sequential_r(A)).max() <= 1e-12 * scale
