"""Plain FP64 CPU oracle for QR-based CP-ALS (CP-ALS-QR / ALS-QR-BR / ALS-QR-BRE).

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the
HIP path is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP library: it has its own tensor algebra, its own
Householder QR, its own back-substitution, its own sweep-order rule and its
own dimension-tree schedule.

Everything is float64 and written for clarity, not speed.  Library matmul is
used as a step (it is a plain definition); nothing is fused or reordered
beyond what the paper's formulas state.

Paper sections followed (arXiv 2503.18759):
  * Section 2.1 -- Kronecker / Khatri-Rao products, eq. (1); mode-n product
    (TTM) definition; multi-TTM and its unfolding form, eq. (3).
  * Section 2.3 -- least-squares subproblem eq. (6) and the Khatri-Rao P^(n).
  * Section 2.4, Algorithm 2 -- CP-ALS-QR: QR of every factor, Z_n = the
    Khatri-Rao of the R-factors, QR of Z_n, multi-TTM, V_n = Y_(n) Q0,
    triangular solve against R0^T, column normalisation, re-QR (eqs. 11-14).
  * Section 3.1 -- restructured dimension tree (update order permuted per
    sweep; schedules reconstructed from Tables 1-6).
  * Section 3.2, eq. (19) -- customised extrapolation of Q0.
  * Section 3.3, Algorithm 3 -- ALS-QR-BRE, and the activation rule for the
    extrapolation (stated after Algorithm 3 and with the synthetic-tensor
    experiments, Section 4.3).
  * Section 4.1 -- fit from intermediate quantities.

Readings where the paper is silent or ambiguous (each is listed in the
design notes of the repository):
  * QR sign convention: every QR has a non-negative diagonal in R.  Where the
    sub-column below the pivot is exactly zero the reflector is the identity
    (tau = 0), so a column c*e1 with c > 0 yields Q[:,0] = e1 exactly.
  * Q0^{k-1} in eq. (19) is the same mode's un-extrapolated Q0 of the
    previous sweep; no extrapolation happens before it exists.
  * Fit with extrapolation: <X,K> = <Vp, Vu> and ||K||^2 = ||Vu||^2, where Vp
    uses the plain Q0 and Vu the extrapolated one (exact algebra of the
    Section 4.1 formulas with P built from the plain Q0 R0).
  * Activation: checked after every sweep k >= 2; the first time
    |fit_k - fit_{k-1}| < 0.03, beta is taken from fit_k
    (> 0.95: 1/20000; (0.90, 0.95]: 1/2000; (0.70, 0.90]: 1/500;
    otherwise 1/250), fixed, and applied from sweep k+1.
  * Stopping: the "fitness >= eps" test is read as |fit_k - fit_{k-1}| < tol
    with tol = 0 meaning "run every sweep".
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "unfold", "fold", "ttm", "multi_ttm_except", "kron", "khatri_rao",
    "householder_qr", "back_substitution", "sweep_order", "beta_from_fit",
    "sum_squares", "reconstruct", "explicit_fit", "cheap_fit", "mode_update",
    "cp_als_qr", "tree_schedule", "schedule_flops", "run_tree_schedule",
    "RankDeficient", "RANK_REL", "splitmix64", "seeded_normal_factors",
]

F64 = np.float64

# Relative rank test (a library convention, not the paper's): a triangular
# factor's diagonal, or the set of column norms lambda, is rank-deficient when
# one entry is at most RANK_REL times the largest (zero included).
RANK_REL = 1e-13
# Learned extrapolation (a library feature): sweeps from the start of the
# learned beta (after sweep 2) to its first acceptance check; the gap doubles
# after every passed check.
LEARNED_FIRST_CHECK = 4


class RankDeficient(FloatingPointError):
    """Numerically dependent columns in an R factor, in R0 or in lambda."""


def _check_rank(d: np.ndarray, what: str) -> None:
    d = np.abs(np.asarray(d, F64))
    if d.size and not np.all(d > RANK_REL * d.max()):
        raise RankDeficient(what)


# ---------------------------------------------------------------------------
# Seeded N(0,1) initial factors (the "Initialize" step leaves the start open;
# this is the library's documented default when no factors are passed)
# ---------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, j: np.ndarray) -> np.ndarray:
    """Outputs j (0-based, uint64 array) of SplitMix64 seeded with ``seed``
    (Steele, Lea and Flood, OOPSLA 2014; the finaliser of Vigna's
    splitmix64.c): the state after j + 1 steps is seed + (j + 1) * golden, and
    the output is that state through the mix z ^= z >> 30, z *= 0xBF58476D1CE4E5B9,
    z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31 (all mod 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(j, np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def seeded_normal_factors(seed: int, dims: Sequence[int], rank: int) -> List[np.ndarray]:
    """Initial factors drawn from ``seed``: entry e (modes in order, each
    I_n x R column-major, e counting across modes) is the Box-Muller normal
    sqrt(-2 ln u_{2e}) cos(2 pi u_{2e+1}) with u_j = ((z_j >> 11) + 0.5) / 2^53
    and z_j = splitmix64(seed, j)."""
    total = int(sum(int(d) for d in dims)) * int(rank)
    j = np.arange(2 * total, dtype=np.uint64)
    u = ((splitmix64(seed, j) >> np.uint64(11)).astype(F64) + 0.5) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log(u[0::2])) * np.cos(2.0 * math.pi * u[1::2])
    out, off = [], 0
    for d in dims:
        n = int(d) * int(rank)
        out.append(np.reshape(z[off:off + n], (int(d), int(rank)), order="F").copy())
        off += n
    return out


# ---------------------------------------------------------------------------
# Section 2.1: tensor algebra
# ---------------------------------------------------------------------------
def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding X_(n): I_n x prod(other dims), remaining modes with the
    smallest index fastest (the convention behind eq. (3))."""
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


def fold(M: np.ndarray, n: int, dims: Sequence[int]) -> np.ndarray:
    """Inverse of :func:`unfold` for a tensor of shape ``dims``."""
    dims = list(dims)
    moved = [dims[n]] + dims[:n] + dims[n + 1:]
    return np.moveaxis(np.reshape(M, moved, order="F"), 0, n)


def ttm(X: np.ndarray, B: np.ndarray, n: int) -> np.ndarray:
    """Mode-n product Y = X x_n B with B of shape J x I_n (Section 2.1):
    Y(..., j, ...) = sum_i X(..., i, ...) B(j, i), i.e. Y_(n) = B X_(n)."""
    dims = list(X.shape)
    assert B.shape[1] == dims[n]
    dims[n] = B.shape[0]
    return fold(np.asarray(B, F64) @ unfold(X, n), n, dims)


def multi_ttm_except(X: np.ndarray, Qs: Sequence[np.ndarray], n: int) -> np.ndarray:
    """Y = X x_1 Q_1^T ... (mode n skipped) ... x_N Q_N^T, contracting the
    modes in ascending order directly from X (Algorithm 2, multi-TTM step)."""
    Y = np.asarray(X, F64)
    for k in range(X.ndim):
        if k != n:
            Y = ttm(Y, Qs[k].T, k)
    return Y


def kron(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Kronecker product with the index rule of Section 2.1:
    [A kron B]_{(K i + k), (L j + l)} = A(i, j) B(k, l) (0-based)."""
    I, J = A.shape
    K, L = B.shape
    out = np.zeros((I * K, J * L), dtype=F64)
    for i in range(I):
        for j in range(J):
            out[i * K:(i + 1) * K, j * L:(j + 1) * L] = A[i, j] * B
    return out


def khatri_rao(mats: Sequence[np.ndarray]) -> np.ndarray:
    """Column-wise Kronecker product M_1 (.) M_2 (.) ... (.) M_p: column r is
    m_1r kron m_2r kron ... kron m_pr, so the LAST factor's row index runs
    fastest (Section 2.1)."""
    R = mats[0].shape[1]
    out = np.asarray(mats[0], F64)
    for M in mats[1:]:
        assert M.shape[1] == R
        # (out (.) M)[k + K*i, r] = out[i, r] * M[k, r]
        out = (out[:, None, :] * np.asarray(M, F64)[None, :, :]).reshape(-1, R)
    return out


# ---------------------------------------------------------------------------
# Section 2.4: compact QR (Householder) and triangular solve
# ---------------------------------------------------------------------------
def householder_qr(A: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Compact QR A = Q R of an M x R matrix by Householder reflections, with
    k = min(M, R): an explicit Q (M x k, orthonormal columns) and an upper
    trapezoidal R (k x R) with a non-negative diagonal.  For M >= R this is
    the thin QR of Section 2.4; a wide factor matrix (a mode smaller than the
    rank) gets k = M reflectors.

    Reflector for column j: x = A[j:, j]; if x[1:] == 0 the reflector is the
    identity; otherwise beta = -sign(x0) ||x||, v = x / (x0 - beta) with
    v[0] = 1 and tau = (beta - x0) / beta.  Q is formed by applying the
    reflectors in reverse order to the first k columns of the identity.  The
    signs are fixed at the end so that diag(R) >= 0.
    """
    A = np.array(A, dtype=F64, copy=True)
    M, R = A.shape
    k = min(M, R)
    vs: List[np.ndarray] = []
    taus: List[float] = []
    for j in range(k):
        x = A[j:, j].copy()
        sigma = float(np.dot(x[1:], x[1:]))
        if sigma == 0.0:
            v = np.zeros_like(x)
            v[0] = 1.0
            tau = 0.0
            beta = x[0]
        else:
            norm = math.sqrt(x[0] * x[0] + sigma)
            beta = -math.copysign(norm, x[0])
            v = x / (x[0] - beta)
            v[0] = 1.0
            tau = (beta - x[0]) / beta
            # apply H = I - tau v v^T to the trailing columns
            if j + 1 < R:
                w = v @ A[j:, j + 1:]
                A[j:, j + 1:] -= tau * np.outer(v, w)
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        vs.append(v)
        taus.append(tau)
    Rm = np.triu(A[:k, :])
    Q = np.zeros((M, k), dtype=F64)
    Q[:k, :k] = np.eye(k)
    for j in reversed(range(k)):
        if taus[j] != 0.0:
            v = vs[j]
            w = v @ Q[j:, :]
            Q[j:, :] -= taus[j] * np.outer(v, w)
    d = np.where(np.diag(Rm) < 0.0, -1.0, 1.0)
    Rm = d[:, None] * Rm
    Q = Q * d[None, :]
    return Q, Rm


def back_substitution(U: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve U X = B for upper-triangular U (R x R) and B (R x m), row by row
    from the bottom."""
    U = np.asarray(U, F64)
    B = np.asarray(B, F64)
    R = U.shape[0]
    X = np.zeros_like(B)
    for i in reversed(range(R)):
        X[i] = (B[i] - U[i, i + 1:] @ X[i + 1:]) / U[i, i]
    return X


# ---------------------------------------------------------------------------
# Sweep order (Section 3.1) and the extrapolation rule (Section 3.3 / 4.3)
# ---------------------------------------------------------------------------
def sweep_order(N: int, tree: str, k: int) -> List[int]:
    """0-based mode update order of sweep k (1-based).

    "none" and "standard" update 1..N every sweep.  The restructured tree
    permutes the order (Section 3.1): for order 3 the second sweep starts
    from Y^(1,3) and the third from Y^(2,3), giving (1,2,3), (1,2,3),
    (2,1,3), (1,2,3), ...; for order N >= 4 sweep k >= 2 runs the descending
    cyclic sequence of 1..N-1 that starts at ((N-2+k-2) mod (N-1)) + 1,
    followed by N (order 4: (1234), (3214), (1324), (2134), ...).
    """
    if tree in ("none", "standard") or k == 1:
        return list(range(N))
    if tree != "restructured":
        raise ValueError(tree)
    if N == 3:
        return [0, 1, 2] if k % 2 == 0 else [1, 0, 2]
    start = ((N - 2 + k - 2) % (N - 1)) + 1          # 1-based
    seq = []
    m = start
    for _ in range(N - 1):
        seq.append(m - 1)
        m = m - 1 if m > 1 else N - 1
    return seq + [N - 1]


def beta_from_fit(fit: float) -> float:
    """Extrapolation weight chosen from the fit at activation (Section 4.3)."""
    if fit > 0.95:
        return 1.0 / 20000.0
    if fit > 0.90:
        return 1.0 / 2000.0
    if fit > 0.70:
        return 1.0 / 500.0
    return 1.0 / 250.0


# ---------------------------------------------------------------------------
# Section 4.1: fit
# ---------------------------------------------------------------------------
def sum_squares(X: np.ndarray) -> float:
    """||X||_F^2 with exactly rounded summation of the squares."""
    x = np.asarray(X, F64).ravel()
    return math.fsum((x * x).tolist()) if x.size <= 4_000_000 else \
        float(sum(math.fsum((c * c).tolist()) for c in np.array_split(x, max(1, x.size // 1_000_000))))


def reconstruct(lam: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """Dense [[lambda; A1, ..., AN]] from the mode-1 unfolding
    K_(1) = A1 diag(lambda) (A_N (.) ... (.) A_2)^T."""
    N = len(factors)
    dims = [f.shape[0] for f in factors]
    P = khatri_rao([factors[k] for k in reversed(range(1, N))])
    K1 = (factors[0] * lam[None, :]) @ P.T
    return fold(K1, 0, dims)


def explicit_fit(X: np.ndarray, lam: np.ndarray, factors: Sequence[np.ndarray]) -> float:
    """1 - ||X - K||_F / ||X||_F with K reconstructed explicitly."""
    K = reconstruct(lam, factors)
    D = np.asarray(X, F64) - K
    return 1.0 - math.sqrt(sum_squares(D)) / math.sqrt(sum_squares(X))


def cheap_fit(nx2: float, Vp: np.ndarray, Vu: np.ndarray) -> float:
    """Fit from intermediate quantities (Section 4.1):
    ||X - K||^2 = ||X||^2 - 2 <X,K> + ||K||^2 with <X,K> = <Vp, Vu> and
    ||K||^2 = ||Vu||^2."""
    res2 = nx2 - 2.0 * float(np.sum(Vp * Vu)) + float(np.sum(Vu * Vu))
    return 1.0 - math.sqrt(max(0.0, res2)) / math.sqrt(nx2)


# ---------------------------------------------------------------------------
# Algorithm 2 / Algorithm 3: one mode update
# ---------------------------------------------------------------------------
def mode_update(Yn: np.ndarray, Rfs: Sequence[np.ndarray], n: int,
                Q0prev: Optional[np.ndarray], beta: float, alpha: float):
    """One ALS-QR mode update given the leaf Y_(n).

    Z_n = R_N (.) ... (.) R_{n+1} (.) R_{n-1} (.) ... (.) R_1; Z_n = Q0 R0;
    Vp = Y_(n) Q0; with extrapolation Vu = Y_(n) Q0hat where
    Q0hat = Q0 + beta (Q0 - alpha Q0prev) (eq. 19), else Vu = Vp;
    solve Ahat R0^T = Vu; lambda = column norms; A = Ahat / lambda.
    Returns (A, lam, Q0, R0, Vp, Vu).
    """
    N = len(Rfs)
    Z = khatri_rao([Rfs[i] for i in reversed(range(N)) if i != n])
    if Z.shape[0] < Z.shape[1]:
        # fewer Khatri-Rao rows than the rank: P^(n) cannot have full column
        # rank and the subproblem (6) has no unique solution
        raise ValueError("Z_n has fewer rows than columns")
    Q0, R0 = householder_qr(Z)
    _check_rank(np.diag(R0), "R0 (dependent R factors)")
    Vp = Yn @ Q0
    if Q0prev is not None and beta != 0.0:
        Q0hat = Q0 + beta * (Q0 - alpha * Q0prev)
        Vu = Yn @ Q0hat
    else:
        Vu = Vp
    Ahat = back_substitution(R0, Vu.T).T
    lam = np.linalg.norm(Ahat, axis=0)
    _check_rank(lam, "lambda (zero column in the updated factor)")
    return Ahat / lam[None, :], lam, Q0, R0, Vp, Vu


def cp_als_qr(X: np.ndarray, rank: int, init: Sequence[np.ndarray], iters: int,
              tree: str = "none", extrap: str = "off", alpha: float = 0.1,
              delta: float = 0.03, tol: float = 0.0, fix_beta: Optional[float] = None,
              explicit_every_sweep: bool = False, explicit_final: bool = True,
              sweep_callback=None, mlp_weights=None, beta_schedule=None, seed: int = 0,
              closing_plain: bool = False) -> Dict:
    """CP-ALS-QR (Algorithm 2) / ALS-QR-BR(E) (Algorithm 3) in FP64 with
    direct multi-TTMs from X.  ``tree`` only selects the update order.

    ``extrap``: "off" (beta = 0), "paper" (eq. 19 with the activation rule)
    or "learned" (a library feature, not the paper's: after sweep 2 beta is
    the MLP output for the fits of sweeps 1-2 (``mlp_weights``, see
    mlp_oracle) and the state after sweep 2 is the checkpoint, with its
    explicit fit.  Checks come after LEARNED_FIRST_CHECK sweeps, then after
    gaps that double, and at the last sweep (and at a tolerance stop): the
    explicit fit, taken with lambda divided by 1 + (1 - alpha) beta, must
    exceed the checkpoint's, and then the state becomes the new checkpoint;
    otherwise the checkpoint is restored, beta becomes the paper's table
    value for the checkpoint's fit, and the sweeps since the checkpoint are
    run again with it, with no further checks).  The division undoes the
    growth of lambda under eq. (19): at a fixed point Q0 of the sweep equals
    Q0 of the previous one and the extrapolated R0 is (1 + beta - alpha beta)
    times the plain one.  ``closing_plain``: the last of ``iters`` sweeps
    runs with beta = 0, so lambda carries no extrapolation factor (its check
    needs no correction).
    ``fix_beta`` (test hook): apply this beta from sweep 2 onward instead of
    the rule.  ``beta_schedule`` (with "paper"): sweep k >= 2 uses
    beta_schedule[k - 1] instead of the rule.  ``sweep_callback(k, fit)``
    (instrumentation hook) is called
    after each sweep; ``explicit_final=False`` skips the final explicit fit.
    ``init=None`` draws the initial factors with seeded_normal_factors(seed).
    Raises RankDeficient when an initial factor, R0, lambda or an R_n has
    numerically dependent columns (relative test, RANK_REL).
    """
    import copy
    X = np.asarray(X, F64)
    N = X.ndim
    R = int(rank)
    nx2 = sum_squares(X)
    if init is None:
        init = seeded_normal_factors(seed, X.shape, R)
    A = [np.array(a, F64, copy=True) for a in init]
    Qs, Rfs = [], []
    for a in A:
        q, r = householder_qr(a)
        _check_rank(np.diag(r), "initial factor (dependent columns)")
        Qs.append(q)
        Rfs.append(r)
    lam = np.ones(R)
    Q0prev: List[Optional[np.ndarray]] = [None] * N
    beta, active, beta_sweep = 0.0, False, 0
    learned = extrap == "learned"
    learned_on, fallback, fallback_sweep, beta_learned = False, False, 0, 0.0
    fit_accept = 0.0
    ckpt_k = next_check = check_gap = 0
    ckpt = None
    fits: List[float] = []
    fitxs: List[float] = []
    orders: List[List[int]] = []
    Vp = Vu = None

    def sweep(order, b):
        nonlocal lam, Vp, Vu
        for n in order:
            Yn = unfold(multi_ttm_except(X, Qs, n), n)
            A[n], lam, Q0, R0, Vp, Vu = mode_update(Yn, Rfs, n, Q0prev[n], b, alpha)
            Q0prev[n] = Q0
            Qs[n], Rfs[n] = householder_qr(A[n])
            _check_rank(np.diag(Rfs[n]), "R_n (dependent columns)")
        return cheap_fit(nx2, Vp, Vu)

    for k in range(1, iters + 1):
        order = sweep_order(N, tree, k)
        orders.append(order)
        if beta_schedule is not None and extrap == "paper":
            b = float(beta_schedule[k - 1]) if k >= 2 else 0.0
        elif fix_beta is not None:
            b = fix_beta if k >= 2 else 0.0
        else:
            b = beta if (extrap in ("paper", "learned") and active) else 0.0
        closing = closing_plain and k == iters
        if closing:
            b = 0.0
        fit = sweep(order, b)
        fits.append(fit)
        if explicit_every_sweep:
            fitxs.append(explicit_fit(X, lam, A))
        if extrap == "paper" and fix_beta is None and beta_schedule is None and not active \
                and k >= 2 and abs(fit - fits[-2]) < delta:
            beta, active, beta_sweep = beta_from_fit(fit), True, k
        if learned and k == 2 and not learned_on:
            from . import mlp_oracle as M
            x = M.features(fits[0], fits[1], N, R, X.shape)
            beta = M.beta_from_output(M.forward(mlp_weights, x)[0])
            beta_learned, active, beta_sweep, learned_on = beta, True, 2, True
            fit_accept = explicit_fit(X, lam, A)
            ckpt_k, check_gap = 2, LEARNED_FIRST_CHECK
            next_check = 2 + check_gap
            ckpt = copy.deepcopy((A, Qs, Rfs, lam, Q0prev))
        tol_stop = tol > 0.0 and k >= 2 and abs(fits[-1] - fits[-2]) < tol
        if learned and learned_on and not fallback and k > 2 and \
                (k == next_check or k == iters or tol_stop):
            scale = 1.0 if closing else 1.0 / (1.0 + (1.0 - alpha) * beta_learned)
            fx = explicit_fit(X, lam * scale, A)
            if fx > fit_accept:
                fit_accept, ckpt_k = fx, k
                check_gap *= 2
                next_check = k + check_gap
                ckpt = copy.deepcopy((A, Qs, Rfs, lam, Q0prev))
            else:
                A, Qs, Rfs, lam, Q0prev = copy.deepcopy(ckpt)
                beta, beta_sweep = beta_from_fit(fit_accept), ckpt_k
                fallback, fallback_sweep = True, ckpt_k + 1
                del fits[ckpt_k:]
                del fitxs[ckpt_k:]
                for j in range(ckpt_k + 1, k + 1):
                    fits.append(sweep(orders[j - 1], 0.0 if closing_plain and j == iters else beta))
                    if explicit_every_sweep:
                        fitxs.append(explicit_fit(X, lam, A))
                tol_stop = tol > 0.0 and abs(fits[-1] - fits[-2]) < tol
        if sweep_callback is not None:
            sweep_callback(k, fits[-1])
        if tol_stop:
            break
    return {
        "factors": A, "lam": lam, "Q": Qs, "R": Rfs, "fits": np.array(fits),
        "fitx": explicit_fit(X, lam, A) if explicit_final else float("nan"),
        "fitxs": np.array(fitxs),
        "orders": orders, "beta": beta if fix_beta is None else fix_beta,
        "beta_sweep": beta_sweep, "sweeps": len(fits), "nx2": nx2,
        "beta_learned": beta_learned, "fallback_sweep": fallback_sweep, "fit_accept": fit_accept,
    }


# ---------------------------------------------------------------------------
# Section 3.1 / 3.4: dimension-tree schedules (test-only executor)
# ---------------------------------------------------------------------------
# A step is ("ttm", src, m) -- contract free mode m of Y{src} with Q_m^T,
# producing Y{src - {m}} -- or ("update", n), which consumes the leaf Y{n}.
# Free-mode sets are frozensets of 0-based modes; the full set denotes X.

def _std_tree(T: Tuple[int, ...], steps: list) -> None:
    """Standard dimension tree on Y{T} (Figure 1 / Tables 1 and 4):
    split off the largest mode; the order-3 second branch contracts the
    middle mode before the first (Table 1, cost 3 = 2 I1 I3 R^2)."""
    p = len(T)
    Tset = frozenset(T)
    if p == 2:
        m1, m2 = T
        steps += [("ttm", Tset, m2), ("update", m1), ("ttm", Tset, m1), ("update", m2)]
        return
    mp = T[-1]
    steps.append(("ttm", Tset, mp))
    _std_tree(T[:-1], steps)
    cur = Tset
    if p == 3:
        chain = [T[1], T[0]]
    else:
        chain = list(T[:-1])
    for m in chain:
        steps.append(("ttm", cur, m))
        cur = cur - {m}
    steps.append(("update", mp))


def tree_schedule(N: int, tree: str, sweeps: int) -> List[list]:
    """Per-sweep step lists for tree in {"none", "standard", "restructured"}.

    Restructured sweeps k >= 2 follow the rule reconstructed from Section 3.1
    and Tables 2 and 5: (1) finish the last two-mode intermediate of the
    previous sweep's final chain with the mode updated last; (2) walk back up
    that chain, turning each level's unused branch into a leaf by contracting
    its other free modes, most recently updated first; (3) one level-1 TTM
    on X for the most recently updated mode, then contract the other modes
    already updated this sweep (most recent first) down to a two-mode
    intermediate that yields the last two leaves (smaller mode first).
    """
    full = tuple(range(N))
    out: List[list] = []
    if tree == "none":
        for _ in range(sweeps):
            steps: list = []
            for n in range(N):
                cur = frozenset(full)
                for m in [k for k in full if k != n]:
                    steps.append(("ttm", cur, m))
                    cur = cur - {m}
                steps.append(("update", n))
            out.append(steps)
        return out
    stamp = {}           # mode -> global update counter
    counter = [0]

    def record(steps):
        for s in steps:
            if s[0] == "update":
                counter[0] += 1
                stamp[s[1]] = counter[0]

    chain: List[frozenset] = []
    for k in range(1, sweeps + 1):
        steps = []
        if tree == "standard" or k == 1:
            _std_tree(full, steps)
            record(steps)
            out.append(steps)
            # the final chain of a standard sweep starts from X
            if N == 3:
                chain = [frozenset({0, 2})]
            else:
                chain = [frozenset(range(j, N)) for j in range(1, N - 1)]
            continue
        if tree != "restructured":
            raise ValueError(tree)
        updated: List[int] = []

        def upd(n):
            steps.append(("update", n))
            counter[0] += 1
            stamp[n] = counter[0]
            updated.append(n)

        Fm = chain[-1]
        u = max(Fm, key=lambda m: stamp.get(m, 0))
        a = next(iter(Fm - {u}))
        steps.append(("ttm", Fm, u))
        upd(a)
        for j in range(len(chain) - 2, -1, -1):
            Fj = chain[j]
            c = next(iter(Fj - chain[j + 1]))
            cur = Fj
            for m in sorted(Fj - {c}, key=lambda m: -stamp.get(m, 0)):
                steps.append(("ttm", cur, m))
                cur = cur - {m}
            upd(c)
        mr = updated[-1]
        cur = frozenset(full)
        steps.append(("ttm", cur, mr))
        cur = cur - {mr}
        new_chain = [cur]
        for m in sorted([m for m in updated if m != mr], key=lambda m: -stamp[m]):
            steps.append(("ttm", cur, m))
            cur = cur - {m}
            new_chain.append(cur)
        p, q = sorted(cur)
        steps.append(("ttm", cur, q))
        upd(p)
        steps.append(("ttm", cur, p))
        upd(q)
        chain = new_chain
        out.append(steps)
    return out


def schedule_flops(sched: List[list], N: int) -> Dict[Tuple[Tuple[int, ...], int], int]:
    """Symbolic TTM cost: contracting mode m of Y{F} costs 2 |Y{F}| R, i.e.
    2 prod_{k in F} I_k R^{N-|F|+1} (Section 3.4).  Returns a map from
    (sorted free modes, power of R) to the integer coefficient."""
    poly: Dict[Tuple[Tuple[int, ...], int], int] = {}
    for steps in sched:
        for s in steps:
            if s[0] == "ttm":
                F = s[1]
                key = (tuple(sorted(F)), N - len(F) + 1)
                poly[key] = poly.get(key, 0) + 2
    return poly


def run_tree_schedule(X: np.ndarray, rank: int, init: Sequence[np.ndarray],
                      sweeps: int, tree: str) -> Dict:
    """Execute CP-ALS-QR with intermediates produced by the tree schedule,
    checking that every leaf equals the direct multi-TTM with the current
    Q's (relative 1e-12) and that every contracted Q is current."""
    X = np.asarray(X, F64)
    N = X.ndim
    full = frozenset(range(N))
    sched = tree_schedule(N, tree, sweeps)
    A = [np.array(a, F64, copy=True) for a in init]
    Qs, Rfs = [], []
    for a in A:
        q, r = householder_qr(a)
        Qs.append(q)
        Rfs.append(r)
    version = [0] * N
    cache: Dict[frozenset, Tuple[np.ndarray, Dict[int, int]]] = {full: (X, {})}
    max_leaf_err = 0.0
    fits = []
    nx2 = sum_squares(X)
    for k, steps in enumerate(sched, start=1):
        order = [s[1] for s in steps if s[0] == "update"]
        assert sorted(order) == list(range(N)), "each sweep updates each mode once"
        for s in steps:
            if s[0] == "ttm":
                _, src, m = s
                Y, vers = cache[src]
                for cm, cv in vers.items():
                    assert cv == version[cm], "stale Q contracted in cached intermediate"
                nv = dict(vers)
                nv[m] = version[m]
                cache[src - {m}] = (ttm(Y, Qs[m].T, m), nv)
            else:
                n = s[1]
                Y, vers = cache[frozenset({n})]
                for cm, cv in vers.items():
                    assert cv == version[cm], "stale Q in leaf"
                Yn = unfold(Y, n)
                Yd = unfold(multi_ttm_except(X, Qs, n), n)
                err = np.linalg.norm(Yn - Yd) / max(np.linalg.norm(Yd), 1e-300)
                max_leaf_err = max(max_leaf_err, err)
                A[n], lam, Q0, R0, Vp, Vu = mode_update(Yn, Rfs, n, None, 0.0, 0.1)
                Qs[n], Rfs[n] = householder_qr(A[n])
                version[n] += 1
        fits.append(cheap_fit(nx2, Vp, Vu))
    return {"max_leaf_err": max_leaf_err, "fits": np.array(fits), "factors": A,
            "orders": [[s[1] for s in st if s[0] == "update"] for st in sched]}
