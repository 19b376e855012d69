"""Seeded synthetic inputs for CP-ALS-QR, shared by the FP64 oracle and the GPU path.

This module only draws random numbers and assembles test tensors; it holds none
of the decomposition's arithmetic.  Every random draw that the method consumes
(the initial factor matrices) is made here and handed to both sides.

Conventions
-----------
* Tensors are numpy arrays in Fortran order, so the flat buffer
  ``X.ravel(order="F")`` has mode 1 fastest (the Kolda unfolding convention
  used throughout the paper, Section 2.1).
* Generator: ``numpy.random.default_rng(seed)`` (PCG64), FP64 draws.  Draw
  order: the factor matrices in mode order, then the noise tensor.  Initial
  factors come from ``default_rng(seed + 1_000_000)``.
* Congruence-c factors follow the synthetic-tensor recipe of Section 4.3:
  ``K = (1-c) I + c 1 1^T``, ``C = chol(K)`` (upper, ``C^T C = K``),
  ``M ~ N(0,1)^{I x R}``, ``Q`` = orthonormal basis of ``M``, ``B = Q C``.
  Columns of ``B`` are unit vectors with pairwise cosine ``c``.
* Homoscedastic noise at relative level ``rho``:
  ``X = X0 + rho * ||X0||_F * N / ||N||_F`` with ``N`` iid N(0,1).  The
  paper's ``l1`` parameter (Section 4.3) corresponds to
  ``rho = 1 / sqrt(100 / l1 - 1)``.
* The second noise term of Section 4.3 (the paper's ``l2``, called
  heteroscedastic there) is added after the first, relative to the noisy
  tensor: ``X'' = X' + rho2 * ||X'||_F * N2 / ||N2||_F`` with ``N2`` iid
  N(0, 3^2) and ``rho2 = 1 / sqrt(100 / l2 - 1)``.  As the paper states it,
  the entries of ``N2`` share one standard deviation, which the
  normalisation by ``||N2||_F`` removes; the draw is still made as stated.
* Draw order: factor matrices in mode order, ``N``, then ``N2``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem",
    "congruent_factors",
    "gaussian_factors",
    "tensor_from_factors",
    "add_noise",
    "init_factors",
    "make_problem",
    "WORKLOADS",
    "workload",
    "batched_workload",
    "rho_from_l1",
    "add_noise_l2",
    "TABLE8",
    "table8_problem",
    "REAL_SHAPES",
    "real_shape_problem",
]


@dataclass
class Problem:
    """A synthetic CP problem: the tensor, the planted truth and the init."""

    X: np.ndarray                 # Fortran-ordered, dtype float64 or float32
    rank: int
    truth: List[np.ndarray]       # planted factors (I_n x R_true), float64
    init: List[np.ndarray]        # initial factors (I_n x R), float64
    rho: float = 0.0
    seed: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def dims(self):
        return tuple(int(d) for d in self.X.shape)

    def flat(self) -> np.ndarray:
        """The tensor as a contiguous 1-D buffer with mode 1 fastest."""
        return np.ascontiguousarray(self.X.ravel(order="F"))


def rho_from_l1(l1: float) -> float:
    """Relative noise level equivalent to the paper's homoscedastic ``l1``."""
    if l1 <= 0:
        return 0.0
    return 1.0 / np.sqrt(100.0 / l1 - 1.0)


def gaussian_factors(rng: np.random.Generator, dims: Sequence[int], rank: int):
    """Factor matrices with iid N(0,1) entries, drawn in mode order."""
    return [rng.standard_normal((int(d), rank)) for d in dims]


def congruent_factors(rng: np.random.Generator, dims: Sequence[int], rank: int,
                      c):
    """Unit-column factors with pairwise column cosine ``c`` (Section 4.3);
    ``c`` is one value for every mode or one value per mode."""
    cs = [float(c)] * len(dims) if np.isscalar(c) else [float(v) for v in c]
    if len(cs) != len(dims):
        raise ValueError("one congruence per mode")
    out = []
    for d, cm in zip(dims, cs):
        if int(d) < rank:
            raise ValueError("congruent factors need I_n >= rank (orthonormal basis of rank columns)")
        K = (1.0 - cm) * np.eye(rank) + cm * np.ones((rank, rank))
        C = np.linalg.cholesky(K).T      # upper, C^T C = K
        M = rng.standard_normal((int(d), rank))
        Q, _ = np.linalg.qr(M)           # orthonormal columns
        out.append(Q @ C)
    return out


def tensor_from_factors(factors: Sequence[np.ndarray],
                        weights: Optional[np.ndarray] = None) -> np.ndarray:
    """Dense sum of rank-1 terms, returned in Fortran order (mode 1 fastest).

    Builds the column-wise Kronecker product of the first N-1 factors (mode 1
    fastest) and multiplies it by the last factor's transpose, which is the
    mode-N unfolding of the tensor.
    """
    R = factors[0].shape[1]
    w = np.ones(R) if weights is None else np.asarray(weights, dtype=np.float64)
    T = factors[0] * w[None, :]
    for A in factors[1:-1]:
        T = (T[:, None, :] * A[None, :, :]).reshape(-1, R, order="F")
    XN = T @ factors[-1].T               # (prod I_1..I_{N-1}) x I_N
    dims = [f.shape[0] for f in factors]
    return np.asfortranarray(XN.reshape(dims, order="F"))


def add_noise(rng: np.random.Generator, X0: np.ndarray, rho: float) -> np.ndarray:
    """``X0 + rho * ||X0|| * N / ||N||`` with ``N`` iid N(0,1) (same shape)."""
    if rho == 0.0:
        return X0
    N = rng.standard_normal(X0.shape)
    scale = rho * np.linalg.norm(X0.ravel()) / np.linalg.norm(N.ravel())
    N *= scale
    N += X0
    return np.asfortranarray(N)


def add_noise_l2(rng: np.random.Generator, X1: np.ndarray, rho2: float) -> np.ndarray:
    """Second noise term of Section 4.3: ``X1 + rho2 * ||X1|| * N2 / ||N2||``
    with ``N2`` iid N(0, 3^2) (same shape)."""
    if rho2 == 0.0:
        return X1
    N2 = 3.0 * rng.standard_normal(X1.shape)
    scale = rho2 * np.linalg.norm(X1.ravel()) / np.linalg.norm(N2.ravel())
    N2 *= scale
    N2 += X1
    return np.asfortranarray(N2)


def init_factors(seed: int, dims: Sequence[int], rank: int):
    """Random N(0,1) initial factors from ``default_rng(seed + 1_000_000)``."""
    rng = np.random.default_rng(seed + 1_000_000)
    return [rng.standard_normal((int(d), rank)) for d in dims]


def make_problem(dims: Sequence[int], rank: int, *, seed: int,
                 congruence=None, rho: float = 0.0, rho2: float = 0.0,
                 true_rank: Optional[int] = None, dtype=np.float64,
                 name: str = "") -> Problem:
    """Planted low-rank tensor plus noise, with seeded random init factors.
    ``congruence``: None (iid N(0,1) factors), one value, or one per mode;
    ``rho``/``rho2``: the two relative noise levels (``l1``/``l2``)."""
    dims = [int(d) for d in dims]
    Rt = rank if true_rank is None else int(true_rank)
    rng = np.random.default_rng(seed)
    if congruence is None:
        truth = gaussian_factors(rng, dims, Rt)
    else:
        truth = congruent_factors(rng, dims, Rt, congruence)
    X0 = tensor_from_factors(truth)
    X = add_noise(rng, X0, rho)
    X = add_noise_l2(rng, X, rho2)
    X = np.asfortranarray(X.astype(dtype))
    return Problem(X=X, rank=rank, truth=truth, init=init_factors(seed, dims, rank),
                   rho=rho, seed=seed, name=name,
                   meta={"congruence": congruence, "true_rank": Rt, "rho2": rho2})


# Workload recipes.  The five named workloads mirror the sizes of the paper's
# random/synthetic suites scaled to one GPU; "small" variants keep the same
# structure at sizes the oracle finishes in seconds.
WORKLOADS = {
    "fp64_40cube_r5": dict(dims=[40, 40, 40], rank=5, seed=1, congruence=None,
                           rho=0.01, dtype=np.float64),
    "fp32_256cube_r32": dict(dims=[256, 256, 256], rank=32, seed=2,
                             congruence=0.9, rho=1e-3, dtype=np.float32),
    "fp32_96pow4_r20": dict(dims=[96, 96, 96, 96], rank=20, seed=3,
                            congruence=0.8, rho=1e-2, dtype=np.float32),
    "fp32_40pow5_r16": dict(dims=[40] * 5, rank=16, seed=5, congruence=0.85,
                            rho=1e-3, dtype=np.float32),
    # small stand-ins with the same structure
    "small_o3": dict(dims=[37, 29, 41], rank=6, seed=11, congruence=0.9,
                     rho=1e-3, dtype=np.float32),
    "small_o4": dict(dims=[13, 11, 17, 9], rank=5, seed=12, congruence=0.8,
                     rho=1e-2, dtype=np.float32),
    "small_o5": dict(dims=[7, 9, 8, 6, 10], rank=4, seed=13, congruence=0.85,
                     rho=1e-3, dtype=np.float32),
}


# Table 8 of the paper (synthetic suite): size, per-mode congruence, true
# rank, fitted rank R, l1, l2.  The third-order rows 4-6 print the
# congruences as "0.5 .09 .09", taken literally.  Rows with R > 32 are beyond
# this build's rank limit.
TABLE8 = {
    1: dict(dims=[500] * 3, c=[0.9, 0.9, 0.9], true_rank=20, rank=10, l1=0.01, l2=0.0),
    2: dict(dims=[500] * 3, c=[0.9, 0.9, 0.9], true_rank=20, rank=75, l1=0.01, l2=0.0),
    3: dict(dims=[500] * 3, c=[0.9, 0.9, 0.9], true_rank=20, rank=150, l1=0.01, l2=0.0),
    4: dict(dims=[600] * 3, c=[0.5, 0.09, 0.09], true_rank=20, rank=10, l1=0.01, l2=0.1),
    5: dict(dims=[600] * 3, c=[0.5, 0.09, 0.09], true_rank=20, rank=75, l1=0.01, l2=0.1),
    6: dict(dims=[600] * 3, c=[0.5, 0.09, 0.09], true_rank=20, rank=175, l1=0.01, l2=0.1),
    7: dict(dims=[100] * 4, c=[0.9] * 4, true_rank=20, rank=10, l1=0.1, l2=0.0),
    8: dict(dims=[100] * 4, c=[0.9] * 4, true_rank=20, rank=20, l1=0.1, l2=0.0),
    9: dict(dims=[100] * 4, c=[0.9] * 4, true_rank=20, rank=30, l1=0.1, l2=0.0),
    10: dict(dims=[120] * 4, c=[0.5, 0.9, 0.9, 0.5], true_rank=20, rank=10, l1=0.1, l2=0.01),
    11: dict(dims=[120] * 4, c=[0.5, 0.9, 0.9, 0.5], true_rank=20, rank=20, l1=0.1, l2=0.01),
    12: dict(dims=[120] * 4, c=[0.5, 0.9, 0.9, 0.5], true_rank=20, rank=30, l1=0.1, l2=0.01),
}


def table8_problem(row: int, *, dims: Optional[Sequence[int]] = None, seed: Optional[int] = None,
                   dtype=np.float32) -> Problem:
    """A Table 8 synthetic tensor (optionally at other mode sizes, e.g.
    smaller ones for tests): congruent planted factors of the true rank,
    homoscedastic noise l1 and the second noise term l2, fitted at rank R."""
    t = TABLE8[row]
    d = list(t["dims"] if dims is None else dims)
    return make_problem(d, t["rank"], seed=(800 + row) if seed is None else seed,
                        congruence=t["c"], rho=rho_from_l1(t["l1"]), rho2=rho_from_l1(t["l2"]),
                        true_rank=t["true_rank"], dtype=dtype, name=f"table8_row{row}")


# Shapes of the paper's real-world tensors (Section 4.4).  The data are not
# available here; ``real_shape_problem`` builds a stand-in of the same shape:
# a planted rank-``true_rank`` tensor with iid N(0,1) factors and noise at
# l1 = 1 (relative level 1 / sqrt(99), about 0.10).
REAL_SHAPES = {
    "indian_pines": [145, 145, 224],
    "salinas": [512, 217, 224],
    "density": [2048, 256, 256],
    "tabby_cat": [720, 1280, 3, 100],
    "winter_landscape": [1510, 1080, 3, 60],
}


def real_shape_problem(name: str, rank: int, *, scale: float = 1.0, true_rank: int = 10,
                       seed: int = 900, dtype=np.float32) -> Problem:
    """Stand-in for a real-world tensor of Section 4.4: its shape (each mode
    multiplied by ``scale`` and rounded, at least the original size if that
    is below 4), planted factors and noise."""
    dims = [d if d < 4 else max(4, int(round(d * scale))) for d in REAL_SHAPES[name]]
    return make_problem(dims, rank, seed=seed, congruence=None, rho=rho_from_l1(1.0),
                        true_rank=true_rank, dtype=dtype, name=f"{name}_standin")


def workload(name: str, dtype=None) -> Problem:
    spec = dict(WORKLOADS[name])
    if dtype is not None:
        spec["dtype"] = dtype
    return make_problem(spec.pop("dims"), spec.pop("rank"), name=name, **spec)


def batched_workload(count: int = 64, *, base_seed: int = 400, lo: int = 32,
                     hi: int = 160, rlo: int = 4, rhi: int = 24, rho: float = 0.01,
                     dtype=np.float32) -> List[Problem]:
    """Independent order-3 problems: dims iid U{lo..hi}, rank U{rlo..rhi}."""
    probs = []
    for t in range(count):
        seed = base_seed + t
        rng = np.random.default_rng(seed)
        dims = [int(v) for v in rng.integers(lo, hi + 1, size=3)]
        R = int(rng.integers(rlo, rhi + 1))
        probs.append(make_problem(dims, R, seed=seed * 7919, congruence=None,
                                  rho=rho, dtype=dtype, name=f"batch{t}"))
    return probs
