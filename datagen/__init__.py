"""Seeded synthetic workloads for Gaussian kernel ridge regression.

This module only draws inputs: data points X, labels y, held-out points, and
the random numbers the anchor-selection sketch consumes (the dense Gaussian
test matrix of Algorithm 1, the index sets and Rademacher signs of
Algorithm 2).  It contains none of the solver's arithmetic, so both the CPU
oracle and the HIP library can be fed from it without sharing any code path.

The paper evaluates on real datasets (Helicopter, an EM-field simulator,
YearSong, CovType, Buzz; Section 5) that are not available here.  The five
workloads below are synthetic stand-ins with fixed shapes and distributions;
they match the paper's scale in n and k, not its data.

Workloads (kernel exp(-||x-x'||^2/eps), i.e. eps = h^2 in the paper's
notation of Eq. (dscrt_gt)):

  small   n=2,000      d=3   eps=0.05  beta=1e-3       k=150   l=170   dense sketch
  fp32    n=100,000    d=8   eps=0.2   beta=1e-2       k=1000  l=1020  sparse sketch r=32
  mixed   n=1,000,000  d=4   eps=0.01  beta=1e-3       k=2000  l=2020  sparse sketch r=32
  adjoint n=200,000 (+20,000 val)  d=16  eps=4.0  beta=1e-2  k=1000  l=1020
  block   n=500,000    d=6   eps=0.05  beta in {1e-4,1e-3,1e-2,1e-1}, 32 labels -> 128 systems,
          k=1500 l=1520
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = ["Workload", "WORKLOADS", "make_workload", "sketch_dense_omega",
           "sketch_sparse_draws", "subset", "uniform_points"]


@dataclass
class Workload:
    name: str
    X: np.ndarray                  # n x d, float64, C-contiguous
    y: np.ndarray                  # n (or n x R for the block workload), float64
    eps: float
    betas: tuple                   # ridge parameter(s)
    k: int                         # preconditioner rank
    l: int                         # sketch width (l >= k)
    r: int                         # nonzeros per sparse sketch column; 0 = dense Gaussian sketch
    tol: float
    X_test: Optional[np.ndarray] = None
    X_val: Optional[np.ndarray] = None
    y_val: Optional[np.ndarray] = None
    col_beta: Optional[np.ndarray] = None   # block workload: beta of each RHS column
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _small(scale: float = 1.0) -> Workload:
    rng = np.random.default_rng(1)
    n = 2000
    X = rng.random((n, 3))
    y = np.sin(2 * np.pi * X[:, 0]) * np.cos(np.pi * X[:, 1]) + 0.1 * rng.standard_normal(n)
    Xt = rng.random((1000, 3))
    return Workload("small", _c(X), _c(y), 0.05, (1e-3,), 150, 170, 0, 1e-10, X_test=_c(Xt))


def _fp32(n: int = 100_000) -> Workload:
    rng = np.random.default_rng(2)
    d = 8
    centers = rng.random((20, d))
    comp = rng.integers(0, 20, n)
    X = centers[comp] + 0.1 * rng.standard_normal((n, d))
    c = rng.random((3, d))
    a = rng.standard_normal(3)
    # three radial bumps of width 0.3: a_b * exp(-|x-c_b|^2 / (2*0.3^2))
    y = sum(a[b] * np.exp(-((X - c[b]) ** 2).sum(1) / (2 * 0.3 ** 2)) for b in range(3))
    y = y + 0.05 * rng.standard_normal(n)
    comp_t = rng.integers(0, 20, 10_000)
    Xt = centers[comp_t] + 0.1 * rng.standard_normal((10_000, d))
    return Workload("fp32", _c(X), _c(y), 0.2, (1e-2,), 1000, 1020, 32, 1e-8, X_test=_c(Xt))


def _mixed(n: int = 1_000_000) -> Workload:
    rng = np.random.default_rng(3)
    d = 4
    X = rng.random((n, d))
    y = sum(np.sin(2 * np.pi * m * X[:, m - 1]) / m for m in range(1, d + 1))
    y = y + 0.1 * rng.standard_normal(n)
    Xt = rng.random((10_000, d))
    return Workload("mixed", _c(X), _c(y), 0.01, (1e-3,), 2000, 2020, 32, 1e-6, X_test=_c(Xt))


def _adjoint(n: int = 200_000, m: int = 20_000) -> Workload:
    rng = np.random.default_rng(4)
    d = 16
    w = rng.standard_normal(d) / 4.0
    Xtr = 0.5 * rng.standard_normal((n, d))
    Xval = 0.5 * rng.standard_normal((m, d))
    ytr = np.tanh(Xtr @ w) + 0.1 * rng.standard_normal(n)
    yval = np.tanh(Xval @ w) + 0.1 * rng.standard_normal(m)
    return Workload("adjoint", _c(Xtr), _c(ytr), 4.0, (1e-2,), 1000, 1020, 32, 1e-8,
                    X_val=_c(Xval), y_val=_c(yval))


def _block(n: int = 500_000) -> Workload:
    rng = np.random.default_rng(5)
    d = 6
    X = rng.random((n, d))
    a = 2.0 * rng.standard_normal((32, d))
    b = 2 * np.pi * rng.random(32)
    labels = np.sin(X @ a.T + b) + 0.05 * rng.standard_normal((n, 32))
    betas = (1e-4, 1e-3, 1e-2, 1e-1)
    # column j <-> (label j // 4, beta index j % 4)
    Y = np.repeat(labels, 4, axis=1)
    col_beta = np.tile(np.array(betas), 32)
    Xt = rng.random((10_000, d))
    return Workload("block", _c(X), _c(Y), 0.05, betas, 1500, 1520, 32, 1e-6,
                    X_test=_c(Xt), col_beta=col_beta)


WORKLOADS = {"small": _small, "fp32": _fp32, "mixed": _mixed, "adjoint": _adjoint, "block": _block}
_SKETCH_SEED = {"small": 101, "fp32": 102, "mixed": 103, "adjoint": 104, "block": 105}


def make_workload(name: str, **kw) -> Workload:
    """Build one of the named workloads (optionally with a smaller n for tests)."""
    return WORKLOADS[name](**kw)


def sketch_seed(name: str) -> int:
    return _SKETCH_SEED[name]


def sketch_dense_omega(n: int, l: int, seed: int) -> np.ndarray:
    """Algorithm 1's Gaussian test matrix, stored n x l (the paper's Omega is l x n)."""
    rng = np.random.default_rng(seed)
    return _c(rng.standard_normal((n, l)))


def sketch_sparse_draws(n: int, l: int, r: int, seed: int):
    """Algorithm 2's random draws: for each of the l sketch columns, r distinct
    point indices (uniform without replacement) and r Rademacher signs.

    Returns (idx, sign): int64 l x r and float64 l x r (entries +-1).
    """
    if r > n:
        raise ValueError("r must not exceed n")
    rng = np.random.default_rng(seed)
    idx = np.empty((l, r), dtype=np.int64)
    for i in range(l):
        idx[i] = rng.choice(n, size=r, replace=False)
    sign = rng.integers(0, 2, size=(l, r)).astype(np.float64) * 2.0 - 1.0
    return np.ascontiguousarray(idx), _c(sign)


def random_anchors(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct point indices drawn uniformly without replacement (random-sampling anchors)."""
    if not 1 <= k <= n:
        raise ValueError("need 1 <= k <= n")
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.choice(n, size=k, replace=False).astype(np.int64))


def uniform_points(n: int, d: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _c(lo + (hi - lo) * rng.random((n, d)))


def subset(wl: Workload, n_train: int, n_val: int = 0) -> Workload:
    """First n_train training points (and first n_val validation points)."""
    y = wl.y[:n_train]
    return Workload(wl.name + f"_sub{n_train}", _c(wl.X[:n_train]), _c(y), wl.eps, wl.betas,
                    min(wl.k, n_train), min(wl.l, n_train), wl.r, wl.tol,
                    X_test=wl.X_test,
                    X_val=None if wl.X_val is None else _c(wl.X_val[:n_val]),
                    y_val=None if wl.y_val is None else _c(wl.y_val[:n_val]),
                    col_beta=wl.col_beta)
