"""Gaussian kernel and kernel matrix-vector products (oracle, FP64).

Definitions followed:
  * KRR estimator f(x) = sum_j k(x_j, x) alpha_j and (K + beta I) alpha = y      (Sec. 1, Eq. 1 and Eq. ridge_regression)
  * Gaussian kernel k(x, x') = exp(-||x - x'||^2 / h^2)                          (Sec. 2.4, Eq. dscrt_gt)
    written here with eps = h^2, i.e. k(x, x') = exp(-||x - x'||^2 / eps).
  * FIG(targets, sources, h, q) is read as the exact weighted sum
    G(t_i) = sum_j q_j k(t_i, s_j)                                               (Sec. 2.4, Def. figtree_def)
    computed directly (the conclusions allow direct computation in parts).
  * Derivative kernel for the gradient path: eps * dk/deps = (D^2/eps) k.
"""
from __future__ import annotations

import numpy as np


def sqdist(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances D2[i, j] = ||A_i - B_j||^2 by explicit differences."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    diff = A[:, None, :] - B[None, :, :]
    return np.einsum("ijk,ijk->ij", diff, diff)


def kernel_matrix(Xt: np.ndarray, Xs: np.ndarray, eps: float) -> np.ndarray:
    """K[i, j] = exp(-||Xt_i - Xs_j||^2 / eps)."""
    return np.exp(-sqdist(Xt, Xs) / eps)


def kernel_deriv_matrix(Xt: np.ndarray, Xs: np.ndarray, eps: float) -> np.ndarray:
    """K'[i, j] = eps * d/deps exp(-D2/eps) = (D2/eps) exp(-D2/eps)."""
    D2 = sqdist(Xt, Xs)
    return (D2 / eps) * np.exp(-D2 / eps)


def kernel_mv(Xt, Xs, eps, V, shift=None, deriv=0, block=None):
    """Matrix-free product U = K(Xt, Xs) V (+ V * shift per column), never storing K.

    V is n (or n x R).  ``shift`` (length R or scalar) adds shift_r * V[:, r];
    it requires Xt and Xs to be the same point set (the ridge term beta*I).
    deriv=0: K V;  deriv=1: K' V;  deriv=2: returns (K V, K' V).
    Rows of the target set are processed in blocks of ``block`` (default: sized so one block's
    distance table stays near 256 MB); every row is computed the same way whatever the block size.
    """
    Xt = np.asarray(Xt, np.float64)
    Xs = np.asarray(Xs, np.float64)
    V = np.asarray(V, np.float64)
    vec = V.ndim == 1
    V2 = V[:, None] if vec else V
    m = Xt.shape[0]
    if block is None:
        block = int(max(1, min(512, (1 << 25) // max(1, Xs.shape[0] * Xs.shape[1]))))
    U = np.zeros((m, V2.shape[1]))
    Ud = np.zeros((m, V2.shape[1])) if deriv == 2 else None
    for s in range(0, m, block):
        e = min(m, s + block)
        D2 = sqdist(Xt[s:e], Xs)
        Kb = np.exp(-D2 / eps)
        if deriv == 0:
            U[s:e] = Kb @ V2
        elif deriv == 1:
            U[s:e] = ((D2 / eps) * Kb) @ V2
        else:
            U[s:e] = Kb @ V2
            Ud[s:e] = ((D2 / eps) * Kb) @ V2
    if shift is not None:
        if Xt.shape != Xs.shape or not np.array_equal(Xt, Xs):
            raise ValueError("shift requires targets == sources")
        U = U + V2 * np.asarray(shift, np.float64)
    if deriv == 2:
        return (U[:, 0], Ud[:, 0]) if vec else (U, Ud)
    return U[:, 0] if vec else U


def kernel_mv_rows(X, eps, v, rows, shift=0.0):
    """Exact ((K + shift I) v)[rows] for a sample of rows (used at sizes where a full product is too slow)."""
    X = np.asarray(X, np.float64)
    rows = np.asarray(rows, np.int64)
    out = kernel_mv(X[rows], X, eps, v)
    return out + shift * np.asarray(v, np.float64)[rows] if np.ndim(v) == 1 else out + shift * v[rows]


def predict(Xq, X, eps, alpha):
    """f(x) = sum_j k(x_j, x) alpha_j  (Sec. 1, Eq. 1)."""
    return kernel_mv(Xq, X, eps, alpha)
