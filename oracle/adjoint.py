"""Validation-loss gradients w.r.t. log eps and log beta (oracle, FP64).

The paper never differentiates; this follows the standard adjoint method.
With A = K + beta I (training points), alpha = A^{-1} y, r_v = K_vt alpha - y_v,
L = 1/2 ||r_v||^2 (a sum, not a mean), and K' = eps dK/deps = (D^2/eps) K:

    lambda        = A^{-1} K_vt^T r_v        (A is symmetric)
    dL/dlog eps   = r_v^T K'_vt alpha - lambda^T K' alpha
    dL/dlog beta  = -beta lambda^T alpha

The preconditioner only changes how A^{-1} is applied, not the result, so it
has no derivative.
"""
from __future__ import annotations

import numpy as np

from .kernel import kernel_matrix, kernel_deriv_matrix


def val_loss(Xtr, ytr, Xval, yval, eps, beta):
    """L(eps, beta) with a dense Cholesky solve."""
    K = kernel_matrix(Xtr, Xtr, eps)
    L = np.linalg.cholesky(K + beta * np.eye(K.shape[0]))
    alpha = np.linalg.solve(L.T, np.linalg.solve(L, ytr))
    rv = kernel_matrix(Xval, Xtr, eps) @ alpha - yval
    return 0.5 * float(rv @ rv)


def val_loss_grad(Xtr, ytr, Xval, yval, eps, beta):
    """Adjoint gradient (dense). Returns (L, dL/dlog eps, dL/dlog beta, alpha, lambda)."""
    K = kernel_matrix(Xtr, Xtr, eps)
    Kp = kernel_deriv_matrix(Xtr, Xtr, eps)
    Kvt = kernel_matrix(Xval, Xtr, eps)
    Kvtp = kernel_deriv_matrix(Xval, Xtr, eps)
    Lc = np.linalg.cholesky(K + beta * np.eye(K.shape[0]))
    solve = lambda b: np.linalg.solve(Lc.T, np.linalg.solve(Lc, b))  # noqa: E731
    alpha = solve(ytr)
    rv = Kvt @ alpha - yval
    lam = solve(Kvt.T @ rv)
    g_eps = float(rv @ (Kvtp @ alpha) - lam @ (Kp @ alpha))
    g_beta = float(-beta * (lam @ alpha))
    return 0.5 * float(rv @ rv), g_eps, g_beta, alpha, lam


def fd_grad(Xtr, ytr, Xval, yval, eps, beta, h=1e-4):
    """Central finite differences in log space (step h)."""
    f = lambda le, lb: val_loss(Xtr, ytr, Xval, yval, np.exp(le), np.exp(lb))  # noqa: E731
    le, lb = np.log(eps), np.log(beta)
    g_eps = (f(le + h, lb) - f(le - h, lb)) / (2 * h)
    g_beta = (f(le, lb + h) - f(le, lb - h)) / (2 * h)
    return g_eps, g_beta

