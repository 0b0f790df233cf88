"""Preconditioned conjugate gradient (oracle, FP64): Algorithm 5 (SolveKRR), Sec. 3.

The Krylov solver is the textbook preconditioned CG (the convergence analysis of
Sec. 4.1 cites Golub and Van Loan).  Readings:
  * x0 = 0 unless given; the stopping test is the true relative residual
    ||y - (K + beta I) x||_2 / ||y||_2 <= tol, evaluated with the exact operator
    whenever the recursively updated residual says the tolerance is met.
  * Residual replacement: every ``replace_every`` iterations the recursive
    residual is overwritten by the true residual y - (K + beta I) x while the
    search direction is kept (reliable updates).  In this FP64 oracle the
    operator is exact, so replacement only removes round-off drift.
  * The step lengths gamma_j and direction coefficients delta_j are returned so
    the Lanczos tridiagonal matrix (and its extreme eigenvalues) can be formed.
"""
from __future__ import annotations

import numpy as np

from .kernel import kernel_mv, kernel_matrix


def pcg(apply_A, y, apply_M=None, *, tol=1e-10, maxit=10_000, x0=None,
        replace_every=0, apply_A_true=None, callback=None):
    """Solve A x = y.  apply_M(r) applies the preconditioner (None: identity)."""
    y = np.asarray(y, np.float64)
    A_true = apply_A_true or apply_A
    M = apply_M or (lambda r: r.copy())
    x = np.zeros_like(y) if x0 is None else np.array(x0, np.float64)
    ynorm = np.linalg.norm(y)
    if ynorm == 0.0:
        return {"x": np.zeros_like(y), "iters": 0, "relres": 0.0, "gammas": [], "deltas": [],
                "history": [0.0], "converged": True}
    r = y - A_true(x)
    z = M(r)
    p = z.copy()
    rho = r @ z
    gammas, deltas, hist = [], [], [np.linalg.norm(r) / ynorm]
    it = 0
    converged = hist[0] <= tol
    while not converged and it < maxit:
        it += 1
        q = apply_A(p)
        pq = p @ q
        if not (pq > 0):
            raise FloatingPointError(f"PCG breakdown: p^T A p = {pq}")
        gamma = rho / pq
        x = x + gamma * p
        r = r - gamma * q
        if replace_every and it % replace_every == 0:
            r = y - A_true(x)
        rel = np.linalg.norm(r) / ynorm
        if rel <= tol:
            r = y - A_true(x)
            rel = np.linalg.norm(r) / ynorm
            converged = rel <= tol
        hist.append(rel)
        gammas.append(gamma)
        if callback is not None:
            callback(it, x, rel)
        if converged:
            break
        z = M(r)
        rho_new = r @ z
        delta = rho_new / rho
        deltas.append(delta)
        p = z + delta * p
        rho = rho_new
    return {"x": x, "iters": it, "relres": hist[-1], "gammas": gammas, "deltas": deltas,
            "history": hist, "converged": converged}


def lanczos_tridiagonal(gammas, deltas):
    """Tridiagonal T of the Lanczos process equivalent to the CG run (Golub & Van Loan, Sec. 11.3).

    T[j, j] = 1/gamma_j + delta_{j-1}/gamma_{j-1};  T[j, j+1] = sqrt(delta_j)/gamma_j.
    """
    m = len(gammas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / gammas[j] + (deltas[j - 1] / gammas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(deltas[j]) / gammas[j]
    return T


def kappa_estimate(gammas, deltas):
    """Condition number estimate of the preconditioned operator from the CG coefficients."""
    if len(gammas) == 0:
        return 1.0
    ev = np.linalg.eigvalsh(lanczos_tridiagonal(gammas, deltas))
    return float(ev[-1] / ev[0])


def krr_operator(X, eps, beta, dense=None):
    """v -> (K + beta I) v, dense when a K is given, matrix-free otherwise."""
    if dense is not None:
        return lambda v: dense @ v + beta * v
    return lambda v: kernel_mv(X, X, eps, v) + beta * v


def solve_dense(X, y, eps, beta):
    """alpha* = (K + beta I)^{-1} y by Cholesky (the O(n^3) direct solve of Sec. 1)."""
    K = kernel_matrix(X, X, eps)
    L = np.linalg.cholesky(K + beta * np.eye(K.shape[0]))
    return np.linalg.solve(L.T, np.linalg.solve(L, y))


def solve_krr(X, y, eps, beta, P=None, *, tol=1e-10, maxit=10_000, dense=True, replace_every=0):
    """Algorithm 5: CG on (K + beta I) alpha = y with the Woodbury preconditioner P (None: plain CG)."""
    from .precond import apply_precond
    K = kernel_matrix(X, X, eps) if dense else None
    A = krr_operator(X, eps, beta, K)
    M = None if P is None else (lambda r: apply_precond(P, beta, r))
    return pcg(A, y, M, tol=tol, maxit=maxit, replace_every=replace_every)
