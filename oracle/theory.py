"""Closed-form bounds of Section 4 (oracle).

  * Theorem maintheorem: cond[(K~+bI)^{-1}(K+bI)] <= 1 + M lam_{k+1}(K) / b
  * ID corollary: M = 2 sqrt(4k(n-k)+1), so cond <= 1 + 2 lam_{k+1} sqrt(4k(n-k)+1)/b <= 1 + 2 lam_{k+1}(n+1)/b
  * SVD remark: with K~ the best rank-k approximation, cond = 1 + lam_{k+1}/b exactly
  * Theorem gaussiankernelbound / Corollary tradeoff (Eq. condbound): rank needed for a target condition number
    gamma = (2/pi) sqrt(h^{-2} ln(Mbar n / (b (xi - 1)))),  k >= prod_i (floor(gamma q_i) + 1),
    on a dataset with q_i its bounding-box side lengths and h = sqrt(eps)
  * Eq. cgrate: ||e_i||_A <= 2 ||e_0||_A ((sqrt(kappa)-1)/(sqrt(kappa)+1))^i
  * Eq. noprecond_rate and Eq. precond_rate2: iteration estimates
"""
from __future__ import annotations

import math

import numpy as np


def cond_bound(lam_k1, beta, M):
    return 1.0 + M * lam_k1 / beta


def cond_bound_id(lam_k1, k, n, beta):
    """Corollary for the ID-built Nystrom preconditioner (both the tight and the (n+1) form)."""
    tight = 1.0 + 2.0 * lam_k1 * math.sqrt(4.0 * k * (n - k) + 1.0) / beta
    loose = 1.0 + 2.0 * lam_k1 * (n + 1.0) / beta
    return tight, loose


def cond_svd(lam_k1, beta):
    """Remark after the ID corollary: best rank-k approximation gives exactly 1 + lam_{k+1}/beta."""
    return 1.0 + lam_k1 / beta


def rank_gamma(h, n, beta, xi, Mbar=None):
    """gamma of Eq. condbound_gamma with delta = beta (xi-1) / (Mbar n); Mbar defaults to n."""
    Mbar = n if Mbar is None else Mbar
    return (2.0 / math.pi) * math.sqrt(h ** -2 * math.log(Mbar * n / (beta * (xi - 1.0))))


def rank_bound(q, h, n, beta, xi, Mbar=None):
    """Eq. condbound: k >= prod_i (floor(gamma q_i) + 1); returned as an exact Python int."""
    g = rank_gamma(h, n, beta, xi, Mbar)
    out = 1
    for qi in q:
        out *= int(math.floor(g * qi)) + 1
    return out


def rank_for_cond(X, eps, beta, xi, Mbar=None):
    """Corollary tradeoff applied to a dataset: q_i are the side lengths of the bounding box of X,
    h = sqrt(eps), n the number of points.  Returns (gamma, k) of Eq. condbound_gamma / Eq. condbound."""
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    q = X.max(axis=0) - X.min(axis=0)
    h = math.sqrt(eps)
    return rank_gamma(h, n, beta, xi, Mbar), rank_bound(q, h, n, beta, xi, Mbar)


def cg_error_bound(kappa, i):
    """Eq. cgrate: ratio ||e_i||_A / ||e_0||_A <= 2 ((sqrt k - 1)/(sqrt k + 1))^i."""
    s = math.sqrt(kappa)
    return 2.0 * ((s - 1.0) / (s + 1.0)) ** i


def iters_noprecond(lam1, beta, delta):
    """Eq. noprecond_rate (large-kappa approximation)."""
    return -math.sqrt(lam1) * math.log(delta) / (2.0 * math.sqrt(beta))


def iters_precond(lam_k1, beta, M, delta):
    """Eq. precond_rate2."""
    a = math.sqrt(beta + M * lam_k1)
    b = math.sqrt(beta)
    return math.log(delta) / math.log((a - b) / (a + b))


def numerical_rank(K, delta):
    """Def. numerical_rank: #{j : sigma_j / sigma_1 >= delta}."""
    s = np.linalg.svd(K, compute_uv=False)
    return int((s / s[0] >= delta).sum())
