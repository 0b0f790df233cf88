"""ID / Nystrom / Woodbury preconditioner (oracle, FP64), Section 3 of the paper.

Steps, in the paper's order:
  Algorithm 1 (AnchorSelection): Y = FIG(X, X, h, Omega) with a Gaussian test
      matrix, then a pivoted QR of Y^T; the first k pivots are the anchors.
  Algorithm 2 (SparseAnchorSelection): column i of Y is the kernel applied to a
      Rademacher vector supported on r random points; then the same pivoted QR.
  Algorithm 3 (BuildCholesky): U^{-1} = K(X_S, X_S); a square root U^{1/2} from
      an EVD; Y = C U^{1/2}; Cholesky of beta I + U^{1/2} C^T C U^{1/2}
      (Eq. to_factor2 and Eq. chol_factor).
  Remark in Sec. 3: the anchors may instead come from random sampling or farthest
      point sampling; Algorithm 3 then runs unchanged on them.
  Algorithm 4 (ApplyPreconditioner): (K~ + beta I)^{-1} x through the Woodbury
      identity (Eq. woodbury) in the stabilised form.

Readings where the paper is loose (all stated in the design notes too):
  * U is the inverse of the anchor block, U^{-1} = K_SS (Sec. 3), not the
    overlap itself as in the Nystrom paragraph of Sec. 2.2.
  * U^{1/2} comes from the symmetric EVD K_SS = V diag(lam) V^T with
    eigenvalues lam_i <= tau * lam_max dropped (pseudo-inverse square root).
    The factor is stored as W = C V_kept diag(lam_kept)^{-1/2}; it differs
    from C U^{1/2} by the orthogonal factor V_kept^T on the right, which
    cancels in W W^T and in the Woodbury apply.
  * Omega is l x n in the paper but applied as weights over the n points, so
    Y = K Omega^T is n x l and the pivoted QR runs on Y^T (l x n).
  * Plain column-pivoted Householder QR stands in for strong RRQR (the paper
    remarks the two perform alike in practice).  Ties go to the lowest point
    index.  The oracle recomputes every residual column norm at every step
    (no norm downdating).
  * Cholesky convention: lower L with L L^T (the paper writes L^T L).
  * Other anchor choices (remark in Sec. 3): random sampling (the indices are an input,
    drawn by the caller) and farthest point sampling, read as the greedy rule that adds the
    point farthest from the chosen set, squared Euclidean distances, ties to the lowest index.
"""
from __future__ import annotations

import numpy as np

from .kernel import kernel_matrix, kernel_mv

DEFAULT_TAU = 1e-12


# ---------------------------------------------------------------- sketches
def sketch_dense(X, eps, omega):
    """Algorithm 1, sketch step: Y = K(X, X) Omega^T with omega stored n x l."""
    return kernel_mv(X, X, eps, np.asarray(omega, np.float64))


def sketch_sparse(X, eps, idx, sign):
    """Algorithm 2, sketch loop: Y[:, i] = sum_s sign[i, s] * K(X, x_{idx[i, s]})."""
    X = np.asarray(X, np.float64)
    idx = np.asarray(idx, np.int64)
    sign = np.asarray(sign, np.float64)
    l = idx.shape[0]
    Y = np.zeros((X.shape[0], l))
    for i in range(l):
        XR = X[idx[i]]                       # X_R = X(R, :)
        Y[:, i] = kernel_mv(X, XR, eps, sign[i])
    return Y


# ---------------------------------------------------------------- pivoted QR
def qrcp(A, k, forced=None):
    """Column-pivoted Householder QR of A (m x N), first k steps.

    At step j the residual norms of all unselected columns are recomputed from
    the updated matrix, the largest is chosen (lowest index on ties), and a
    Householder reflector zeroes the pivot column below row j.

    forced: optional pivot sequence to follow instead of the argmax; used to
    check that another implementation's pivots are valid choices.

    Returns dict(piv, rdiag, maxnorm): piv[j] the j-th pivot column, rdiag[j] =
    |R_jj| (the pivot's residual norm), maxnorm[j] the largest residual norm
    among unselected columns at step j (equals rdiag[j] unless forced).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    m, N = A.shape
    k = min(k, m, N)
    selected = np.zeros(N, dtype=bool)
    piv = np.empty(k, dtype=np.int64)
    rdiag = np.empty(k)
    maxnorm = np.empty(k)
    for j in range(k):
        norms = np.sqrt((A[j:, :] ** 2).sum(axis=0))
        norms[selected] = -1.0
        best = int(np.argmax(norms))
        p = best if forced is None else int(forced[j])
        if selected[p]:
            raise ValueError(f"pivot {p} selected twice")
        piv[j] = p
        rdiag[j] = norms[p]
        maxnorm[j] = norms[best]
        selected[p] = True
        # Householder reflector H = I - 2 u u^T / (u^T u) mapping A[j:, p] to -sign(a0)|a| e_1
        a = A[j:, p].copy()
        alpha = np.linalg.norm(a)
        if alpha == 0.0:
            continue
        u = a.copy()
        u[0] += np.copysign(alpha, a[0]) if a[0] != 0 else alpha
        uu = u @ u
        A[j:, :] -= np.outer(u, (2.0 / uu) * (u @ A[j:, :]))
    return {"piv": piv, "rdiag": rdiag, "maxnorm": maxnorm}


def anchor_selection(Y, k):
    """Algorithms 1-2, last steps: S = P(1:k) from the pivoted QR of Y^T."""
    return qrcp(np.asarray(Y).T, k)["piv"]


# ---------------------------------------------------------------- Nystrom factor
def nystrom_factor(X, S, eps, tau=DEFAULT_TAU):
    """Algorithm 3 up to the core: returns W (n x k') with W W^T = C U C^T.

    U^{-1} = K(X_S, X_S); EVD; drop eigenvalues <= tau * max; W = C V diag(lam)^{-1/2}.
    """
    X = np.asarray(X, np.float64)
    XS = X[np.asarray(S, np.int64)]
    Kss = kernel_matrix(XS, XS, eps)                 # U^{-1}
    lam, V = np.linalg.eigh(Kss)
    keep = lam > tau * lam.max()
    T = V[:, keep] / np.sqrt(lam[keep])              # V_kept diag(lam_kept)^{-1/2}
    C = kernel_matrix(X, XS, eps)                    # C = K(X, X_S)
    W = C @ T
    return {"W": W, "lam": lam, "kept": int(keep.sum()), "T": T, "Kss": Kss}


def symmetric_sqrt_inv(Kss, tau=DEFAULT_TAU):
    """U^{1/2} = V diag(lam)^{-1/2} V^T (pseudo-inverse square root of K_SS)."""
    lam, V = np.linalg.eigh(Kss)
    keep = lam > tau * lam.max()
    return (V[:, keep] / np.sqrt(lam[keep])) @ V[:, keep].T


def core_cholesky(W, beta):
    """Eq. chol_factor: lower L with L L^T = beta I + W^T W (W^T W = U^{1/2} C^T C U^{1/2})."""
    M = W.T @ W
    return np.linalg.cholesky(beta * np.eye(M.shape[0]) + M)


def woodbury_apply(W, L, beta, x):
    """Algorithm 4 with W = C U^{1/2}: t = W^T x; L L^T z = t; return (x - W z) / beta."""
    x = np.asarray(x, np.float64)
    t = W.T @ x
    z = np.linalg.solve(L.T, np.linalg.solve(L, t))   # two triangular solves (dense solver used as one)
    return (x - W @ z) / beta


def woodbury_apply_unstabilised(C, Kss, beta, x):
    """Eq. woodbury as printed: x/beta - C (beta U^{-1} + C^T C)^{-1} C^T x / beta, U^{-1} = K_SS."""
    core = beta * Kss + C.T @ C
    return (x - C @ np.linalg.solve(core, C.T @ x)) / beta


def build_precond(X, eps, betas, k, *, omega=None, idx=None, sign=None, tau=DEFAULT_TAU):
    """Setup stage: anchors (Alg. 1 if omega is given, else Alg. 2), Nystrom factor, one core factor per beta."""
    if omega is not None:
        Y = sketch_dense(X, eps, omega)
    else:
        Y = sketch_sparse(X, eps, idx, sign)
    qr = qrcp(Y.T, k)
    P = build_precond_from_anchors(X, eps, betas, qr["piv"], tau=tau)
    P.update(Y=Y, rdiag=qr["rdiag"])
    return P


def build_precond_from_anchors(X, eps, betas, S, *, tau=DEFAULT_TAU):
    """Algorithm 3 for anchors chosen some other way (remark in Sec. 3: random sampling or FPS
    in place of the ID; the theoretical bounds then no longer apply)."""
    S = np.asarray(S, np.int64)
    nf = nystrom_factor(X, S, eps, tau)
    Ls = {float(b): core_cholesky(nf["W"], float(b)) for b in np.atleast_1d(betas)}
    return {"S": S, "W": nf["W"], "lam": nf["lam"], "kept": nf["kept"], "L": Ls}


# ---------------------------------------------------------------- farthest point sampling
def sqdist_to_point(X, x):
    """||X[i] - x||^2 for every row, accumulated coordinate by coordinate: each difference,
    square and sum is rounded on its own (no fused multiply-add)."""
    X = np.asarray(X, np.float64)
    acc = np.zeros(X.shape[0])
    for c in range(X.shape[1]):
        t = X[:, c] - x[c]
        acc = acc + t * t
    return acc


def fps(X, k, start=0):
    """Farthest point sampling, the second alternative anchor choice named in the remark of Sec. 3.

    S[0] = start.  Step j picks, among the points not yet chosen, the one whose squared distance
    to the nearest chosen point is largest (ties to the lowest index).  Returns (S, dsel) with
    dsel[j] that largest squared distance (dsel[0] = inf).
    """
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    if not 1 <= k <= n or not 0 <= start < n:
        raise ValueError("need 1 <= k <= n and 0 <= start < n")
    S = np.empty(k, np.int64)
    dsel = np.empty(k)
    S[0], dsel[0] = start, np.inf
    chosen = np.zeros(n, bool)
    chosen[start] = True
    dmin = np.full(n, np.inf)
    for j in range(1, k):
        dmin = np.minimum(dmin, sqdist_to_point(X, X[S[j - 1]]))
        cand = np.where(chosen, -np.inf, dmin)
        i = int(np.argmax(cand))             # first maximum = lowest index
        S[j], dsel[j] = i, cand[i]
        chosen[i] = True
    return S, dsel


def apply_precond(P, beta, x):
    return woodbury_apply(P["W"], P["L"][float(beta)], float(beta), x)


def preconditioned_spectrum(K, W, beta):
    """Eigenvalues of (K~ + beta I)^{-1/2} (K + beta I) (K~ + beta I)^{-1/2} with K~ = W W^T (dense, small n)."""
    n = K.shape[0]
    Pm = W @ W.T + beta * np.eye(n)
    lp, Vp = np.linalg.eigh(Pm)
    Pmh = (Vp / np.sqrt(lp)) @ Vp.T
    A = Pmh @ (K + beta * np.eye(n)) @ Pmh
    return np.linalg.eigvalsh((A + A.T) / 2)
