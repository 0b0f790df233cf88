"""End-to-end solves in the arithmetic of the n = 1,000,000, d = 4 workload, at a size the dense oracle
solves: uniform points in [0,1]^4, eps = 0.01, beta = 1e-3, Algorithm 2 anchors, split-BF16 cross term
with FP32 exp and FP64 residual replacement every 10 iterations, tol 1e-6 (Algorithm 5).

alpha* = (K + beta I)^{-1} y is unique, so every solve is held to the perturbation bound
||alpha - alpha*|| / ||alpha*|| <= kappa(K + beta I) ||y - (K + beta I) alpha|| / ||y||, with kappa bounded
above by (max row sum of K + beta) / beta (Gershgorin; K has positive entries) and the residual recomputed
in FP64 on the CPU.  The mixed solve is also compared with an FP64 GPU solve run to 1e-9.

Also here: the truncation path of the anchor eigendecomposition (eigenvalues of K_SS at or below
tau * max dropped; remark before Eq. to_factor2 that anchors may be very close), forced with
near-duplicate points among random anchors.
"""
import numpy as np
import pytest
import torch

import datagen
from oracle import kernel as ok
from oracle import pcg as oc
from oracle import precond as op


@pytest.fixture(scope="module")
def mixed10k(gpu_lib):
    wl = datagen.make_workload("mixed", n=10_000)
    K = ok.kernel_matrix(wl.X, wl.X, wl.eps)
    beta = wl.betas[0]
    A = K + beta * np.eye(wl.n)
    L = np.linalg.cholesky(A)
    alpha = np.linalg.solve(L.T, np.linalg.solve(L, wl.y))
    kappa_ub = (K.sum(1).max() + beta) / beta
    k, l, r = 1000, 1020, 32
    idx, sign = datagen.sketch_sparse_draws(wl.n, l, r, datagen.sketch_seed("mixed"))
    P = gpu_lib.Preconditioner(torch.from_numpy(wl.X), wl.eps, [beta], k, l, idx=torch.from_numpy(idx),
                               sign=torch.from_numpy(sign), prec="mixed")
    return wl, A, alpha, kappa_ub, P


def _relres(A, y, a):
    return np.linalg.norm(y - A @ a) / np.linalg.norm(y)


@pytest.mark.gpu
def test_mixed_solve_reaches_tol_and_matches_oracle(gpu_lib, mixed10k):
    wl, A, astar, kub, P = mixed10k
    X, y = torch.from_numpy(wl.X), torch.from_numpy(wl.y)
    beta = wl.betas[0]
    am, its, rel, st, status = gpu_lib.pcg_solve(X, y, wl.eps, beta, P, tol=1e-6, maxit=20000, replace_every=10,
                                                 prec="mixed")
    assert status == 0 and rel[0] <= 1e-6
    am = am.cpu().numpy()
    rr = _relres(A, wl.y, am)
    err = np.linalg.norm(am - astar) / np.linalg.norm(astar)
    # FP64 reference on the GPU, same preconditioner, to 1e-9
    a64, its64, rel64, st64, status64 = gpu_lib.pcg_solve(X, y, wl.eps, beta, P, tol=1e-9, maxit=20000,
                                                          prec="fp64")
    assert status64 == 0 and rel64[0] <= 1e-9
    a64 = a64.cpu().numpy()
    err64 = np.linalg.norm(a64 - astar) / np.linalg.norm(astar)
    dm = np.linalg.norm(am - a64) / np.linalg.norm(a64)
    # held-out predictions f = K(X*, X) alpha (Eq. 1): the GPU FP64 product of the mixed alpha against the
    # oracle's prediction with alpha*
    Xq = wl.X_test[:1000]
    f_gpu = gpu_lib.kernel_mv(torch.from_numpy(Xq), X, wl.eps, torch.from_numpy(am), prec="fp64").cpu().numpy()
    f_ref = ok.predict(Xq, wl.X, wl.eps, astar)
    ferr = np.linalg.norm(f_gpu - f_ref) / np.linalg.norm(f_ref)
    print(f"mixed: {its[0]} its, relres GPU {rel[0]:.3e} CPU {rr:.3e}, alpha err vs Cholesky {err:.3e}; "
          f"FP64 (1e-9): {its64[0]} its, err {err64:.3e}; mixed vs FP64 {dm:.3e}; predictions {ferr:.3e}; "
          f"kappa upper bound {kub:.3e}, Lanczos kappa (preconditioned) {st['kappa_est']:.3e}")
    assert rr <= 1.01e-6
    assert err <= kub * rr
    assert err64 <= kub * _relres(A, wl.y, a64)
    assert dm <= kub * (1e-6 + 1e-9)
    assert ferr <= kub * rr
    # the measured levels sit far inside the bounds; these bars state them (about 10x above what MI355X gives)
    assert err <= 5e-5 and dm <= 5e-5 and ferr <= 5e-6


@pytest.mark.gpu
def test_fp64_and_mixed_solves_at_1e6_agree_within_bound(gpu_lib, mixed10k):
    """Both working precisions stopped at 1e-6: their difference is bounded by 2 kappa tol."""
    wl, A, astar, kub, P = mixed10k
    X, y = torch.from_numpy(wl.X), torch.from_numpy(wl.y)
    beta = wl.betas[0]
    res = {}
    for prec, rep in (("mixed", 10), ("fp32", 10), ("fp64", 0)):
        a, its, rel, st, status = gpu_lib.pcg_solve(X, y, wl.eps, beta, P, tol=1e-6, maxit=20000,
                                                    replace_every=rep, prec=prec)
        assert status == 0 and rel[0] <= 1e-6
        res[prec] = a.cpu().numpy()
        assert _relres(A, wl.y, res[prec]) <= 1.01e-6
    for p in ("mixed", "fp32"):
        d = np.linalg.norm(res[p] - res["fp64"]) / np.linalg.norm(res["fp64"])
        print(f"{p} vs fp64 at tol 1e-6: {d:.3e}")
        assert d <= 2 * kub * 1e-6


def _dup_points(n=600, ndup=20, seed=12):
    rng = np.random.default_rng(seed)
    X = rng.random((n, 2))
    X[n - ndup:] = X[:ndup] + 1e-9 * rng.standard_normal((ndup, 2))
    return X


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_evd_truncation_drops_near_duplicate_anchors(gpu_lib, prec):
    n, ndup, eps, beta = 600, 20, 0.01, 1e-3
    X = _dup_points(n, ndup)
    rng = np.random.default_rng(13)
    others = rng.choice(np.arange(ndup, n - ndup), size=40, replace=False)
    # ten duplicate pairs among the anchors: K_SS has ten eigenvalues near (1e-9)^2 / eps
    S = np.concatenate([np.arange(10), np.arange(n - ndup, n - ndup + 10), others]).astype(np.int64)
    k = len(S)
    ref = op.build_precond_from_anchors(X, eps, [beta], S)
    assert ref["kept"] == k - 10
    P = gpu_lib.Preconditioner(torch.from_numpy(X), eps, [beta], k, anchors=torch.from_numpy(S), prec=prec)
    info = P.info()
    assert info["kept"] == k - 10
    W = P.get(P.W64).cpu().numpy()
    assert W.shape == (n, k - 10)
    np.testing.assert_allclose(W @ W.T, ref["W"] @ ref["W"].T, rtol=0, atol=1e-9)
    # Lemma schur survives the truncation: the preconditioned eigenvalues stay >= 1
    K = ok.kernel_matrix(X, X, eps)
    lam = op.preconditioned_spectrum(K, W, beta)
    assert lam.min() >= 1 - 1e-9
    y = np.sin(5 * X[:, 0]) + X[:, 1]
    a, its, rel, st, status = gpu_lib.pcg_solve(torch.from_numpy(X), torch.from_numpy(y), eps, beta, P,
                                                tol=1e-8, maxit=5000, replace_every=10 if prec != "fp64" else 0,
                                                prec=prec)
    assert status == 0 and rel[0] <= 1e-8
    astar = oc.solve_dense(X, y, eps, beta)
    kub = (K.sum(1).max() + beta) / beta
    A = K + beta * np.eye(n)
    assert np.linalg.norm(a.cpu().numpy() - astar) / np.linalg.norm(astar) <= kub * _relres(A, y, a.cpu().numpy())
