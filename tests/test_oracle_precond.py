"""Pins for the oracle's preconditioner (Algorithms 1-4) on the CPU.

Anchors: the sketches equal K times an explicitly assembled test matrix; the
pivoted QR agrees with LAPACK's column-pivoted QR and with a greedy brute
force built on an independent orthogonal basis; the Nystrom factor
interpolates the anchor block and satisfies Lemma schur (K - K~ PSD); the
Woodbury apply equals an explicit inverse; the preconditioned spectrum is
bounded below by 1 (proof of Theorem maintheorem) and above by the ID
corollary; a best rank-k factor gives exactly 1 + lam_{k+1}/beta (SVD remark).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import datagen
from oracle import kernel as ok
from oracle import precond as op
from oracle import theory as th


def test_sketch_dense_is_K_times_omega():
    rng = np.random.default_rng(0)
    X = rng.random((120, 3))
    om = datagen.sketch_dense_omega(120, 9, seed=1)
    np.testing.assert_allclose(op.sketch_dense(X, 0.05, om), ok.kernel_matrix(X, X, 0.05) @ om, rtol=1e-12, atol=1e-13)


def test_sketch_sparse_is_K_times_sparse_matrix():
    rng = np.random.default_rng(1)
    X = rng.random((150, 4))
    idx, sign = datagen.sketch_sparse_draws(150, 11, 6, seed=2)
    Om = np.zeros((150, 11))
    for i in range(11):
        for s in range(6):
            Om[idx[i, s], i] += sign[i, s]
    np.testing.assert_allclose(op.sketch_sparse(X, 0.2, idx, sign), ok.kernel_matrix(X, X, 0.2) @ Om, rtol=1e-12, atol=1e-13)
    # the draws themselves: distinct indices per column, Rademacher signs
    assert all(len(set(row)) == 6 for row in idx)
    assert set(np.unique(sign)) <= {-1.0, 1.0}


def test_qrcp_matches_lapack():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((12, 40)) @ np.diag(rng.random(40) * 3)
    ours = op.qrcp(A, 12)
    _, R, P = sla.qr(A, pivoting=True, mode="economic")
    np.testing.assert_array_equal(ours["piv"], P[:12])
    np.testing.assert_allclose(ours["rdiag"], np.abs(np.diag(R)), rtol=1e-10)


def test_qrcp_greedy_brute_force():
    # each pivot maximises the distance of a column to the span of the previous pivots,
    # measured with an orthonormal basis from numpy's (unpivoted) QR
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 25))
    res = op.qrcp(A, 5)
    chosen = []
    for j in range(5):
        if chosen:
            Q, _ = np.linalg.qr(A[:, chosen])
            Rm = A - Q @ (Q.T @ A)
        else:
            Rm = A
        nrm = np.linalg.norm(Rm, axis=0)
        nrm[chosen] = -1
        assert res["piv"][j] == int(np.argmax(nrm))
        np.testing.assert_allclose(res["rdiag"][j], nrm.max(), rtol=1e-12)
        chosen.append(int(res["piv"][j]))


def test_qrcp_rank_revealing_and_forced():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((10, 3)) @ rng.standard_normal((3, 30))   # rank 3
    res = op.qrcp(A, 5)
    assert res["rdiag"][2] > 1e-3 and res["rdiag"][3] < 1e-10 * res["rdiag"][0]
    forced = op.qrcp(A, 5, forced=res["piv"])
    np.testing.assert_array_equal(forced["piv"], res["piv"])
    np.testing.assert_allclose(forced["rdiag"], res["maxnorm"][:5], rtol=1e-12, atol=1e-14)
    # a non-greedy forced sequence is reported as such
    alt = op.qrcp(A, 3, forced=[res["piv"][1], res["piv"][0], res["piv"][2]])
    assert alt["rdiag"][0] <= alt["maxnorm"][0]


def test_qrcp_ties_lowest_index():
    A = np.array([[1.0, 0.0, 1.0, 0.0], [0.0, 1.0, 0.0, 1.0]])
    np.testing.assert_array_equal(op.qrcp(A, 2)["piv"], [0, 1])


@pytest.fixture(scope="module")
def small_problem():
    rng = np.random.default_rng(5)
    X = rng.random((220, 3))
    eps = 0.05
    om = datagen.sketch_dense_omega(220, 40, seed=6)
    Y = op.sketch_dense(X, eps, om)
    S = op.anchor_selection(Y, 30)
    return X, eps, S


def test_nystrom_factor_properties(small_problem):
    X, eps, S = small_problem
    nf = op.nystrom_factor(X, S, eps)
    W = nf["W"]
    K = ok.kernel_matrix(X, X, eps)
    C = K[:, S]
    Kss = K[np.ix_(S, S)]
    Kt = W @ W.T
    # C U C^T with U = K_SS^{-1} (paper's Sec. 3 reading), and the symmetric square root form
    np.testing.assert_allclose(Kt, C @ np.linalg.solve(Kss, C.T), atol=1e-8)
    Uh = op.symmetric_sqrt_inv(Kss)
    np.testing.assert_allclose(Kt, (C @ Uh) @ (C @ Uh).T, atol=1e-8)
    # Nystrom interpolates the anchor block exactly
    np.testing.assert_allclose(Kt[np.ix_(S, S)], Kss, atol=1e-9)
    # Lemma schur: K - K~ >= 0
    assert np.linalg.eigvalsh(K - Kt).min() > -1e-9


def test_woodbury_against_explicit_inverse(small_problem):
    X, eps, S = small_problem
    nf = op.nystrom_factor(X, S, eps)
    W = nf["W"]
    beta = 1e-3
    L = op.core_cholesky(W, beta)
    np.testing.assert_allclose(L @ L.T, beta * np.eye(W.shape[1]) + W.T @ W, rtol=1e-13, atol=1e-12)
    x = np.random.default_rng(7).standard_normal(X.shape[0])
    explicit = np.linalg.inv(W @ W.T + beta * np.eye(X.shape[0])) @ x
    got = op.woodbury_apply(W, L, beta, x)
    np.testing.assert_allclose(got, explicit, rtol=1e-9, atol=1e-9 * np.abs(explicit).max())
    K = ok.kernel_matrix(X, X, eps)
    unst = op.woodbury_apply_unstabilised(K[:, S], K[np.ix_(S, S)], beta, x)
    np.testing.assert_allclose(unst, got, rtol=1e-6, atol=1e-6 * np.abs(got).max())


def test_preconditioned_spectrum_bounds(small_problem):
    X, eps, S = small_problem
    beta = 1e-3
    K = ok.kernel_matrix(X, X, eps)
    W = op.nystrom_factor(X, S, eps)["W"]
    ev = op.preconditioned_spectrum(K, W, beta)
    assert ev.min() >= 1 - 1e-8                                    # K~ + bI <= K + bI
    lamK = np.linalg.eigvalsh(K)[::-1]
    k, n = len(S), K.shape[0]
    tight, loose = th.cond_bound_id(lamK[k], k, n, beta)
    cond = ev.max() / ev.min()
    assert cond <= tight <= loose
    # SVD remark: best rank-k factor gives exactly 1 + lam_{k+1}/beta
    lam, V = np.linalg.eigh(K)
    Wb = V[:, -k:] * np.sqrt(lam[-k:])
    evb = op.preconditioned_spectrum(K, Wb, beta)
    np.testing.assert_allclose(evb.max() / evb.min(), th.cond_svd(lam[-k - 1], beta), rtol=1e-7)
    assert cond >= th.cond_svd(lam[-k - 1], beta) * (1 - 1e-8)     # no rank-k Nystrom beats the optimum


def test_full_rank_preconditioner_is_exact():
    rng = np.random.default_rng(8)
    X = rng.random((40, 2))
    eps, beta = 0.02, 1e-2                       # K well conditioned: K_SS = K is inverted exactly
    P = op.build_precond(X, eps, [beta], 40, omega=datagen.sketch_dense_omega(40, 40, 9), tau=0.0)
    K = ok.kernel_matrix(X, X, eps)
    x = rng.standard_normal(40)
    np.testing.assert_allclose(op.apply_precond(P, beta, (K + beta * np.eye(40)) @ x), x, rtol=1e-6)


# ---------------------------------------------------------------- other anchor choices (remark in Sec. 3)
def test_fps_on_a_line_bisects():
    # 17 points at 0, 1, ..., 16 starting from 0: the far end, then the midpoint, then the
    # quarter points, eighth points and the odd points, each level left to right (ties -> lowest index)
    X = np.arange(17, dtype=np.float64)[:, None]
    S, dsel = op.fps(X, 17, start=0)
    np.testing.assert_array_equal(S, [0, 16, 8, 4, 12, 2, 6, 10, 14, 1, 3, 5, 7, 9, 11, 13, 15])
    np.testing.assert_array_equal(dsel[1:], [256, 64, 16, 16, 4, 4, 4, 4] + [1] * 8)
    assert np.isinf(dsel[0])


def test_fps_k_center_two_approximation():
    # FPS is Gonzalez's greedy k-center rule: its covering radius is at most twice the optimum,
    # found here by brute force over every k-subset
    import itertools
    rng = np.random.default_rng(11)
    for trial in range(4):
        X = rng.random((11, 2))
        D = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
        for k in (2, 3, 4):
            S, _ = op.fps(X, k, start=trial)
            r_fps = D[:, S].min(axis=1).max()
            r_opt = min(D[:, list(c)].min(axis=1).max() for c in itertools.combinations(range(11), k))
            assert r_opt <= r_fps + 1e-15 and r_fps <= 2 * r_opt + 1e-12


def test_fps_separation_and_monotone():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((300, 3))
    S, dsel = op.fps(X, 40, start=7)
    assert len(set(S.tolist())) == 40 and S[0] == 7
    assert np.all(np.diff(dsel[1:]) <= 0)                     # the pick distance never grows
    for j in range(1, 40):
        # pick j is exactly dsel[j] away from its nearest earlier pick, and no point is farther
        d2 = ((X[S[:j]] - X[S[j]]) ** 2).sum(-1)
        np.testing.assert_allclose(d2.min(), dsel[j], rtol=1e-14)
        dall = ((X[:, None, :] - X[None, S[:j], :]) ** 2).sum(-1).min(axis=1)
        assert dall.max() <= dsel[j] * (1 + 1e-14)


def test_fps_duplicates_give_distinct_indices():
    X = np.ones((6, 2))
    S, dsel = op.fps(X, 6, start=3)
    np.testing.assert_array_equal(S, [3, 0, 1, 2, 4, 5])
    np.testing.assert_array_equal(dsel[1:], 0.0)


def test_anchors_given_all_points_reproduce_K():
    # every point an anchor: the Nystrom approximation is K itself, so the preconditioner inverts K + bI
    rng = np.random.default_rng(13)
    X = rng.random((50, 2))
    eps, beta = 0.02, 1e-2
    S = datagen.random_anchors(50, 50, seed=14)
    assert sorted(S.tolist()) == list(range(50))
    P = op.build_precond_from_anchors(X, eps, [beta], S, tau=0.0)
    K = ok.kernel_matrix(X, X, eps)
    np.testing.assert_allclose(P["W"] @ P["W"].T, K, atol=1e-10)
    x = rng.standard_normal(50)
    np.testing.assert_allclose(op.apply_precond(P, beta, (K + beta * np.eye(50)) @ x), x, rtol=1e-6)


@pytest.mark.parametrize("how", ["random", "fps"])
def test_anchors_given_nystrom_properties(how):
    # any anchor set: K~ interpolates the anchor block, K - K~ is PSD (Lemma schur) and the
    # preconditioned spectrum stays at or above 1
    rng = np.random.default_rng(15)
    X = rng.random((200, 3))
    eps, beta = 0.05, 1e-3
    S = datagen.random_anchors(200, 25, seed=16) if how == "random" else op.fps(X, 25, start=0)[0]
    P = op.build_precond_from_anchors(X, eps, [beta], S)
    K = ok.kernel_matrix(X, X, eps)
    Kt = P["W"] @ P["W"].T
    np.testing.assert_allclose(Kt[np.ix_(S, S)], K[np.ix_(S, S)], atol=1e-9)
    assert np.linalg.eigvalsh(K - Kt).min() > -1e-9
    assert op.preconditioned_spectrum(K, P["W"], beta).min() >= 1 - 1e-8
