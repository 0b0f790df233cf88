"""GPU parity of the preconditioner build and apply (Algorithms 1-4) against the oracle.

* Sketches (Algorithm 1 dense, Algorithm 2 sparse) element by element.
* Pivoted QR: the pivots are an argmax decided in floating point, so they are checked as valid
  greedy choices: the oracle's Householder QR is run forced along the GPU's pivot sequence and at
  every step the GPU's pivot must attain the largest residual norm (to 1e-10 relative, FP64), and
  |R_jj| must match.  On inputs without near-ties the pivots must be identical.
* The Nystrom factor is compared through what is unique: W W^T = C K_SS^+ C^T for the GPU's anchors
  (column signs and order of W depend on the eigensolver).
* The Woodbury apply against the oracle's apply for the same anchors and against an explicit inverse.
* Lemma schur consequence: the preconditioned spectrum is >= 1.
"""
import numpy as np
import pytest
import torch

import datagen
from oracle import kernel as ok
from oracle import precond as op


def _pts(n, d, seed):
    return np.random.default_rng(seed).random((n, d))


@pytest.mark.gpu
# mixed: the l sketch columns go through the block MVM (two BF16 parts of K and Omega; measured 3e-6)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6), ("mixed", 1e-5)])
@pytest.mark.parametrize("l", [37, 300])     # 300: two column chunks (256 + 44)
def test_sketch_dense_parity(gpu_lib, prec, tol, l):
    X = _pts(1300, 3, 1)
    om = datagen.sketch_dense_omega(1300, l, seed=2)
    ref = op.sketch_dense(X, 0.05, om)
    scale = ok.kernel_matrix(X, X, 0.05) @ np.abs(om)
    Y = gpu_lib.sketch(torch.from_numpy(X), 0.05, omega=torch.from_numpy(om), prec=prec).cpu().numpy()
    err = np.max(np.abs(Y - ref) / scale)
    print(f"dense sketch {prec}: max scaled error {err:.2e}")
    assert err <= tol


@pytest.mark.gpu
# FP32: the relative error of exp(-q) computed in FP32 grows like q * 2^-23; rows whose 9 sketch
# points are all far away sum only such entries (measured 1.2e-5).
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 5e-5)])
def test_sketch_sparse_parity(gpu_lib, prec, tol):
    X = _pts(2100, 4, 3)
    idx, sign = datagen.sketch_sparse_draws(2100, 53, 9, seed=4)
    ref = op.sketch_sparse(X, 0.02, idx, sign)
    Om = np.zeros((2100, 53))
    for i in range(53):
        np.add.at(Om[:, i], idx[i], np.abs(sign[i]))
    scale = ok.kernel_matrix(X, X, 0.02) @ Om
    Y = gpu_lib.sketch(torch.from_numpy(X), 0.02, idx=torch.from_numpy(idx), sign=torch.from_numpy(sign),
                       prec=prec).cpu().numpy()
    err = np.max(np.abs(Y - ref) / scale)
    print(f"sparse sketch {prec}: max scaled error {err:.2e}")
    assert err <= tol


@pytest.mark.gpu
def test_qrcp_identical_without_ties(gpu_lib):
    rng = np.random.default_rng(5)
    # column norms spread over decades: no near-ties anywhere in the greedy sequence
    Y = rng.standard_normal((900, 30)) * np.exp(rng.uniform(-3, 3, size=(900, 1)))
    piv, rd = gpu_lib.qrcp(torch.from_numpy(Y), 25, prec="fp64")
    ref = op.qrcp(Y.T, 25)
    np.testing.assert_array_equal(piv.cpu().numpy(), ref["piv"])
    np.testing.assert_allclose(rd.cpu().numpy(), ref["rdiag"], rtol=1e-10)


@pytest.mark.gpu
@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_qrcp_valid_greedy_on_sketch(gpu_lib, prec, rtol):
    X = _pts(2000, 3, 6)
    om = datagen.sketch_dense_omega(2000, 170, seed=101)
    Y = op.sketch_dense(X, 0.05, om)
    piv, rd = gpu_lib.qrcp(torch.from_numpy(Y), 150, prec=prec)
    piv = piv.cpu().numpy()
    assert len(set(piv.tolist())) == 150
    forced = op.qrcp(Y.T, 150, forced=piv)
    # each pivot attains the largest residual norm among unselected columns
    assert np.all(forced["rdiag"] >= forced["maxnorm"] * (1 - rtol))
    np.testing.assert_allclose(rd.cpu().numpy(), forced["rdiag"], rtol=max(rtol, 1e-9) * 10,
                               atol=1e-12 * forced["rdiag"][0])


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_qrcp_candidates_match_full_pass(gpu_lib, prec, monkeypatch):
    """The candidate-set pivoting (exact norms for the top candidates, stale upper bounds for the rest,
    batched refresh passes) against one pass over the sketch per step: same pivots; and valid greedy
    pivots for the oracle's Householder QR run along them.  30,000 columns, so the candidate set (1024)
    is a small part and picks fall outside it (refreshes before the batch limit)."""
    n, l, k = 30_000, 320, 300
    X = _pts(n, 3, 60)
    idx, sign = datagen.sketch_sparse_draws(n, l, 8, seed=61)
    Y = gpu_lib.sketch(torch.from_numpy(X), 0.01, idx=torch.from_numpy(idx), sign=torch.from_numpy(sign),
                       prec="fp64")
    monkeypatch.setenv("KRR_QR_VERBOSE", "1")
    piv_c, rd_c = gpu_lib.qrcp(Y, k, prec=prec)
    monkeypatch.setenv("KRR_QR_FULL", "1")
    piv_f, rd_f = gpu_lib.qrcp(Y, k, prec=prec)
    monkeypatch.delenv("KRR_QR_FULL")
    piv_c, piv_f = piv_c.cpu().numpy(), piv_f.cpu().numpy()
    np.testing.assert_array_equal(piv_c, piv_f)
    np.testing.assert_allclose(rd_c.cpu().numpy(), rd_f.cpu().numpy(), rtol=1e-9)
    forced = op.qrcp(Y.cpu().numpy().T, k, forced=piv_c)
    assert np.all(forced["rdiag"] >= forced["maxnorm"] * (1 - (1e-10 if prec == "fp64" else 1e-4)))


@pytest.fixture(scope="module")
def small_build(gpu_lib):
    wl = datagen.make_workload("small")
    om = datagen.sketch_dense_omega(wl.n, wl.l, datagen.sketch_seed("small"))
    P = gpu_lib.Preconditioner(torch.from_numpy(wl.X), wl.eps, [wl.betas[0], 1e-2], wl.k, wl.l,
                               omega=torch.from_numpy(om), prec="mixed", keep_sketch=True)
    return wl, om, P


@pytest.mark.gpu
def test_build_anchors_and_factor(gpu_lib, small_build):
    wl, om, P = small_build
    info = P.info()
    S = np.array(info["S"])
    ref = op.build_precond(wl.X, wl.eps, [wl.betas[0]], wl.k, omega=om)
    # the sketch used by the build equals the oracle's (mixed build: block MVM, two BF16 parts)
    Ysk = P.get(P.SKETCH).cpu().numpy()
    np.testing.assert_allclose(Ysk, ref["Y"], rtol=0, atol=5e-5 * np.abs(ref["Y"]).max())
    # anchors: valid greedy pivots of the oracle's sketch (the build's sketch ran in FP32 here)
    forced = op.qrcp(ref["Y"].T, wl.k, forced=S)
    assert np.all(forced["rdiag"] >= forced["maxnorm"] * (1 - 1e-4))
    # W W^T equals C K_SS^+ C^T for these anchors
    W = P.get(P.W64).cpu().numpy()
    nf = op.nystrom_factor(wl.X, S, wl.eps)
    Kt_ref = nf["W"] @ nf["W"].T
    np.testing.assert_allclose(W @ W.T, Kt_ref, rtol=0, atol=1e-9)
    assert info["kept"] == nf["kept"]
    lam = np.array(info["lam"])
    np.testing.assert_allclose(lam, np.sort(nf["lam"]), rtol=1e-9, atol=1e-12 * lam.max())
    # the FP32 copy is the rounded FP64 factor
    W32 = P.get(P.W32).cpu().numpy()
    np.testing.assert_array_equal(W32, W.astype(np.float32))
    # Cholesky factor: L L^T = beta I + W^T W
    L = P.get(P.LCORE, 0).cpu().numpy().T     # column-major storage
    M = W.T @ W
    np.testing.assert_allclose(L @ L.T, wl.betas[0] * np.eye(M.shape[0]) + M, rtol=1e-12, atol=1e-10)
    assert np.allclose(L, np.tril(L))


@pytest.mark.gpu
# k = 40: scalar Jacobi rounds; k = 700: blocks of 8 columns; k = 1500: blocks of 4 columns (the LDS
# holds a pair of blocks); the partial last block and the bye block occur at 700 and 1500.  eps is set
# so that K_SS stays well conditioned (no eigenvalue near the truncation threshold).
@pytest.mark.parametrize("k,eps", [(40, 0.02), (700, 0.004), (1500, 0.003)])
def test_anchor_evd_paths(gpu_lib, k, eps):
    """The eigendecomposition of K_SS on every code path: eigenvalues and W W^T = C K_SS^+ C^T against the
    oracle for the GPU's anchors."""
    n, d = 3500, 3
    X = _pts(n, d, 40 + k)
    l = k + 20
    idx, sign = datagen.sketch_sparse_draws(n, l, 8, seed=41 + k)
    P = gpu_lib.Preconditioner(torch.from_numpy(X), eps, [1e-3], k, l, idx=torch.from_numpy(idx),
                               sign=torch.from_numpy(sign), prec="fp64")
    info = P.info()
    S = np.array(info["S"])
    nf = op.nystrom_factor(X, S, eps)
    lam = np.array(info["lam"])
    print(f"k={k}: {info['kept']} eigenvalues kept (oracle {nf['kept']}), sweeps {P.timings()['jacobi_sweeps']}")
    np.testing.assert_allclose(lam, np.sort(nf["lam"]), rtol=1e-9, atol=1e-12 * lam.max())
    assert info["kept"] == nf["kept"]
    W = P.get(P.W64).cpu().numpy()
    np.testing.assert_allclose(W @ W.T, nf["W"] @ nf["W"].T, rtol=0, atol=1e-9)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_woodbury_apply_parity(gpu_lib, small_build, prec):
    wl, om, P = small_build
    S = np.array(P.info()["S"])
    W = P.get(P.W64).cpu().numpy()
    if prec == "mixed":
        W = P.get(P.W32).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((wl.n, 3))
    betas = [wl.betas[0], 1e-2, wl.betas[0]]
    got = P.apply(torch.from_numpy(x), betas=betas, prec=prec).cpu().numpy()
    for c, b in enumerate(betas):
        Lb = op.core_cholesky(W, b)
        ref = op.woodbury_apply(W, Lb, b, x[:, c])
        err = np.linalg.norm(got[:, c] - ref) / np.linalg.norm(ref)
        print(f"woodbury {prec} beta={b}: rel err {err:.2e}")
        assert err <= (1e-9 if prec == "fp64" else 1e-5)
    # single-column path
    one = P.apply(torch.from_numpy(x[:, 0].copy()), betas=[betas[0]], prec=prec).cpu().numpy()
    np.testing.assert_allclose(one, got[:, 0], rtol=1e-6, atol=1e-6 * np.abs(got[:, 0]).max())
    # explicit inverse on the same factor
    if prec == "fp64":
        Pm = W @ W.T + betas[0] * np.eye(wl.n)
        exp = np.linalg.solve(Pm, x[:, 0])
        assert np.linalg.norm(one - exp) / np.linalg.norm(exp) < 1e-8


@pytest.mark.gpu
def test_preconditioned_spectrum_at_least_one(gpu_lib):
    X = _pts(400, 2, 8)
    eps, beta = 0.05, 1e-3
    om = datagen.sketch_dense_omega(400, 40, seed=9)
    P = gpu_lib.Preconditioner(torch.from_numpy(X), eps, [beta], 30, 40, omega=torch.from_numpy(om), prec="fp64")
    Minv = P.apply(torch.eye(400, dtype=torch.float64), betas=[beta] * 400).cpu().numpy()
    A = ok.kernel_matrix(X, X, eps) + beta * np.eye(400)
    ev = np.linalg.eigvals(Minv @ A).real
    assert ev.min() >= 1 - 1e-8
    np.testing.assert_allclose(Minv, Minv.T, atol=1e-8 * np.abs(Minv).max())


@pytest.mark.gpu
def test_precond_rejects_bad_arguments(gpu_lib):
    X = torch.from_numpy(_pts(100, 2, 10))
    om = torch.from_numpy(datagen.sketch_dense_omega(100, 10, seed=1))
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.Preconditioner(X, 0.1, [1e-3], 11, 10, omega=om)           # k > l
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.Preconditioner(X, 0.1, [-1.0], 5, 10, omega=om)            # beta <= 0
    idx = torch.full((10, 3), 100, dtype=torch.int64)                      # index out of range
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.Preconditioner(X, 0.1, [1e-3], 5, 10, idx=idx, sign=torch.ones(10, 3, dtype=torch.float64))
    P = gpu_lib.Preconditioner(X, 0.1, [1e-3], 5, 10, omega=om)
    with pytest.raises(gpu_lib.KRRError):
        P.apply(torch.ones(100, dtype=torch.float64), betas=[0.5])       # beta not in the handle
