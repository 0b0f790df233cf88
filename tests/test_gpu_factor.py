"""The Nystrom factor and the Woodbury products on the library's FP64 matrix-core kernels (Algorithm 3:
W = C U^{1/2} with the kernel block applied inside the product, M = W^T W, the core inverse from the
Cholesky factor; Algorithm 4 for several right-hand sides), against the oracle.

Sizes span several 128-wide tiles with ragged last tiles, several row splits, every column-tile width of
the several-column apply (16, 32, 64, 128) and the kernel-block fallback for d > 16 (C formed, then C T).
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
@pytest.mark.parametrize("n,d,k,eps,prec", [(3100, 3, 300, 0.01, "mixed"), (2000, 20, 130, 2.0, "fp64"),
                                            (1500, 6, 257, 0.08, "fp32")])
def test_factor_and_core_against_oracle(gpu_lib, n, d, k, eps, prec):
    X = _pts(n, d, 50 + d)
    rng = np.random.default_rng(51)
    S = rng.choice(n, size=k, replace=False).astype(np.int64)
    beta = 1e-3
    P = gpu_lib.Preconditioner(torch.from_numpy(X), eps, [beta, 0.1], k, anchors=torch.from_numpy(S), prec=prec)
    ref = op.build_precond_from_anchors(X, eps, [beta], S)
    info = P.info()
    assert info["kept"] == ref["kept"]
    W = P.get(P.W64).cpu().numpy()
    Kt = ref["W"] @ ref["W"].T
    err = np.abs(W @ W.T - Kt).max()
    print(f"n={n} d={d} k={k}: kept {info['kept']}, max |W W^T - C K_SS^+ C^T| = {err:.2e}")
    assert err <= 1e-9
    # M = W^T W from the device's own W, exactly symmetric
    M = P.get(P.MCORE).cpu().numpy()
    Mref = W.T @ W
    np.testing.assert_allclose(M, Mref, rtol=0, atol=1e-12 * np.abs(Mref).max())
    assert np.array_equal(M, M.T)
    # Cholesky factor of beta I + M for both betas
    for b, beta_b in enumerate((beta, 0.1)):
        L = P.get(P.LCORE, b).cpu().numpy().T
        np.testing.assert_allclose(L @ L.T, beta_b * np.eye(M.shape[0]) + M, rtol=1e-12, atol=1e-10)
    if prec != "fp64":
        W32 = P.get(P.W32).cpu().numpy()
        np.testing.assert_array_equal(W32, W.astype(np.float32))


@pytest.mark.gpu
@pytest.mark.parametrize("R", [5, 40, 130])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_block_woodbury_every_tile_width(gpu_lib, R, prec):
    n, d, k, eps = 2600, 3, 200, 0.02
    X = _pts(n, d, 60)
    idx, sign = datagen.sketch_sparse_draws(n, k + 20, 16, 61)
    betas_all = [1e-3, 1e-2, 1e-1]
    P = gpu_lib.Preconditioner(torch.from_numpy(X), eps, betas_all, k, k + 20, idx=torch.from_numpy(idx),
                               sign=torch.from_numpy(sign), prec=prec)
    W = (P.get(P.W32).cpu().numpy().astype(np.float64) if prec == "mixed" else P.get(P.W64).cpu().numpy())
    x = np.random.default_rng(62).standard_normal((n, R))
    betas = [betas_all[c % 3] for c in range(R)]
    got = P.apply(torch.from_numpy(x), betas=betas, prec=prec).cpu().numpy()
    Ls = {b: op.core_cholesky(W, b) for b in betas_all}
    worst = 0.0
    for c in range(R):
        ref = op.woodbury_apply(W, Ls[betas[c]], betas[c], x[:, c])
        worst = max(worst, np.linalg.norm(got[:, c] - ref) / np.linalg.norm(ref))
    print(f"R={R} {prec}: worst column rel err {worst:.2e}")
    assert worst <= 1e-10
    # each column equals the one-column path (hand-written GEMV kernels) on the same factor
    for c in (0, R - 1):
        one = P.apply(torch.from_numpy(x[:, c].copy()), betas=[betas[c]], prec=prec).cpu().numpy()
        assert np.linalg.norm(one - got[:, c]) / np.linalg.norm(one) <= 1e-12
