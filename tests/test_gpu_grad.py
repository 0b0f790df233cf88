"""GPU parity of the adjoint gradient (krr_grad) and its torch.autograd wrapper.

References: the oracle's dense adjoint (Cholesky solves in FP64), central finite differences
(h = 1e-4 in log space) of the oracle's dense loss, and the closed form checks the oracle itself is
pinned by.  The adjoint workload (n=200,000 train, 20,000 validation, d=16, eps=4, beta=1e-2) is
checked on its first 5,000 training and 500 validation points, where dense FP64 solves are cheap.
"""
import math

import numpy as np
import pytest
import torch

import datagen
from oracle import adjoint as oa


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.gpu
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("fp32", 3e-5), ("mixed", 3e-5)])
def test_grad_matches_dense_adjoint(gpu_lib, prec, tol):
    rng = np.random.default_rng(0)
    w = rng.standard_normal(3)
    Xtr, Xv = 0.5 * rng.standard_normal((600, 3)), 0.5 * rng.standard_normal((150, 3))
    ytr, yv = np.tanh(Xtr @ w) + 0.1 * rng.standard_normal(600), np.tanh(Xv @ w)
    eps, beta = 0.5, 1e-2
    L, ge, gb, alpha_ref, lam_ref = oa.val_loss_grad(Xtr, ytr, Xv, yv, eps, beta)
    # plain CG (no preconditioner); kappa(K + beta I) ~ 3e4 bounds the attainable residual near 1e-12
    g = gpu_lib.grad(*(torch.from_numpy(a) for a in (Xtr, ytr, Xv, yv)), eps, beta, None,
                     tol=1e-11, maxit=20000,
                     replace_every=10 if prec != "fp64" else 0, prec=prec)
    print(f"{prec}: loss {g[0]:.12g} vs {L:.12g}; dlogeps {g[1]:.10g} vs {ge:.10g}; dlogbeta {g[2]:.10g} vs {gb:.10g}")
    assert _rel(g[0], L) <= tol and _rel(g[1], ge) <= tol and _rel(g[2], gb) <= tol
    np.testing.assert_allclose(g[3].cpu().numpy(), alpha_ref, rtol=0, atol=tol * 10 * np.abs(alpha_ref).max())


@pytest.fixture(scope="module")
def adjoint_subset():
    wl = datagen.subset(datagen.make_workload("adjoint"), 5000, 500)
    L, ge, gb, _, _ = oa.val_loss_grad(wl.X, wl.y, wl.X_val, wl.y_val, wl.eps, wl.betas[0])
    fe, fb = oa.fd_grad(wl.X, wl.y, wl.X_val, wl.y_val, wl.eps, wl.betas[0], h=1e-4)
    return wl, (L, ge, gb), (fe, fb)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_grad_adjoint_workload_subset_vs_fd(gpu_lib, adjoint_subset, prec):
    """5,000 / 500 subset of the adjoint workload: adjoint PCG gradients vs central FD to 1e-4."""
    wl, (L, ge, gb), (fe, fb) = adjoint_subset
    beta = wl.betas[0]
    idx, sign = datagen.sketch_sparse_draws(wl.n, 520, 32, seed=datagen.sketch_seed("adjoint"))
    P = gpu_lib.Preconditioner(torch.from_numpy(wl.X), wl.eps, [beta], 500, 520, idx=torch.from_numpy(idx),
                               sign=torch.from_numpy(sign), prec=prec)
    g = gpu_lib.grad(torch.from_numpy(wl.X), torch.from_numpy(wl.y), torch.from_numpy(wl.X_val),
                     torch.from_numpy(wl.y_val), wl.eps, beta, P, tol=1e-10, maxit=20000,
                     replace_every=10 if prec != "fp64" else 0, prec=prec)
    print(f"{prec}: dL/dlogeps {g[1]:.8g} (adjoint ref {ge:.8g}, FD {fe:.8g}); "
          f"dL/dlogbeta {g[2]:.8g} (adjoint ref {gb:.8g}, FD {fb:.8g})")
    assert _rel(g[1], fe) <= 1e-4 and _rel(g[2], fb) <= 1e-4
    bar = 1e-6 if prec == "fp64" else 3e-5      # mixed-precision products in the gradient assembly
    assert _rel(g[1], ge) <= bar and _rel(g[2], gb) <= bar
    assert _rel(g[0], L) <= (1e-8 if prec == "fp64" else 1e-6)


@pytest.mark.gpu
def test_autograd_function(gpu_lib):
    rng = np.random.default_rng(2)
    Xtr, Xv = rng.random((400, 2)), rng.random((90, 2))
    ytr, yv = np.sin(3 * Xtr[:, 0]), np.sin(3 * Xv[:, 0])
    le = torch.tensor(math.log(0.1), dtype=torch.float64, device="cuda", requires_grad=True)
    lb = torch.tensor(math.log(1e-2), dtype=torch.float64, device="cuda", requires_grad=True)
    args = [torch.from_numpy(a).cuda() for a in (Xtr, ytr, Xv, yv)]
    loss = gpu_lib.KRRValLoss.apply(le, lb, *args, None, {"tol": 1e-11, "maxit": 20000})
    loss.backward()
    L, ge, gb, _, _ = oa.val_loss_grad(Xtr, ytr, Xv, yv, 0.1, 1e-2)
    assert _rel(loss.item(), L) <= 1e-8
    assert _rel(le.grad.item(), ge) <= 1e-6 and _rel(lb.grad.item(), gb) <= 1e-6
