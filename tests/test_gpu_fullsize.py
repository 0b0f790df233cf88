"""Parity at the workloads' full sizes, in the launch configuration the benchmark uses.

The oracle cannot form these products whole, so outputs are checked on sampled rows it computes one by
one (exact FP64 sums over all n sources); the preconditioner's factor on sampled rows of W W^T against the
oracle's own EVD of the anchor block (given the GPU's anchors), and its apply through a property that holds
at any size: applying it to (W W^T + beta I) x returns x.
"""
import numpy as np
import pytest
import torch

import datagen
from oracle import kernel as ok

ROWS = 48


def _sampled(Xt, Xs, eps, V, rows):
    ref = ok.kernel_mv(Xt[rows], Xs, eps, V)
    scale = ok.kernel_mv(Xt[rows], Xs, eps, np.abs(V))
    return ref, scale


def _check(U, rows, ref, scale, tol, label):
    Us = U[rows]
    err = float(np.max(np.abs(Us - ref) / scale))
    print(f"{label}: max scaled error on {len(rows)} sampled rows {err:.2e}", flush=True)
    assert err <= tol


@pytest.mark.gpu
@pytest.mark.parametrize("prec,tol", [("mixed", 2e-6), ("fp64", 1e-14)])
def test_mixed_workload_mvm(gpu_lib, prec, tol):
    """n = 1,000,000, d = 4, eps = 0.01: the solver's operator (K + beta I) v."""
    wl = datagen.make_workload("mixed")
    rng = np.random.default_rng(11)
    v = rng.standard_normal(wl.n)
    rows = np.sort(rng.choice(wl.n, ROWS, replace=False))
    print(f"mixed workload n={wl.n} prec={prec}", flush=True)
    U = gpu_lib.kernel_mv(torch.from_numpy(wl.X), None, wl.eps, torch.from_numpy(v), shift=wl.betas[0],
                          prec=prec).cpu().numpy()
    ref, scale = _sampled(wl.X, wl.X, wl.eps, v, rows)
    ref = ref + wl.betas[0] * v[rows]
    scale = scale + wl.betas[0] * np.abs(v[rows])
    _check(U, rows, ref, scale, tol, f"mixed workload {prec}")


@pytest.mark.gpu
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("fp64", 1e-14), ("mixed", 2e-6)])
def test_fp32_workload_mvm(gpu_lib, prec, tol):
    """n = 100,000, d = 8, eps = 0.2, Gaussian-mixture points."""
    wl = datagen.make_workload("fp32")
    rng = np.random.default_rng(12)
    v = rng.standard_normal(wl.n)
    rows = np.sort(rng.choice(wl.n, ROWS, replace=False))
    U = gpu_lib.kernel_mv(torch.from_numpy(wl.X), None, wl.eps, torch.from_numpy(v), prec=prec).cpu().numpy()
    ref, scale = _sampled(wl.X, wl.X, wl.eps, v, rows)
    _check(U, rows, ref, scale, tol, f"fp32 workload {prec}")


@pytest.mark.gpu
def test_block_workload_mvm(gpu_lib):
    """n = 500,000, d = 6, 128 right-hand sides: the block MVM (MFMA K.V contraction)."""
    wl = datagen.make_workload("block")
    rows = np.sort(np.random.default_rng(13).choice(wl.n, 16, replace=False))
    U = gpu_lib.kernel_mv(torch.from_numpy(wl.X), None, wl.eps, torch.from_numpy(wl.y), prec="mixed").cpu().numpy()
    ref, scale = _sampled(wl.X, wl.X, wl.eps, wl.y, rows)
    _check(U, rows, ref, scale, 5e-6, "block workload mixed R=128")


@pytest.mark.gpu
def test_block_workload_fp64_replacement_product(gpu_lib):
    """n = 500,000, d = 6, 128 right-hand sides in FP64: the block solve's residual-replacement product
    (FP64 matrix-core kernel), with the per-column ridge shifts of the four beta values.

    Bar: each block sums its source range (at most 65,536 sources) recursively in FP64, so the rounding
    error of a row has a standard deviation of about sqrt(m) u = 256 x 1.1e-16 = 2.8e-14 of sum |K v|
    (worst case m u = 7e-12); 2e-13 is about 7 standard deviations."""
    wl = datagen.make_workload("block")
    R = wl.y.shape[1]
    betas = np.repeat(np.asarray(wl.betas, dtype=np.float64), R // len(wl.betas))
    assert gpu_lib.kmv_variant(wl.d, R, "fp64", square=True) == (3, False)
    rows = np.sort(np.random.default_rng(14).choice(wl.n, 16, replace=False))
    U = gpu_lib.kernel_mv(torch.from_numpy(wl.X), None, wl.eps, torch.from_numpy(wl.y), shift=list(betas),
                          prec="fp64").cpu().numpy()
    ref, scale = _sampled(wl.X, wl.X, wl.eps, wl.y, rows)
    ref = ref + betas * wl.y[rows]
    scale = scale + betas * np.abs(wl.y[rows])
    _check(U, rows, ref, scale, 2e-13, "block workload fp64 R=128 (+ ridge shifts)")


@pytest.mark.gpu
def test_adjoint_workload_cross_products(gpu_lib):
    """Validation x training products of the adjoint workload (20,000 x 200,000, d = 16), fused (K, K')."""
    wl = datagen.make_workload("adjoint")
    rng = np.random.default_rng(14)
    a = rng.standard_normal(wl.n)
    rows = np.sort(rng.choice(wl.X_val.shape[0], ROWS, replace=False))
    U = gpu_lib.kernel_mv(torch.from_numpy(wl.X_val), torch.from_numpy(wl.X), wl.eps, torch.from_numpy(a),
                          deriv=2, prec="fp64").cpu().numpy()
    ref = ok.kernel_mv(wl.X_val[rows], wl.X, wl.eps, a, deriv=2)
    scale = ok.kernel_mv(wl.X_val[rows], wl.X, wl.eps, np.abs(a), deriv=2)
    for c in range(2):
        _check(U[:, c], rows, ref[c], scale[c], 1e-13, f"adjoint workload {'K' if c == 0 else 'Kprime'} fp64")


@pytest.mark.gpu
def test_fp32_workload_preconditioner_inverts_its_operator(gpu_lib):
    """Built at full size (n = 100,000, k = 1000, Algorithm 2): P^{-1} (W W^T + beta I) x = x."""
    wl = datagen.make_workload("fp32")
    beta = wl.betas[0]
    idx, sign = datagen.sketch_sparse_draws(wl.n, wl.l, wl.r, datagen.sketch_seed("fp32"))
    P = gpu_lib.Preconditioner(torch.from_numpy(wl.X), wl.eps, [beta], wl.k, wl.l, idx=torch.from_numpy(idx),
                               sign=torch.from_numpy(sign), prec="mixed")
    info = P.info()
    assert len(set(info["S"])) == wl.k and info["kept"] >= 1
    for which, prec, tol in ((P.W64, "fp64", 1e-9), (P.W32, "mixed", 1e-6)):
        W = P.get(which).double()
        x = torch.randn(wl.n, dtype=torch.float64, device="cuda")
        b = W @ (W.T @ x) + beta * x
        got = P.apply(b, betas=[beta], prec=prec)
        err = float(torch.linalg.norm(got - x) / torch.linalg.norm(x))
        print(f"fp32 workload preconditioner {prec}: ||P^-1 (WW^T + bI) x - x|| / ||x|| = {err:.2e}", flush=True)
        assert err <= tol


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["fp32", "mixed"])
def test_precond_factor_rows_against_oracle(gpu_lib, name):
    """The Nystrom factor at full size (Algorithm 3 with Algorithm 2 anchors; n = 1e5, k = 1000 and n = 1e6,
    k = 2000) against the oracle on sampled rows: W W^T restricted to the rows I (invariant under the EVD's
    sign and order choices) equals C_I V diag(1/lambda) V^T C_I^T, with C_I = K(X_I, X_S) computed by the
    oracle, K_SS's eigenpairs from numpy.linalg.eigh, the GPU's anchors S and its kept count (the largest
    eigenvalues).  The FP32 copy of W is compared the same way at the FP32 rounding bar."""
    wl = datagen.make_workload(name)
    beta = wl.betas[0]
    idx, sign = datagen.sketch_sparse_draws(wl.n, wl.l, wl.r, datagen.sketch_seed(name))
    P = gpu_lib.Preconditioner(torch.from_numpy(wl.X), wl.eps, [beta], wl.k, wl.l, idx=torch.from_numpy(idx),
                               sign=torch.from_numpy(sign), prec="mixed")
    info = P.info()
    S = np.array(info["S"], dtype=np.int64)
    kept = int(info["kept"])
    rng = np.random.default_rng(17)
    rows = np.sort(rng.choice(wl.n, ROWS, replace=False))
    Kss = ok.kernel_matrix(wl.X[S], wl.X[S], wl.eps)
    lam, V = np.linalg.eigh(Kss)
    lam, V = lam[::-1][:kept], V[:, ::-1][:, :kept]
    C = ok.kernel_matrix(wl.X[rows], wl.X[S], wl.eps)
    B = C @ V / np.sqrt(lam)
    ref = B @ B.T
    ridx = torch.from_numpy(rows).cuda()
    for which, tol in ((P.W64, 1e-9), (P.W32, 1e-6)):
        Wr = P.get(which)[ridx].double().cpu().numpy()
        got = Wr @ Wr.T
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        print(f"{name} workload factor ({'FP64' if which == P.W64 else 'FP32'} copy): kept {kept} of {len(S)}, "
              f"max |W_I W_I^T - oracle| / max|oracle| = {err:.2e}", flush=True)
        assert err <= tol
