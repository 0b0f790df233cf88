"""Exact far-tile culling of the symmetric mixed product (the paper's replaceable MVM, Sec. 2.4, made faster
without an approximation): on spread-out points most 16-source steps are skipped, and the product equals the
unculled one bit for bit and the oracle within the mixed-precision bar; a PCG solve gives identical iterates
with and without it."""
import numpy as np
import pytest
import torch

from oracle import kernel as ok


def _spread(n, d, side, seed):
    return side * np.random.default_rng(seed).random((n, d))


@pytest.mark.gpu
# (the last value: the least fraction of pairs the case must skip; Morton boxes in 8 dimensions are loose)
@pytest.mark.parametrize("n,d,side,eps,min_frac", [(40000, 3, 4.0, 0.01, 0.5), (30000, 4, 1.0, 0.01, 0.01),
                                                   (20000, 8, 3.0, 0.05, 0.01), (5000, 2, 10.0, 0.02, 0.5)])
def test_culled_product_is_exact(gpu_lib, n, d, side, eps, min_frac):
    X = _spread(n, d, side, 70 + d)
    v = np.random.default_rng(71).standard_normal(n)
    Xg, vg = torch.from_numpy(X), torch.from_numpy(v)
    try:
        gpu_lib.set_cull(2)   # the same spatial order, nothing skipped
        u0 = gpu_lib.kernel_mv(Xg, None, eps, vg, shift=0.5, prec="mixed").cpu().numpy()
        tot0, sk0 = gpu_lib.cull_stats()
        gpu_lib.set_cull(0)   # the caller's order
        uc = gpu_lib.kernel_mv(Xg, None, eps, vg, shift=0.5, prec="mixed").cpu().numpy()
        gpu_lib.set_cull(1)
        u1 = gpu_lib.kernel_mv(Xg, None, eps, vg, shift=0.5, prec="mixed").cpu().numpy()
        tot1, sk1 = gpu_lib.cull_stats()
        _, _, sym = gpu_lib.kmv_last_launch()
    finally:
        gpu_lib.set_cull(-1)
    assert sym and sk0 == 0 and tot1 == tot0
    frac = sk1 / tot1
    print(f"n={n} d={d} side={side}: {frac:.3f} of the pairs skipped")
    # bit for bit: every skipped kernel value is exactly zero in FP32
    assert np.array_equal(u0, u1)
    rows = np.random.default_rng(72).choice(n, 200, replace=False)
    ref = ok.kernel_mv(X[rows], X, eps, v) + 0.5 * v[rows]
    scale = ok.kernel_mv(X[rows], X, eps, np.abs(v)) + 0.5 * np.abs(v[rows])
    # the split cross term accumulates terms up to c |z|^2 (c = log2(e)/eps, z = x - mean) in FP32, so the
    # exp2 argument carries an absolute error of a few 2^-24 c max|z|^2: the bar follows the data's extent
    c = np.log2(np.e) / eps
    r2 = ((X - X.mean(0)) ** 2).sum(1).max()
    bar = max(1e-6, 2.0 ** -23 * c * r2)
    e1 = np.abs((u1[rows] - ref) / scale).max()
    ec = np.abs((uc[rows] - ref) / scale).max()
    print(f"  error vs oracle {e1:.2e} (caller's order {ec:.2e}), bar {bar:.2e}")
    assert e1 <= bar and ec <= bar
    assert frac >= min_frac


@pytest.mark.gpu
def test_culled_solve_identical_iterates(gpu_lib):
    n, d, eps, beta = 30000, 3, 0.005, 1e-2
    X = _spread(n, d, 2.5, 73)
    y = np.sin(2 * X[:, 0]) + np.cos(3 * X[:, 1])
    Xg, yg = torch.from_numpy(X), torch.from_numpy(y)
    out = {}
    try:
        for mode in (2, 1):
            gpu_lib.set_cull(mode)
            a, its, rel, st, status = gpu_lib.pcg_solve(Xg, yg, eps, beta, None, tol=1e-6, maxit=3000,
                                                        replace_every=10, prec="mixed")
            out[mode] = (a.cpu().numpy(), its[0], rel[0], status)
    finally:
        gpu_lib.set_cull(-1)
    assert out[2][3] == 0 and out[1][3] == 0
    assert out[2][1] == out[1][1]
    assert np.array_equal(out[2][0], out[1][0])
