"""The two PCG drivers (Algorithm 5): host loop and graph-captured cycles with device-side convergence claims.

Both launch the same kernels in the same order, so the iterates must be bit-identical: the returned alpha,
the iteration counts, the true relative residuals, the product counts and the Lanczos estimates are compared
exactly.  Cases cover a cycle that runs to its end, claims that halt a cycle before its end (the solve's
convergence), claims that fail the true-residual check (the stall rule), maxit inside a cycle, several
columns with different betas, and solves without replacement or preconditioner.  The oracle comparison of
the solution itself is in test_gpu_pcg.py; here alpha is also checked against the dense solve once.
"""
import numpy as np
import pytest
import torch

import datagen
from oracle import pcg as oc


@pytest.fixture(scope="module")
def small(gpu_lib):
    wl = datagen.make_workload("small")
    om = datagen.sketch_dense_omega(wl.n, wl.l, datagen.sketch_seed("small"))
    P = gpu_lib.Preconditioner(torch.from_numpy(wl.X), wl.eps, [wl.betas[0], 1e-2], wl.k, wl.l,
                               omega=torch.from_numpy(om), prec="mixed")
    return wl, P


def _both(gpu_lib, *args, **kw):
    out = {}
    try:
        for mode in (0, 1):
            gpu_lib.set_pcg_mode(mode)
            a, its, rel, st, status = gpu_lib.pcg_solve(*args, **kw)
            out[mode] = (a.cpu().numpy().copy(), its, rel, st, status)
    finally:
        gpu_lib.set_pcg_mode(-1)
    return out[0], out[1]


def _same(h, g):
    a0, its0, rel0, st0, s0 = h
    a1, its1, rel1, st1, s1 = g
    assert s0 == s1
    assert its0 == its1
    assert rel0 == rel1
    assert np.array_equal(a0.view(np.uint64), a1.view(np.uint64)), "iterates differ between the drivers"
    for k in ("iters_max", "n_mvm", "n_mvm_fp64", "n_replace", "kappa_est", "lam_min_est", "lam_max_est"):
        assert st0[k] == st1[k], k
    assert st0["n_graph_cycles"] == 0 and st1["n_graph_cycles"] >= 1
    assert 0 < st1["n_graph_iters"] <= st1["iters_max"]


@pytest.mark.gpu
def test_graph_fp64_no_replacement(gpu_lib, small):
    """Workload small (n=2000, d=3, FP64, tol 1e-10): 16-iteration cycles, the last one halted by the claim."""
    wl, P = small
    h, g = _both(gpu_lib, torch.from_numpy(wl.X), torch.from_numpy(wl.y), wl.eps, wl.betas[0], P, tol=wl.tol,
                 maxit=5000, prec="fp64")
    print(f"fp64: {h[1][0]} its; host {h[3]['t_total_ms']:.1f} ms, graph {g[3]['t_total_ms']:.1f} ms "
          f"({g[3]['n_graph_cycles']} cycles, {g[3]['n_graph_iters']} iterations in cycles)")
    _same(h, g)
    assert h[4] == 0 and h[2][0] <= wl.tol
    ref = oc.solve_dense(wl.X, wl.y, wl.eps, wl.betas[0])
    assert np.linalg.norm(g[0] - ref) / np.linalg.norm(ref) <= 1e-6


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_graph_with_replacement(gpu_lib, small, prec):
    """Cycles of 10 iterations ending in the FP64 check of the scheduled replacement."""
    wl, P = small
    h, g = _both(gpu_lib, torch.from_numpy(wl.X), torch.from_numpy(wl.y), wl.eps, wl.betas[0], P, tol=1e-9,
                 maxit=5000, replace_every=10, prec=prec)
    print(f"{prec}: {h[1][0]} its, {h[3]['n_replace']} replacements; host {h[3]['t_total_ms']:.1f} ms, "
          f"graph {g[3]['t_total_ms']:.1f} ms")
    _same(h, g)
    assert h[4] == 0 and h[2][0] <= 1e-9


@pytest.mark.gpu
def test_graph_failed_claims_and_stall(gpu_lib, small):
    """tol below the mixed recurrence's attainable accuracy: claims fail the check, the column waits before
    its next check, and stops after eight failed claims with its best iterate (KRR_ENOCONV)."""
    wl, P = small
    h, g = _both(gpu_lib, torch.from_numpy(wl.X), torch.from_numpy(wl.y), wl.eps, wl.betas[0], P, tol=1e-15,
                 maxit=600, replace_every=10, prec="mixed")
    print(f"stall: status {h[4]}, {h[1][0]} its, relres {h[2][0]:.2e}, FP64 products {h[3]['n_mvm_fp64']}")
    _same(h, g)
    assert h[4] == 1


@pytest.mark.gpu
def test_graph_maxit_inside_cycle(gpu_lib, small):
    wl, P = small
    h, g = _both(gpu_lib, torch.from_numpy(wl.X), torch.from_numpy(wl.y), wl.eps, wl.betas[0], P, tol=1e-12,
                 maxit=37, replace_every=10, prec="mixed")
    _same(h, g)
    assert h[4] == 1 and h[1][0] == 37


@pytest.mark.gpu
def test_graph_block_columns(gpu_lib, small):
    """Three columns with two betas; they converge at different iterations inside cycles."""
    wl, P = small
    rng = np.random.default_rng(3)
    Y = np.stack([wl.y, np.sin(5 * wl.X[:, 1]), rng.standard_normal(wl.n)], axis=1)
    betas = [wl.betas[0], 1e-2, wl.betas[0]]
    for prec, rep in (("fp64", 0), ("mixed", 10)):
        h, g = _both(gpu_lib, torch.from_numpy(wl.X), torch.from_numpy(Y), wl.eps, betas, P, tol=1e-9,
                     maxit=5000, replace_every=rep, prec=prec)
        print(f"block {prec}: its {h[1]}")
        _same(h, g)
        assert h[4] == 0 and len(set(h[1])) > 1


@pytest.mark.gpu
def test_graph_without_preconditioner(gpu_lib, small):
    wl, _ = small
    h, g = _both(gpu_lib, torch.from_numpy(wl.X), torch.from_numpy(wl.y), wl.eps, 1e-1, None, tol=1e-8,
                 maxit=3000, replace_every=5, prec="fp32")
    _same(h, g)
    assert h[4] == 0


@pytest.mark.gpu
def test_graph_automatic_choice(gpu_lib, small):
    """Automatic mode: cycles for this small product, the host loop when phase timing is asked for."""
    wl, P = small
    X, y = torch.from_numpy(wl.X), torch.from_numpy(wl.y)
    _, _, _, st, _ = gpu_lib.pcg_solve(X, y, wl.eps, wl.betas[0], P, tol=wl.tol, maxit=5000, prec="fp64")
    assert st["n_graph_cycles"] >= 1
    _, _, _, st, _ = gpu_lib.pcg_solve(X, y, wl.eps, wl.betas[0], P, tol=wl.tol, maxit=5000, prec="fp64",
                                       timing=True)
    assert st["n_graph_cycles"] == 0


@pytest.mark.gpu
@pytest.mark.parametrize("n,R,prec,rep", [(20000, 1, "mixed", 10), (7000, 3, "fp64", 0), (24000, 1, "fp32", 10)],
                         ids=["n20000_R1_mixed", "n7000_R3_fp64", "n24000_R1_fp32"])
def test_graph_two_stage_reductions(gpu_lib, n, R, prec, rep):
    """Problems above the one-workgroup limit (n R > 16384): the gated two-stage column reductions and the
    separate update kernels inside the captured cycles, against the host loop, bit for bit."""
    rng = np.random.default_rng(n + R)
    X = rng.random((n, 4))
    Y = np.sin(3.0 * X[:, :1] + np.arange(R)[None, :]) + 0.1 * rng.standard_normal((n, R))
    eps = 0.05
    betas = [1e-2, 1e-1, 1e-2][:R]
    k, l = 300, 320
    idx, sign = datagen.sketch_sparse_draws(n, l, 16, n + R)
    P = gpu_lib.Preconditioner(torch.from_numpy(X), eps, sorted(set(betas)), k, l, idx=torch.from_numpy(idx),
                               sign=torch.from_numpy(sign), prec="mixed")
    Yt = torch.from_numpy(Y if R > 1 else Y[:, 0].copy())
    h, g = _both(gpu_lib, torch.from_numpy(X), Yt, eps, betas if R > 1 else betas[0], P, tol=1e-8, maxit=3000,
                 replace_every=rep, prec=prec)
    print(f"n={n} R={R} {prec}: its {h[1]}; host {h[3]['t_total_ms']:.1f} ms, graph {g[3]['t_total_ms']:.1f} ms "
          f"({g[3]['n_graph_cycles']} cycles)")
    _same(h, g)
    assert h[4] == 0


@pytest.mark.gpu
@pytest.mark.parametrize("prec,rep", [("fp64", 0), ("mixed", 10)])
def test_graph_active_set_shrinks(gpu_lib, small, prec, rep):
    """Twenty columns, twelve at the larger beta: once columns converge the cycles' products form the active
    columns only, in narrower staged blocks (20 columns stage as 32 in FP64 and in the mixed block form,
    eight or fewer as 8 or 16).  The staging buffers keep their size, so the cycles captured after a column
    set shrinks allocate nothing; the iterates stay bit-identical to the host loop's."""
    wl, P = small
    R = 20
    rng = np.random.default_rng(17)
    Y = np.sin(np.outer(wl.X[:, 0] + wl.X[:, 2], np.arange(1, R + 1))) + 0.05 * rng.standard_normal((wl.n, R))
    betas = [1e-2] * 12 + [wl.betas[0]] * 8
    h, g = _both(gpu_lib, torch.from_numpy(wl.X), torch.from_numpy(Y), wl.eps, betas, P, tol=1e-9, maxit=5000,
                 replace_every=rep, prec=prec)
    its = np.asarray(h[1])
    print(f"{prec}: its {its.tolist()}; {g[3]['n_graph_cycles']} cycles, {g[3]['n_graph_iters']} iterations in "
          f"cycles")
    _same(h, g)
    assert h[4] == 0
    cycle = rep if rep else 16
    assert its.max() - its.min() > 2 * cycle, "the active set should shrink well before the last column converges"
