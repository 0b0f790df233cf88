"""GPU parity of the other anchor choices (remark in Sec. 3) and of the data-driven rank (Corollary tradeoff).

* Farthest point sampling: the picks are argmax decisions taken in FP64 on both sides with the same
  unfused arithmetic, so indices and pick distances must be identical bit for bit, ties included
  (integer grids with many equal distances, repeated points, one block, many blocks, rows beyond
  one pass of the grid).
* Algorithm 3 on given anchors (random sampling) and on FPS anchors: anchors identical to the
  oracle's, W W^T = C K_SS^+ C^T, the Woodbury apply against the oracle's apply, and PCG converging
  with either preconditioner.
* Eq. condbound on the data: bounding box, gamma and the rank bound equal to the oracle's.
"""
import math

import numpy as np
import pytest
import torch

import datagen
from oracle import kernel as ok
from oracle import precond as op
from oracle import theory as th


def _pts(n, d, seed):
    return np.random.default_rng(seed).random((n, d))


def _grid(n, d, levels, seed):
    return np.random.default_rng(seed).integers(0, levels, size=(n, d)).astype(np.float64)


FPS_CASES = [
    # (name, X builder, k, start)
    ("single", lambda: _pts(1, 3, 1), 1, 0),
    ("k_eq_n_two_blocks", lambda: _pts(257, 3, 2), 257, 5),
    ("ragged", lambda: _pts(5000, 2, 3), 300, 17),
    ("many_blocks_d8", lambda: _pts(70001, 8, 4), 150, 70000),
    ("grid_stride_rows", lambda: _pts(600_000, 4, 5), 40, 123),
    ("integer_grid_ties", lambda: _grid(3000, 3, 5, 6), 200, 0),       # 125 positions: later picks at 0
    ("repeated_points", lambda: np.repeat(_pts(10, 2, 7), 100, axis=0), 60, 999),
    ("d_max", lambda: _pts(2000, 128, 8), 30, 1),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,k,start", FPS_CASES, ids=[c[0] for c in FPS_CASES])
def test_fps_bit_exact(gpu_lib, name, make, k, start):
    X = make()
    print(f"fps case {name}: n={X.shape[0]} d={X.shape[1]} k={k} start={start}", flush=True)
    S, dsel = gpu_lib.fps(torch.from_numpy(X), k, start)
    S_ref, dsel_ref = op.fps(X, k, start)
    np.testing.assert_array_equal(S.cpu().numpy(), S_ref)
    got = dsel.cpu().numpy()
    assert np.isinf(got[0])
    bad = np.nonzero(got[1:].view(np.uint64) != dsel_ref[1:].view(np.uint64))[0] + 1
    for j in bad[:5]:
        print(f"  dsel[{j}] gpu {got[j]!r} ({got[j].hex()}) oracle {dsel_ref[j]!r} ({dsel_ref[j].hex()})")
    assert bad.size == 0


@pytest.mark.gpu
def test_fps_rejects_bad_arguments(gpu_lib):
    X = torch.from_numpy(_pts(50, 2, 9))
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.fps(X, 51, 0)            # k > n
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.fps(X, 5, 50)            # start out of range
    bad = X.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.fps(bad, 5, 0)


@pytest.mark.gpu
@pytest.mark.parametrize("how", ["random", "fps"])
def test_build_on_given_anchors(gpu_lib, how):
    n, d, k, eps, beta = 3000, 3, 120, 0.01, 1e-3
    X = _pts(n, d, 20)
    S_in = datagen.random_anchors(n, k, seed=21) if how == "random" else None
    anchors = torch.from_numpy(S_in) if how == "random" else "fps"
    P = gpu_lib.Preconditioner(torch.from_numpy(X), eps, [beta, 1e-2], k, anchors=anchors, fps_start=7,
                               prec="mixed")
    info = P.info()
    S = np.array(info["S"])
    S_ref = S_in if how == "random" else op.fps(X, k, 7)[0]
    np.testing.assert_array_equal(S, S_ref)
    assert info["rdiag"] == [0.0] * k
    ref = op.build_precond_from_anchors(X, eps, [beta], S_ref)
    W = P.get(P.W64).cpu().numpy()
    assert info["kept"] == ref["kept"]
    np.testing.assert_allclose(W @ W.T, ref["W"] @ ref["W"].T, rtol=0, atol=1e-9)
    x = np.random.default_rng(22).standard_normal(n)
    got = P.apply(torch.from_numpy(x), betas=[beta], prec="fp64").cpu().numpy()
    want = op.apply_precond(ref, beta, x)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"{how} anchors: kept {info['kept']}, apply rel err {err:.2e}, timings {P.timings()}")
    assert err <= 1e-9
    t = P.timings()
    assert t["sketch"] == 0.0 and t["total"] >= t["qr"]


@pytest.mark.gpu
def test_pcg_with_fps_and_random_anchors(gpu_lib):
    wl = datagen.make_workload("fp32", n=12_000)
    X = torch.from_numpy(wl.X)
    y = torch.from_numpy(wl.y)
    k, beta = 400, wl.betas[0]
    its = {}
    for how in ("fps", "random", "none"):
        if how == "none":
            P = None
        else:
            anchors = "fps" if how == "fps" else torch.from_numpy(datagen.random_anchors(wl.n, k, seed=23))
            P = gpu_lib.Preconditioner(X, wl.eps, [beta], k, anchors=anchors, prec="mixed")
        alpha, it, rel, st, status = gpu_lib.pcg_solve(X, y, wl.eps, [beta], P, tol=1e-8, maxit=5000,
                                                        replace_every=10, prec="mixed")
        r = y.numpy() - (ok.kernel_mv(wl.X, wl.X, wl.eps, alpha.cpu().numpy()) + beta * alpha.cpu().numpy())
        true_rel = np.linalg.norm(r) / np.linalg.norm(wl.y)
        its[how] = int(np.atleast_1d(it)[0])
        print(f"anchors {how}: {its[how]} iterations, true relres {true_rel:.2e}", flush=True)
        assert status == 0 and true_rel <= 1e-8 * 1.5
    assert its["fps"] < its["none"] and its["random"] < its["none"]


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["uniform", "box", "clusters"])
def test_rank_for_cond_parity(gpu_lib, case):
    if case == "uniform":
        X, eps, beta, xi, Mbar = _pts(200_001, 3, 30), 0.5, 1e-2, 10.0, None
    elif case == "box":
        corners = np.array([[a, b, c] for a in (0.0, 2.0) for b in (-1.0, 0.0) for c in (3.0, 3.5)])
        X = np.vstack([corners, [[1.0, -0.5, 3.2], [0.3, -0.1, 3.4]]])
        eps, beta, Mbar = 1.0, 0.5, None
        xi = 1.0 + 100.0 * math.exp(-(1.05 * math.pi) ** 2) / beta
    else:
        wl = datagen.make_workload("fp32", n=30_000)
        X, eps, beta, xi, Mbar = wl.X, wl.eps, wl.betas[0], 4.0, 1e3
    g, kb, q = gpu_lib.rank_for_cond(torch.from_numpy(X), eps, beta, xi, Mbar)
    g_ref, k_ref = th.rank_for_cond(X, eps, beta, xi, Mbar)
    np.testing.assert_array_equal(q, X.max(axis=0) - X.min(axis=0))
    assert g == g_ref
    assert kb == float(k_ref)
    print(f"rank_for_cond {case}: gamma {g:.4f}, k >= {kb:.6g}")
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.rank_for_cond(torch.from_numpy(X), eps, beta, 1.0)       # xi must exceed 1


@pytest.mark.gpu
def test_given_anchors_rejected(gpu_lib):
    X = torch.from_numpy(_pts(100, 2, 31))
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.Preconditioner(X, 0.1, [1e-3], 3, anchors=torch.tensor([1, 5, 1]))       # repeated
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.Preconditioner(X, 0.1, [1e-3], 3, anchors=torch.tensor([1, 5, 100]))     # out of range
    with pytest.raises(gpu_lib.KRRError):
        gpu_lib.Preconditioner(X, 0.1, [1e-3], 3, anchors="fps", fps_start=100)
    with pytest.raises(ValueError):
        gpu_lib.Preconditioner(X, 0.1, [1e-3], 3, anchors=torch.tensor([1, 5]))
