"""Failure reporting through the C ABI: non-finite inputs are rejected with KRR_EINVAL before any GPU work,
a solve that stops before its tolerance is reported (KRR_ENOCONV) by the gradient and its autograd wrapper,
and the library keeps working after each error."""
import math
import warnings

import numpy as np
import pytest
import torch

import datagen
from oracle import kernel as ok


def _pts(n=300, d=3, seed=0):
    return np.random.default_rng(seed).random((n, d))


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("what", ["Xt", "Xs", "V"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_kernel_mv_rejects_non_finite(gpu_lib, prec, what, bad):
    X, Y = _pts(seed=1), _pts(200, seed=2)
    v = np.random.default_rng(3).standard_normal(200)
    args = {"Xt": X.copy(), "Xs": Y.copy(), "V": v.copy()}
    a = args[what]
    a.flat[a.size // 2] = bad
    with pytest.raises(gpu_lib.KRRError, match="NaN or Inf") as e:
        gpu_lib.kernel_mv(torch.from_numpy(args["Xt"]), torch.from_numpy(args["Xs"]), 0.1,
                          torch.from_numpy(args["V"]), prec=prec)
    assert e.value.status == -1
    # the next call is unaffected
    u = gpu_lib.kernel_mv(torch.from_numpy(X), torch.from_numpy(Y), 0.1, torch.from_numpy(v), prec=prec)
    ref = ok.kernel_mv(X, Y, 0.1, v)
    assert np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-5


@pytest.mark.gpu
def test_kernel_mv_rejects_non_finite_shift(gpu_lib):
    X = _pts()
    v = np.ones(len(X))
    with pytest.raises(gpu_lib.KRRError, match="shift"):
        gpu_lib.kernel_mv(torch.from_numpy(X), None, 0.1, torch.from_numpy(v), shift=float("nan"))


@pytest.mark.gpu
@pytest.mark.parametrize("what", ["X", "y", "x0"])
def test_pcg_solve_rejects_non_finite(gpu_lib, what):
    X = _pts(400, 2, seed=5)
    y = np.sin(4 * X[:, 0])
    x0 = np.zeros(400)
    arr = {"X": X.copy(), "y": y.copy(), "x0": x0.copy()}
    arr[what].flat[7] = float("nan") if what != "x0" else float("-inf")
    with pytest.raises(gpu_lib.KRRError, match="NaN or Inf") as e:
        gpu_lib.pcg_solve(torch.from_numpy(arr["X"]), torch.from_numpy(arr["y"]), 0.05, 1e-2, None, tol=1e-8,
                          x0=torch.from_numpy(arr["x0"]))
    assert e.value.status == -1
    _, _, rel, _, status = gpu_lib.pcg_solve(torch.from_numpy(X), torch.from_numpy(y), 0.05, 1e-2, None,
                                             tol=1e-8, maxit=5000)
    assert status == 0 and rel[0] <= 1e-8


@pytest.mark.gpu
@pytest.mark.parametrize("what", ["X", "sign", "omega"])
def test_build_precond_rejects_non_finite(gpu_lib, what):
    n, k, l = 500, 40, 50
    X = _pts(n, 3, seed=6)
    if what == "omega":
        om = datagen.sketch_dense_omega(n, l, 9)
        om[3, 4] = float("inf")
        kw = {"omega": torch.from_numpy(om)}
        Xb = X
    else:
        idx, sign = datagen.sketch_sparse_draws(n, l, 8, 9)
        if what == "sign":
            sign = sign.copy()
            sign[2, 1] = float("nan")
        Xb = X.copy()
        if what == "X":
            Xb[10, 1] = float("nan")
        kw = {"idx": torch.from_numpy(idx), "sign": torch.from_numpy(sign)}
    with pytest.raises(gpu_lib.KRRError, match="NaN or Inf") as e:
        gpu_lib.Preconditioner(torch.from_numpy(Xb), 0.05, [1e-2], k, l, prec="mixed", **kw)
    assert e.value.status == -1


@pytest.mark.gpu
def test_grad_reports_unconverged_solves(gpu_lib):
    """maxit too small for the forward solve: krr_grad returns KRR_ENOCONV, the binding passes it on, and
    KRRValLoss refuses the values unless told to accept them (then it warns)."""
    rng = np.random.default_rng(8)
    Xtr, Xv = rng.random((500, 2)), rng.random((80, 2))
    ytr, yv = np.sin(3 * Xtr[:, 0]), np.sin(3 * Xv[:, 0])
    args = [torch.from_numpy(a).cuda() for a in (Xtr, ytr, Xv, yv)]
    g = gpu_lib.grad(*args, 0.1, 1e-3, None, tol=1e-12, maxit=3, prec="fp64")
    assert g[5] == 1
    g = gpu_lib.grad(*args, 0.1, 1e-3, None, tol=1e-8, maxit=20000, prec="fp64")
    assert g[5] == 0
    le = torch.tensor(math.log(0.1), dtype=torch.float64, device="cuda", requires_grad=True)
    lb = torch.tensor(math.log(1e-3), dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.raises(gpu_lib.KRRError) as e:
        gpu_lib.KRRValLoss.apply(le, lb, *args, None, {"tol": 1e-12, "maxit": 3})
    assert e.value.status == 1
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        loss = gpu_lib.KRRValLoss.apply(le, lb, *args, None, {"tol": 1e-12, "maxit": 3, "allow_noconv": True})
    assert any("KRR_ENOCONV" in str(x.message) for x in w)
    assert math.isfinite(loss.item())
