"""Pins for the oracle's PCG (Algorithm 5) on the CPU.

Anchors: a dense Cholesky solve (the O(n^3) direct method of Sec. 1), the CG
error bound of Eq. cgrate with the exact condition number, identity
preconditioning reducing to plain CG, finite termination, the Lanczos
estimate against eigvalsh, and the workload `small` (n=2000, d=3) end to end.
"""
import numpy as np
import pytest

import datagen
from oracle import kernel as ok
from oracle import pcg as oc
from oracle import precond as op
from oracle import theory as th


def _problem(n=150, d=2, eps=0.05, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    y = np.sin(3 * X[:, 0]) + 0.1 * rng.standard_normal(n)
    return X, y, eps


def test_pcg_matches_cholesky():
    X, y, eps = _problem()
    beta = 1e-2
    ref = oc.solve_dense(X, y, eps, beta)
    K = ok.kernel_matrix(X, X, eps)
    A = K + beta * np.eye(len(y))
    kappa = np.linalg.cond(A)
    res = oc.solve_krr(X, y, eps, beta, None, tol=1e-12)
    assert res["converged"]
    assert np.linalg.norm(res["x"] - ref) / np.linalg.norm(ref) <= kappa * 1e-12 * 10
    np.testing.assert_allclose(A @ ref, y, rtol=0, atol=1e-10)


def test_cg_error_bound_eq_cgrate():
    X, y, eps = _problem(n=80, eps=0.1)
    beta = 1e-1
    K = ok.kernel_matrix(X, X, eps)
    A = K + beta * np.eye(len(y))
    xs = np.linalg.solve(A, y)
    lam = np.linalg.eigvalsh(A)
    kappa = lam[-1] / lam[0]
    errs = []
    oc.pcg(lambda v: A @ v, y, tol=1e-14, maxit=200, callback=lambda it, x, rel: errs.append(x.copy()))
    e0 = np.sqrt(xs @ A @ xs)
    for i, x in enumerate(errs, start=1):
        e = xs - x
        assert np.sqrt(e @ A @ e) <= th.cg_error_bound(kappa, i) * e0 * (1 + 1e-6) + 1e-12


def test_identity_preconditioner_is_plain_cg():
    X, y, eps = _problem(n=60)
    K = ok.kernel_matrix(X, X, eps)
    A = lambda v: K @ v + 1e-2 * v  # noqa: E731
    a = oc.pcg(A, y, None, tol=1e-9)
    b = oc.pcg(A, y, lambda r: r.copy(), tol=1e-9)
    assert a["iters"] == b["iters"]
    np.testing.assert_array_equal(a["x"], b["x"])


def test_finite_termination_and_replacement():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    A = Q @ np.diag(np.linspace(1, 4, 12)) @ Q.T
    y = rng.standard_normal(12)
    res = oc.pcg(lambda v: A @ v, y, tol=1e-13, maxit=100)
    assert res["converged"] and res["iters"] <= 14
    rep = oc.pcg(lambda v: A @ v, y, tol=1e-13, maxit=100, replace_every=3)
    np.testing.assert_allclose(rep["x"], res["x"], rtol=1e-11)


def test_lanczos_kappa_estimate():
    X, y, eps = _problem(n=120, eps=0.05)
    beta = 1e-2
    K = ok.kernel_matrix(X, X, eps)
    A = K + beta * np.eye(len(y))
    res = oc.pcg(lambda v: A @ v, y, tol=1e-13, maxit=500)
    est = oc.kappa_estimate(res["gammas"], res["deltas"])
    lam = np.linalg.eigvalsh(A)
    assert abs(est / (lam[-1] / lam[0]) - 1) < 0.05


def test_preconditioned_solve_small_workload():
    """Workload `small`: Alg. 1 preconditioner (k=150, l=170), PCG to 1e-10 vs dense Cholesky."""
    wl = datagen.make_workload("small")
    beta = wl.betas[0]
    om = datagen.sketch_dense_omega(wl.n, wl.l, datagen.sketch_seed("small"))
    P = op.build_precond(wl.X, wl.eps, [beta], wl.k, omega=om)
    K = ok.kernel_matrix(wl.X, wl.X, wl.eps)
    A = lambda v: K @ v + beta * v  # noqa: E731
    pre = oc.pcg(A, wl.y, lambda r: op.apply_precond(P, beta, r), tol=wl.tol, maxit=5000)
    plain = oc.pcg(A, wl.y, None, tol=wl.tol, maxit=20000)
    ref = oc.solve_dense(wl.X, wl.y, wl.eps, beta)
    assert pre["converged"] and plain["converged"]
    assert pre["iters"] < plain["iters"] / 3
    kappa_est = oc.kappa_estimate(pre["gammas"], pre["deltas"])
    err = np.linalg.norm(pre["x"] - ref) / np.linalg.norm(ref)
    assert err < 1e-6
    # the preconditioned system's condition number obeys the ID corollary
    lamK = np.linalg.eigvalsh(K)[::-1]
    tight, _ = th.cond_bound_id(lamK[wl.k], wl.k, wl.n, beta)
    assert kappa_est <= tight
