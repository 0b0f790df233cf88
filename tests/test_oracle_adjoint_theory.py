"""Pins for the oracle's adjoint gradient and the Section 4 formulas (CPU).

Gradient anchors: central finite differences (h=1e-4 in log space), a closed
form with a single training point, and torch float64 autograd through a dense
Cholesky solve on the CPU.  Theory anchors: the worked values printed after
Corollary tradeoff (tests/golden/rank_bound_examples.json) and the algebra
linking Eq. cgrate to Eq. precond_rate2.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import kernel as ok
from oracle import theory as th

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rank_bound_examples.json")


def _data(n=150, m=40, d=3, seed=0):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(d) / 2
    Xtr = 0.5 * rng.standard_normal((n, d))
    Xv = 0.5 * rng.standard_normal((m, d))
    return Xtr, np.tanh(Xtr @ w) + 0.1 * rng.standard_normal(n), Xv, np.tanh(Xv @ w)


def test_adjoint_vs_finite_differences():
    Xtr, ytr, Xv, yv = _data()
    eps, beta = 2.0, 1e-2
    L, ge, gb, _, _ = oa.val_loss_grad(Xtr, ytr, Xv, yv, eps, beta)
    fe, fb = oa.fd_grad(Xtr, ytr, Xv, yv, eps, beta, h=1e-4)
    assert abs(ge - fe) <= 1e-6 * max(abs(ge), 1e-12) + 1e-10
    assert abs(gb - fb) <= 1e-6 * max(abs(gb), 1e-12) + 1e-10
    assert L == pytest.approx(oa.val_loss(Xtr, ytr, Xv, yv, eps, beta), rel=1e-13)


def test_adjoint_single_training_point_closed_form():
    rng = np.random.default_rng(1)
    x0 = rng.random((1, 2))
    Xv = rng.random((5, 2))
    y0, yv = np.array([0.7]), rng.standard_normal(5)
    eps, beta = 0.3, 0.2
    D2 = ((Xv - x0) ** 2).sum(1)
    kv = np.exp(-D2 / eps)
    a = y0[0] / (1 + beta)                           # K = [1]
    rv = kv * a - yv
    want_L = 0.5 * rv @ rv
    want_e = rv @ ((D2 / eps) * kv * a)              # K' = 0 on the single training pair
    want_b = rv @ (kv * (-beta * y0[0] / (1 + beta) ** 2))
    L, ge, gb, _, _ = oa.val_loss_grad(x0, y0, Xv, yv, eps, beta)
    assert L == pytest.approx(want_L, rel=1e-14)
    assert ge == pytest.approx(want_e, rel=1e-12)
    assert gb == pytest.approx(want_b, rel=1e-12)


def test_adjoint_vs_torch_autograd():
    torch = pytest.importorskip("torch")
    Xtr, ytr, Xv, yv = _data(n=90, m=30, seed=2)
    eps, beta = 1.5, 3e-2
    le = torch.tensor(math.log(eps), dtype=torch.float64, requires_grad=True)
    lb = torch.tensor(math.log(beta), dtype=torch.float64, requires_grad=True)
    Xt, Xvt = torch.from_numpy(Xtr), torch.from_numpy(Xv)
    D2 = ((Xt[:, None, :] - Xt[None, :, :]) ** 2).sum(-1)
    D2v = ((Xvt[:, None, :] - Xt[None, :, :]) ** 2).sum(-1)
    K = torch.exp(-D2 / torch.exp(le))
    Kv = torch.exp(-D2v / torch.exp(le))
    A = K + torch.exp(lb) * torch.eye(len(ytr), dtype=torch.float64)
    Lc = torch.linalg.cholesky(A)
    alpha = torch.cholesky_solve(torch.from_numpy(ytr)[:, None], Lc)[:, 0]
    loss = 0.5 * ((Kv @ alpha - torch.from_numpy(yv)) ** 2).sum()
    loss.backward()
    _, ge, gb, _, _ = oa.val_loss_grad(Xtr, ytr, Xv, yv, eps, beta)
    assert ge == pytest.approx(le.grad.item(), rel=1e-9)
    assert gb == pytest.approx(lb.grad.item(), rel=1e-9)


def test_rank_bound_worked_examples():
    g = json.load(open(GOLDEN))
    for c in g["cases"]:
        if c["what"] == "gamma":
            got = th.rank_gamma(c["h"], c["n"], c["beta"], c["xi"])
            assert 0 <= got - c["expected"] < 0.01       # printed to two decimals (3.3464 appears as 3.34)
        else:
            k = th.rank_bound([c["q"]] * c["d"], c["h"], c["n"], c["beta"], c["xi"])
            assert k == c["expected_base"] ** c["expected_exponent"]
            assert 1e46 < k < 1e47


def test_rank_for_cond_on_a_box():
    # 8 corners of a 2 x 1 x 0.5 box plus two interior points (n = 10), h = 1, Mbar = n, and
    # beta (xi - 1) = n^2 exp(-(1.05 pi)^2): then gamma = 2.1 exactly in real arithmetic, so the
    # factors of Eq. condbound are floor(4.2)+1, floor(2.1)+1, floor(1.05)+1 = 5, 3, 2
    corners = np.array([[a, b, c] for a in (0.0, 2.0) for b in (-1.0, 0.0) for c in (3.0, 3.5)])
    X = np.vstack([corners, [[1.0, -0.5, 3.2], [0.3, -0.1, 3.4]]])
    beta = 0.5
    xi = 1.0 + 100.0 * math.exp(-(1.05 * math.pi) ** 2) / beta
    g, k = th.rank_for_cond(X, 1.0, beta, xi)
    assert abs(g - 2.1) < 1e-12
    assert k == 5 * 3 * 2
    # eps = h^2: halving h doubles gamma
    g2, _ = th.rank_for_cond(X, 0.25, beta, xi)
    assert abs(g2 - 4.2) < 1e-12


def test_cg_rate_formulas():
    assert th.cg_error_bound(1.0, 3) == 0.0
    # Eq. precond_rate2 equals Eq. cgrate solved for i with kappa = 1 + M lam/beta (without the factor 2)
    lam, beta, M, delta = 5.0, 1e-2, 3.0, 1e-6
    kappa = th.cond_bound(lam, beta, M)
    i = th.iters_precond(lam, beta, M, delta)
    s = math.sqrt(kappa)
    assert ((s - 1) / (s + 1)) ** i == pytest.approx(delta, rel=1e-9)


def test_cond_bound_id_hand_values():
    # ID corollary with lam_{k+1} = 0.5, k = 3, n = 10, beta = 0.25:
    #   tight = 1 + 2 (0.5) sqrt(4 * 3 * 7 + 1) / 0.25 = 1 + 4 sqrt(85);  loose = 1 + 2 (0.5) 11 / 0.25 = 45
    tight, loose = th.cond_bound_id(0.5, 3, 10, 0.25)
    assert tight == pytest.approx(1.0 + 4.0 * 85 ** 0.5, rel=1e-15)
    assert loose == 45.0
    # k = n / 2 makes 4k(n - k) + 1 = n^2 + 1, just below (n + 1)^2
    tight, loose = th.cond_bound_id(1.0, 50, 100, 1.0)
    assert tight == pytest.approx(1.0 + 2.0 * math.sqrt(100 ** 2 + 1), rel=1e-15)
    assert loose == 1.0 + 2.0 * 101
    # k = n: the ID reproduces K exactly, the square root is 1
    tight, _ = th.cond_bound_id(2.0, 7, 7, 4.0)
    assert tight == 2.0


def test_iters_noprecond_closed_form_and_cgrate():
    # lam1 = 100, beta = 1, delta = e^-2: -sqrt(100) (-2) / (2 sqrt(1)) = 10 iterations
    assert th.iters_noprecond(100.0, 1.0, math.exp(-2.0)) == pytest.approx(10.0, rel=1e-15)
    # it is Eq. cgrate solved for i with kappa = lam1 / beta, in the large-kappa limit: the exact count
    # ln(delta) / ln((sqrt k - 1)/(sqrt k + 1)) differs from it by a relative O(1/kappa)
    for lam1, beta, delta in ((1e4, 1e-2, 1e-6), (3e3, 0.5, 1e-3), (1e5, 1e-3, 1e-8)):
        kappa = lam1 / beta
        s = math.sqrt(kappa)
        exact = math.log(delta) / math.log((s - 1.0) / (s + 1.0))
        got = th.iters_noprecond(lam1, beta, delta)
        assert abs(got - exact) / exact < 2.0 / kappa
    # doubling lam1 multiplies the count by sqrt 2; squaring delta doubles it
    a = th.iters_noprecond(50.0, 0.1, 1e-4)
    assert th.iters_noprecond(100.0, 0.1, 1e-4) == pytest.approx(a * math.sqrt(2.0), rel=1e-14)
    assert th.iters_noprecond(50.0, 0.1, 1e-8) == pytest.approx(2.0 * a, rel=1e-14)


def test_numerical_rank_on_known_spectra():
    # identity: every singular value equals sigma_1
    assert th.numerical_rank(np.eye(9), 1.0) == 9
    # two points: K = [[1, e], [e, 1]] has eigenvalues 1 + e and 1 - e, ratio (1 - e)/(1 + e)
    e = 0.5
    K2 = np.array([[1.0, e], [e, 1.0]])
    ratio = (1 - e) / (1 + e)
    assert th.numerical_rank(K2, ratio * 0.999) == 2
    assert th.numerical_rank(K2, ratio * 1.001) == 1
    # rank one: all points equal
    assert th.numerical_rank(np.ones((6, 6)), 1e-12) == 1
    # Kronecker structure: the Gaussian kernel on a tensor grid is K1 (x) K2 (separable), so its singular
    # values are the products of the 1-D ones, counted independently here
    g1 = np.linspace(0.0, 1.0, 7)[:, None]
    g2 = np.linspace(0.0, 0.6, 5)[:, None]
    eps = 0.08
    X = np.array([[a, b] for a in g1[:, 0] for b in g2[:, 0]])
    K = ok.kernel_matrix(X, X, eps)
    l1 = np.linalg.eigvalsh(ok.kernel_matrix(g1, g1, eps))
    l2 = np.linalg.eigvalsh(ok.kernel_matrix(g2, g2, eps))
    prod = np.sort(np.abs(np.outer(l1, l2).ravel()))[::-1]
    for delta in (0.5, 1e-2, 1e-4, 1e-7):
        want = int((prod / prod[0] >= delta).sum())
        # keep clear of values that sit on the threshold to rounding
        if np.min(np.abs(prod / prod[0] - delta)) > 1e-9:
            assert th.numerical_rank(K, delta) == want


def test_predict_interpolates_the_solve():
    # at the training points f(X) = K alpha = y - beta alpha for alpha = (K + beta I)^{-1} y (Eq. 1 and
    # Eq. ridge_regression)
    rng = np.random.default_rng(11)
    X = rng.random((60, 3))
    y = rng.standard_normal(60)
    eps, beta = 0.3, 0.05
    K = np.exp(-np.array([[np.sum((a - b) ** 2) for b in X] for a in X]) / eps)   # brute force
    alpha = np.linalg.solve(K + beta * np.eye(60), y)
    f = ok.predict(X, X, eps, alpha)
    np.testing.assert_allclose(f, y - beta * alpha, rtol=0, atol=1e-12)
    # a single training point: f(x) = alpha_1 exp(-||x - x_1||^2 / eps) at new points
    Xq = rng.random((4, 3))
    f1 = ok.predict(Xq, X[:1], eps, np.array([2.5]))
    np.testing.assert_allclose(f1, 2.5 * np.exp(-((Xq - X[0]) ** 2).sum(1) / eps), rtol=1e-15)
    # queries are rows of the output: m query points give m values
    assert ok.predict(Xq, X, eps, alpha).shape == (4,)
