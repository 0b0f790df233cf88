"""Pins for the oracle's Gaussian kernel and kernel MVM (CPU only).

Each check ties the oracle to something other than itself: pure-Python brute
force, a two-point closed form, matrix invariants (symmetry, unit diagonal, PSD
— Sec. 1 and Lemma schur), invariances of the kernel, the Kronecker structure
of the kernel on a tensor grid, and a finite difference in eps for K'.
"""
import math

import numpy as np
import pytest

from oracle import kernel as ok


def brute_kernel(Xt, Xs, eps):
    out = []
    for a in Xt:
        row = []
        for b in Xs:
            s = 0.0
            for p, q in zip(a, b):
                s += (p - q) * (p - q)
            row.append(math.exp(-s / eps))
        out.append(row)
    return np.array(out)


def test_brute_force_small():
    rng = np.random.default_rng(0)
    X = rng.random((13, 3))
    Z = rng.random((7, 3))
    np.testing.assert_allclose(ok.kernel_matrix(X, Z, 0.3), brute_kernel(X, Z, 0.3), rtol=1e-14, atol=0)
    v = rng.standard_normal(7)
    np.testing.assert_allclose(ok.kernel_mv(X, Z, 0.3, v), brute_kernel(X, Z, 0.3) @ v, rtol=1e-13, atol=1e-15)


def test_two_point_closed_form():
    # distance^2 = eps ln 2  =>  k = exp(-ln 2) = 1/2 ; eigenvalues of [[1, e], [e, 1]] are 1 +- e
    eps = 0.37
    delta = math.sqrt(eps * math.log(2.0))
    X = np.array([[0.1, 0.2], [0.1 + delta, 0.2]])
    K = ok.kernel_matrix(X, X, eps)
    assert abs(K[0, 1] - 0.5) < 1e-15 and abs(K[1, 0] - 0.5) < 1e-15
    np.testing.assert_allclose(np.linalg.eigvalsh(K), [0.5, 1.5], rtol=1e-14)


def test_matrix_invariants():
    rng = np.random.default_rng(1)
    X = rng.random((300, 4))
    K = ok.kernel_matrix(X, X, 0.05)
    assert np.array_equal(K, K.T)
    assert np.all(np.diag(K) == 1.0)
    assert np.all(K > 0) and np.all(K <= 1.0)
    lam = np.linalg.eigvalsh(K)
    assert lam.min() >= -K.shape[0] * np.finfo(float).eps * lam.max()


def test_special_cases():
    X = np.tile(np.array([[0.3, -1.2, 4.0]]), (5, 1))
    assert np.all(ok.kernel_matrix(X, X, 0.01) == 1.0)                   # coincident points: K = 1 1^T
    rng = np.random.default_rng(2)
    Y = rng.random((20, 3))
    np.testing.assert_allclose(ok.kernel_matrix(Y, Y, 1e12), 1.0, atol=1e-11)   # eps -> infinity
    G = np.arange(10.0)[:, None] * np.ones((1, 2))                      # points 1.41 apart, tiny eps
    np.testing.assert_array_equal(ok.kernel_matrix(G, G, 1e-3), np.eye(10))


def test_invariances():
    rng = np.random.default_rng(3)
    X = rng.random((60, 3))
    K = ok.kernel_matrix(X, X, 0.1)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Xm = X @ Q.T + np.array([5.0, -2.0, 0.25])
    np.testing.assert_allclose(ok.kernel_matrix(Xm, Xm, 0.1), K, atol=1e-13)
    perm = rng.permutation(60)
    np.testing.assert_allclose(ok.kernel_matrix(X[perm], X[perm], 0.1), K[np.ix_(perm, perm)], atol=0)


def test_separable_and_kronecker():
    # exp(-||x-x'||^2/eps) = prod_m exp(-(x_m-x'_m)^2/eps): on a tensor grid K = K1 (x) K2
    g1 = np.linspace(0, 1, 7)
    g2 = np.linspace(0, 2, 5)
    X = np.array([[a, b] for a in g1 for b in g2])
    eps = 0.2
    K1 = ok.kernel_matrix(g1[:, None], g1[:, None], eps)
    K2 = ok.kernel_matrix(g2[:, None], g2[:, None], eps)
    np.testing.assert_allclose(ok.kernel_matrix(X, X, eps), np.kron(K1, K2), rtol=1e-14)
    lam = np.sort(np.outer(np.linalg.eigvalsh(K1), np.linalg.eigvalsh(K2)).ravel())
    np.testing.assert_allclose(np.linalg.eigvalsh(ok.kernel_matrix(X, X, eps)), lam, atol=1e-12)
    # and a 1-D closed form: adjacent grid points at spacing s give exp(-s^2/eps)
    np.testing.assert_allclose(K1[0, 1], math.exp(-(1 / 6) ** 2 / eps), rtol=1e-15)


@pytest.mark.parametrize("R", [1, 3])
def test_tiled_mv_matches_dense(R):
    rng = np.random.default_rng(4)
    X = rng.random((1000, 3))
    Xs = rng.random((333, 3))
    V = rng.standard_normal((333, R)) if R > 1 else rng.standard_normal(333)
    dense = ok.kernel_matrix(X, Xs, 0.07) @ V
    np.testing.assert_allclose(ok.kernel_mv(X, Xs, 0.07, V, block=97), dense, rtol=1e-12, atol=1e-12)
    # rows of the square operator with the ridge shift
    v = rng.standard_normal(1000)
    full = ok.kernel_mv(X, X, 0.07, v, shift=0.01)
    rows = np.array([0, 17, 999])
    np.testing.assert_allclose(ok.kernel_mv_rows(X, 0.07, v, rows, shift=0.01), full[rows], rtol=1e-12)


def test_deriv_kernel_is_eps_dk_deps():
    rng = np.random.default_rng(5)
    X = rng.random((40, 2))
    eps, h = 0.3, 1e-5
    Kp = ok.kernel_deriv_matrix(X, X, eps)
    fd = (ok.kernel_matrix(X, X, eps * math.exp(h)) - ok.kernel_matrix(X, X, eps * math.exp(-h))) / (2 * h)
    np.testing.assert_allclose(Kp, fd, atol=1e-9)
    assert np.all(np.diag(Kp) == 0.0)
    v = rng.standard_normal(40)
    U, Ud = ok.kernel_mv(X, X, eps, v, deriv=2, block=9)
    np.testing.assert_allclose(U, ok.kernel_matrix(X, X, eps) @ v, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(Ud, Kp @ v, rtol=1e-12, atol=1e-13)
