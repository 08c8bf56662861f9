"""Pins of the oracle's dense model and likelihood definitions (CPU only).

What fixes them independently of their own code:
  * the DST-I closed form (eigenvalues of the Dirichlet stencils), a separate
    derivation that never forms K;
  * dense eigenvalues (numpy.linalg.eigvalsh) of the assembled K;
  * finite differences of the log-likelihood for the gradient;
  * symmetric positive semi-definiteness of the Fisher matrix;
  * brute-force double sums for the trace of a product;
  * a hand-derived 2x2 case (N = 2, 1D) written out in closed form;
  * the tree-ordering rule checked on a small rectangle by hand.
"""
import math

import numpy as np
import pytest

from oracle.exact import likelihood_gradient_fisher, loglik_terms, trace_of_product_bruteforce
from oracle.model import Tree, apply_covariance, dense_covariance, neg_laplacian, to_tree_order
from oracle.spectral import mode_eigenvalues, spectral_quantities

ALL = ("kappa", "alpha", "tau2", "sigma2")


def _y(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


@pytest.mark.parametrize("dim,N,theta", [
    (1, 64, (10.0, 0.01, 1e-4, 1.0)),
    (1, 97, (3.0, 0.05, 1e-2, 2.5)),
    (2, 8, (20.0, 2e-4, 1e-3, 1e3)),
    (2, 13, (5.0, 1e-3, 1e-2, 50.0)),
])
def test_dense_matches_spectral(dim, N, theta):
    K, dKs = dense_covariance(dim, N, theta, ALL)
    y = _y(K.shape[0], 5)
    d = likelihood_gradient_fisher(K, dKs, y)
    s = spectral_quantities(dim, N, theta, y, ALL)
    assert abs(d["loglik"] - s["loglik"]) <= 1e-11 * abs(s["loglik"])
    assert abs(d["logdet"] - s["logdet"]) <= 1e-11 * abs(s["logdet"])
    for j in range(4):
        assert abs(d["grad_nll"][j] - s["grad_nll"][j]) <= 1e-9 * max(abs(s["grad_nll"][j]), 1e-30)
    for i in range(4):
        for j in range(4):
            ref = s["fim"][i, j]
            scale = math.sqrt(abs(s["fim"][i, i] * s["fim"][j, j]))
            assert abs(d["fim"][i, j] - ref) <= 1e-9 * scale


def test_dense_eigenvalues_are_the_mode_eigenvalues():
    dim, N, theta = 2, 10, (7.0, 3e-3, 1e-3, 40.0)
    K, _ = dense_covariance(dim, N, theta, ())
    ev = np.sort(np.linalg.eigvalsh(K))
    kappa, alpha, tau2, sigma2 = theta
    mu = mode_eigenvalues(dim, N)
    e = np.sort(sigma2 / ((1 + alpha * mu) ** 2 * (kappa ** 2 + mu) ** 2) + tau2)
    assert np.max(np.abs(ev - e)) <= 1e-12 * np.max(e)


def test_two_point_closed_form():
    # 1D, N = 2, h = 1/3: T = 9 [[2,-1],[-1,2]], eigenpairs (9, [1,1]/sqrt2), (27, [1,-1]/sqrt2).
    kappa, alpha, tau2, sigma2 = 2.0, 0.1, 0.3, 1.7
    K, _ = dense_covariance(1, 2, (kappa, alpha, tau2, sigma2), ())
    lam = [sigma2 / ((1 + alpha * m) ** 2 * (kappa ** 2 + m) ** 2) for m in (9.0, 27.0)]
    u = np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0)
    ref = u @ np.diag(lam) @ u.T + tau2 * np.eye(2)
    assert np.max(np.abs(K - ref)) <= 1e-15 * np.max(np.abs(ref))


def test_laplacian_stencil():
    T = neg_laplacian(2, 3).toarray()
    h2 = (1.0 / 4) ** 2
    # centre point (1,1) -> index 4: 4/h^2 on the diagonal, -1/h^2 to its 4 neighbours
    assert T[4, 4] == pytest.approx(4 / h2)
    for j in (1, 3, 5, 7):
        assert T[4, j] == pytest.approx(-1 / h2)
    assert T[0, 4] == 0.0 and T[0, 8] == 0.0


@pytest.mark.parametrize("dim,N", [(1, 40), (2, 9)])
def test_gradient_matches_finite_differences(dim, N):
    theta = np.array([6.0, 4e-3, 2e-2, 30.0]) if dim == 2 else np.array([6.0, 4e-3, 2e-2, 3.0])
    K, dKs = dense_covariance(dim, N, theta, ALL)
    y = _y(K.shape[0], 9)
    g = likelihood_gradient_fisher(K, dKs, y)["grad_nll"]
    for j in range(4):
        h = 1e-6 * theta[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        lp = loglik_terms(dense_covariance(dim, N, tp, ())[0], y)[0]
        lm = loglik_terms(dense_covariance(dim, N, tm, ())[0], y)[0]
        fd = -(lp - lm) / (2 * h)
        assert abs(fd - g[j]) <= 1e-5 * max(abs(g[j]), 1e-8) + 1e-9


def test_dK_matches_finite_differences():
    dim, N = 2, 7
    theta = np.array([6.0, 4e-3, 2e-2, 30.0])
    _, dKs = dense_covariance(dim, N, theta, ALL)
    for j in range(4):
        h = 1e-6 * theta[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (dense_covariance(dim, N, tp, ())[0] - dense_covariance(dim, N, tm, ())[0]) / (2 * h)
        assert np.max(np.abs(fd - dKs[j])) <= 1e-6 * np.max(np.abs(dKs[j]))


def test_fisher_symmetric_psd():
    K, dKs = dense_covariance(2, 9, (15.0, 1e-3, 1e-3, 200.0), ALL)
    f = likelihood_gradient_fisher(K, dKs, _y(81, 3))["fim"]
    assert np.max(np.abs(f - f.T)) <= 1e-12 * np.max(np.abs(f))
    ev = np.linalg.eigvalsh(0.5 * (f + f.T))
    assert ev.min() >= -1e-12 * ev.max()


def test_trace_of_product_vectorised_vs_bruteforce():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((17, 17))
    B = rng.standard_normal((17, 17))
    assert abs(float(np.sum(A * B.T)) - trace_of_product_bruteforce(A, B)) <= 1e-12 * 17 * 17
    assert abs(np.trace(A @ B) - trace_of_product_bruteforce(A, B)) <= 1e-11


@pytest.mark.parametrize("which,j", [("K", None), ("kappa", 0), ("alpha", 1), ("sigma2", 3), ("tau2", 2)])
def test_apply_covariance_matches_dense(which, j):
    dim, N, theta = 2, 9, (8.0, 2e-3, 1e-3, 60.0)
    K, dKs = dense_covariance(dim, N, theta, ALL)
    X = np.random.default_rng(2).standard_normal((81, 3))
    ref = (K if j is None else dKs[j]) @ X
    out = apply_covariance(dim, N, theta, X, which)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_tree_ordering_rule():
    # 1D: bisection keeps natural order
    t1 = Tree(1, 16, 2)
    assert np.array_equal(t1.perm, np.arange(16))
    assert t1.nodes[2] == [(0, 4), (4, 4), (8, 4), (12, 4)]
    # 2D 4x4, two levels: split x (tie) -> two 2x4 halves, then split y (longer side)
    t2 = Tree(2, 4, 2)
    # leaf 0: x in {0,1}, y in {0,1}; leaf 1: x in {0,1}, y in {2,3}; leaf 2: x in {2,3}, y in {0,1}
    assert list(t2.perm[:4]) == [0, 1, 4, 5]
    assert list(t2.perm[4:8]) == [8, 9, 12, 13]
    assert list(t2.perm[8:12]) == [2, 3, 6, 7]
    assert sorted(t2.perm) == list(range(16))
    # odd side: left child gets floor(side/2)
    t3 = Tree(2, 5, 1)
    assert t3.nodes[1] == [(0, 10), (10, 15)]


def test_to_tree_order_is_a_similarity():
    tree = Tree(2, 6, 2)
    rng = np.random.default_rng(4)
    A = rng.standard_normal((36, 36))
    A = A + A.T
    At = to_tree_order(tree, A)
    assert np.allclose(np.sort(np.linalg.eigvalsh(At)), np.sort(np.linalg.eigvalsh(A)))
