"""CPU pins of the bivariate co-kriging covariance (oracle/bivariate.py).

The oracle assembles K = sigma2 [[C, C A^-T], [A^-1 C, A^-1 C A^-T]] + diag(tau2_1 I, tau2_2 I),
C = B^-1 B^-T, from sparse solves.  Pinned by routes that share none of that code:
  * the sine basis diagonalises A and B, so in it every mode e is a 2 x 2 block
    sigma2 / b_e^2 [[1, 1/a_e], [1/a_e, 1/a_e^2]] + diag(tau2_1, tau2_2) (a = 1 + alpha mu,
    b = kappa^2 + mu), zero between modes -- per-mode rank one in the physics;
  * each variable's marginal is the univariate model's covariance (oracle.model,
    itself pinned to the spectral closed form): variable 2 with (alpha, tau2_2),
    variable 1 with alpha = 0 and tau2_1;
  * central differences of K in all five parameters;
  * the pair tree keeps a location's two rows adjacent.
"""
import math

import numpy as np
import pytest

from oracle.bivariate import PairTree, bivariate_covariance, grid_locations
from oracle.model import PointTree, dense_covariance

THETA = (7.0, 3e-3, 0.02, 3.0, 0.05)


def _sine(N):
    i = np.arange(1, N + 1)
    return math.sqrt(2.0 / (N + 1)) * np.sin(math.pi * np.outer(i, i) / (N + 1))


@pytest.mark.parametrize("dim,N", [(2, 9), (1, 30)])
def test_modes_are_2x2_rank_one_blocks(dim, N):
    K, _ = bivariate_covariance(dim, N, THETA)
    S1 = _sine(N)
    S = S1 if dim == 1 else np.kron(S1, S1)          # index y N + x: kron(S_y, S_x)
    nl = S.shape[0]
    Q = np.zeros((2 * nl, 2 * nl))
    Q[:nl, :nl] = S
    Q[nl:, nl:] = S
    Kh = Q.T @ K @ Q
    h = 1.0 / (N + 1)
    mu1 = (4.0 / h ** 2) * np.sin(np.arange(1, N + 1) * math.pi * h / 2) ** 2
    mu = mu1 if dim == 1 else (mu1[None, :] + mu1[:, None]).ravel()
    kappa, alpha, t1, s2, t2 = THETA
    a, b = 1.0 + alpha * mu, kappa ** 2 + mu
    ref = np.zeros_like(Kh)
    ref[:nl, :nl] = np.diag(s2 / b ** 2 + t1)
    ref[:nl, nl:] = ref[nl:, :nl] = np.diag(s2 / (a * b ** 2))
    ref[nl:, nl:] = np.diag(s2 / (a * b) ** 2 + t2)
    assert np.abs(Kh - ref).max() <= 1e-12 * np.abs(ref).max()


def test_marginals_are_the_univariate_model():
    dim, N = 2, 8
    kappa, alpha, t1, s2, t2 = THETA
    K, _ = bivariate_covariance(dim, N, THETA)
    nl = N * N
    K2, _ = dense_covariance(dim, N, (kappa, alpha, t2, s2))
    K1, _ = dense_covariance(dim, N, (kappa, 0.0, t1, s2))
    assert np.abs(K[nl:, nl:] - K2).max() <= 1e-13 * np.abs(K2).max()
    assert np.abs(K[:nl, :nl] - K1).max() <= 1e-13 * np.abs(K1).max()
    # alpha = 0: all four physics blocks coincide
    K0, _ = bivariate_covariance(dim, N, (kappa, 0.0, t1, s2, t2))
    P = K0 - np.diag(np.r_[np.full(nl, t1), np.full(nl, t2)])
    for blk in (P[:nl, nl:], P[nl:, :nl], P[nl:, nl:]):
        assert np.abs(blk - P[:nl, :nl]).max() <= 1e-13 * np.abs(P).max()


def test_central_differences_in_every_parameter():
    dim, N = 2, 7
    th = np.array(THETA)
    _, dK = bivariate_covariance(dim, N, th)
    for j in range(5):
        hstep = 1e-5 * th[j]
        tp, tm = th.copy(), th.copy()
        tp[j] += hstep
        tm[j] -= hstep
        fd = (bivariate_covariance(dim, N, tp)[0] - bivariate_covariance(dim, N, tm)[0]) / (2 * hstep)
        assert np.abs(fd - dK[j]).max() <= 1e-6 * np.abs(dK[j]).max(), j


def test_symmetric_positive_definite_and_pair_tree():
    K, _ = bivariate_covariance(2, 10, THETA)
    assert np.array_equal(K, K.T)
    assert np.linalg.eigvalsh(K).min() > 0.5 * min(THETA[2], THETA[4])
    base = PointTree(grid_locations(2, 10), 2)
    t = PairTree(base, 100)
    assert t.n == 200 and sorted(t.perm.tolist()) == list(range(200))
    assert np.array_equal(t.perm[0::2], base.perm) and np.array_equal(t.perm[1::2], base.perm + 100)
    assert [sz for _, sz in t.leaves] == [2 * sz for _, sz in base.leaves]


def test_closed_form_likelihood_matches_the_dense_one():
    from oracle.bivariate import spectral_quantities
    from oracle.exact import likelihood_gradient_fisher
    for dim, N in ((2, 8), (1, 25)):
        K, dK = bivariate_covariance(dim, N, THETA)
        y = np.random.default_rng(8).standard_normal(K.shape[0])
        d = likelihood_gradient_fisher(K, dK, y)
        s = spectral_quantities(dim, N, THETA, y)
        assert abs(s["loglik"] - d["loglik"]) <= 1e-11 * abs(d["loglik"])
        sd = np.sqrt(np.diag(d["fim"]))
        assert np.max(np.abs(s["grad_nll"] - d["grad_nll"]) / sd) <= 1e-9
        assert np.max(np.abs(s["fim"] - d["fim"]) / np.outer(sd, sd)) <= 1e-10


def test_sparse_apply_matches_the_dense_assembly():
    from oracle.bivariate import apply_bivariate
    for dim, N in ((2, 9), (1, 30)):
        K, dK = bivariate_covariance(dim, N, THETA)
        X = np.random.default_rng(9).standard_normal((K.shape[0], 3))
        for which, M in (("K", K), ("kappa", dK[0]), ("alpha", dK[1])):
            Y = apply_bivariate(dim, N, THETA, X, which)
            assert np.abs(Y - M @ X).max() <= 1e-12 * np.abs(M @ X).max(), (dim, which)
