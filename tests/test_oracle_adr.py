"""CPU pins of the advection-diffusion-reaction oracle (oracle/adr.py)."""
import numpy as np

from oracle.adr import adr_operator, apply_adr_covariance, dense_adr_covariance


def test_operator_stencil_and_non_normality():
    N, kd, vx, vy, c = 6, 0.7, 2.0, -1.5, 0.3
    h = 1.0 / (N + 1)
    L = adr_operator(N, kd, vx, vy, c).toarray()
    # interior point (x, y) = (2, 3): its row by hand
    g = 3 * N + 2
    row = np.zeros(N * N)
    row[g] = 4 * kd / h**2 + c
    row[g - 1] = -kd / h**2 - vx / (2 * h)
    row[g + 1] = -kd / h**2 + vx / (2 * h)
    row[g - N] = -kd / h**2 - vy / (2 * h)
    row[g + N] = -kd / h**2 + vy / (2 * h)
    assert np.allclose(L[g], row, rtol=0, atol=1e-9)
    assert not np.allclose(L, L.T)
    assert not np.allclose(L @ L.T, L.T @ L)          # non-normal: L^{-1} and L^{-T} differ


def test_covariance_matches_sparse_solves_and_derivatives():
    N, kd, vx, vy = 7, 1.0, 3.0, 1.0
    th = np.array([6.0, 0.5, 1e-3, 2.0])
    free = ("kappa", "c", "tau2", "sigma2")
    K, dKs = dense_adr_covariance(N, kd, vx, vy, th, free)
    assert np.max(np.abs(K - K.T)) <= 1e-14 * np.max(np.abs(K))
    assert np.linalg.eigvalsh(K).min() > 0.9 * th[2]
    X = np.random.default_rng(1).standard_normal((N * N, 3))
    assert np.max(np.abs(K @ X - apply_adr_covariance(N, kd, vx, vy, th, X))) <= 1e-12 * np.max(np.abs(K @ X))
    for j, k in enumerate((0, 1, 2, 3)):
        hstep = 1e-4 * th[k]
        tp, tm = th.copy(), th.copy()
        tp[k] += hstep
        tm[k] -= hstep
        fd = (dense_adr_covariance(N, kd, vx, vy, tp, ())[0] - dense_adr_covariance(N, kd, vx, vy, tm, ())[0])
        fd /= 2 * hstep
        assert np.max(np.abs(fd - dKs[j])) <= 1e-6 * np.max(np.abs(dKs[j])), free[j]
