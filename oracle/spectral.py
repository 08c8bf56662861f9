"""Closed-form likelihood quantities for the Dirichlet stencil model.

The 1D Dirichlet second-difference matrix and its 2D Kronecker sum are
diagonalised by the orthonormal DST-I basis S (S_pi = sqrt(2/(N+1)) sin(pi p i/(N+1))),
with eigenvalues mu_p = (4/h^2) sin^2(p pi h / 2) of T = -Laplacian.  A and B are
polynomials in T, so K = S diag(e) S with
    e = sigma2 / ((1 + alpha mu)^2 (kappa^2 + mu)^2) + tau2.
The quantities of Sec. 2.2 then reduce to sums over modes:
    L = -n/2 log 2pi - 1/2 sum log e - 1/2 sum yhat^2 / e,
    g_j = 1/2 sum de_j / e - 1/2 sum yhat^2 de_j / e^2,
    I_ij = 1/2 sum de_i de_j / e^2.
This is an independent route to the exact targets (no dense matrix), valid at
every n.  Parity: cross-checked with the dense assembly (tests/test_oracle_model.py).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

PARAMS = ("kappa", "alpha", "tau2", "sigma2")


def mode_eigenvalues(dim: int, N: int) -> np.ndarray:
    h = 1.0 / (N + 1)
    p = np.arange(1, N + 1, dtype=np.float64)
    mu1 = (4.0 / (h * h)) * np.sin(p * math.pi * h / 2.0) ** 2
    if dim == 1:
        return mu1
    return (mu1[:, None] + mu1[None, :]).ravel()   # index q*N + p (y mode outer)


def dst_grid(dim: int, N: int, y: np.ndarray) -> np.ndarray:
    """Orthonormal DST-I of a grid-ordered vector (x fastest)."""
    if dim == 1:
        return sfft.dst(y, type=1, norm="ortho")
    return sfft.dstn(y.reshape(N, N), type=1, norm="ortho").ravel()


def spectral_quantities(dim: int, N: int, theta_full, y: np.ndarray, free=PARAMS):
    kappa, alpha, tau2, sigma2 = [float(t) for t in theta_full]
    mu = mode_eigenvalues(dim, N)
    n = mu.size
    a = 1.0 + alpha * mu
    b = kappa * kappa + mu
    lam = sigma2 / (a * a * b * b)
    e = lam + tau2
    yh = dst_grid(dim, N, y)
    de = {
        "kappa": -4.0 * kappa * lam / b,
        "alpha": -2.0 * mu * lam / a,
        "tau2": np.ones_like(mu),
        "sigma2": lam / sigma2,
    }
    ll = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * float(np.sum(np.log(e))) - 0.5 * float(np.sum(yh * yh / e))
    g = np.array([0.5 * np.sum(de[f] / e) - 0.5 * np.sum(yh * yh * de[f] / (e * e)) for f in free])
    p = len(free)
    fim = np.empty((p, p))
    for i, fi in enumerate(free):
        for j, fj in enumerate(free):
            fim[i, j] = 0.5 * float(np.sum(de[fi] * de[fj] / (e * e)))
    return dict(loglik=ll, logdet=float(np.sum(np.log(e))), grad_nll=g, fim=fim, eigs=e)
