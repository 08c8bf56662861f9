"""Observed subsets of the stencil field (oracle side; test infrastructure only).

Observations of a selection of grid points (Sec. 5.1, eq. "projection", with the
observation operator Phi a selection: each observation reads one grid node; Sec. 5.2.1
builds its smaller data sets this way, by subsampling the grid):
    K_obs = sigma2 Phi M M^T Phi^T + tau2 I,   M = A^{-1} B^{-1},
where the physics stays on the full N x N (or N) grid and the nugget acts on the
observations only.

Dense assembly without a dense full-grid matrix: A and B are polynomials in the
Dirichlet -Laplacian, which the orthonormal DST-I S diagonalises (S_pi =
sqrt(2/(N+1)) sin(pi p i/(N+1)), mu_p = (4/h^2) sin^2(p pi h/2)), so
    (M M^T)[g, g'] = sum_modes lam_e S_e(g) S_e(g'),  lam = 1 / ((1 + alpha mu)^2 (kappa^2 + mu)^2).
In 2D S_e(g) = S_p(x) S_q(y) for mode e = (p, q) and node g = (x, y), so the sum over
modes factorises into one pass over the y modes and one over the x modes.  The
derivatives replace lam by d lam / d kappa = -4 kappa lam / b and
d lam / d alpha = -2 mu lam / a (a = 1 + alpha mu, b = kappa^2 + mu).

Parity: pinned against the sparse-solve assembly of oracle.model.dense_covariance
restricted to the selected rows and columns (tests/test_oracle_selection.py).
"""
from __future__ import annotations

import math

import numpy as np

PARAMS = ("kappa", "alpha", "tau2", "sigma2")


def _sine_basis(N: int) -> np.ndarray:
    """S[p, i], p, i = 0..N-1 (mode p+1 at node i+1)."""
    i = np.arange(1, N + 1, dtype=np.float64)
    return math.sqrt(2.0 / (N + 1)) * np.sin(math.pi * np.outer(i, i) / (N + 1))


def _mu(N: int) -> np.ndarray:
    h = 1.0 / (N + 1)
    p = np.arange(1, N + 1, dtype=np.float64)
    return (4.0 / (h * h)) * np.sin(p * math.pi * h / 2.0) ** 2


def _mode_sum(dim: int, N: int, weight, obs: np.ndarray) -> np.ndarray:
    """sum_e weight_e S_e(g) S_e(g') for g, g' in obs (grid indices, x fastest in 2D).

    weight: function (mu_x, mu_y) -> per-mode weight array (1D: mu_y is None)."""
    S = _sine_basis(N)
    mu = _mu(N)
    obs = np.asarray(obs, dtype=np.int64)
    if dim == 1:
        Sg = S[:, obs]                                   # modes x obs
        w = weight(mu, None)
        return (Sg * w[:, None]).T @ Sg
    gx, gy = obs % N, obs // N
    W = weight(mu[:, None], mu[None, :])                 # W[p, q]: x mode p, y mode q
    xs, ys = np.unique(gx), np.unique(gy)
    if obs.size == xs.size * ys.size and np.array_equal(obs, (ys[:, None] * N + xs[None, :]).ravel()):
        # a tensor-product selection (every x of xs on every y of ys, y outer): with
        # X = S[:, xs], Y = S[:, ys], K[(j, i), (j', i')] = sum_p X[p,i] X[p,i'] R[p, j, j'],
        # R[p, j, j'] = sum_q W[p, q] Y[q, j] Y[q, j']
        X, Y = S[:, xs], S[:, ys]
        R = np.einsum("pq,qj,ql->pjl", W, Y, Y, optimize=True)
        P = np.einsum("pi,pk->pik", X, X)
        K4 = (P.reshape(N, -1).T @ R.reshape(N, -1)).reshape(xs.size, xs.size, ys.size, ys.size)
        return K4.transpose(2, 0, 3, 1).reshape(obs.size, obs.size)
    Sx, Sy = S[:, gx], S[:, gy]                          # modes x obs, per axis
    # sum_{p,q} W[p,q] Sx[p,g] Sx[p,g'] Sy[q,g] Sy[q,g']:
    #   R[p, g, g'] = sum_q W[p, q] Sy[q, g] Sy[q, g'], then sum_p Sx[p,g] Sx[p,g'] R[p,g,g']
    n = obs.size
    out = np.zeros((n, n))
    for p in range(N):
        R = (Sy * W[p][:, None]).T @ Sy
        out += np.outer(Sx[p], Sx[p]) * R
    return out


def selected_covariance(dim: int, N: int, theta_full, obs, free=PARAMS):
    """(K_obs, [dK_obs/dtheta_j for j in free]) with rows and columns in the order of obs."""
    kappa, alpha, tau2, sigma2 = [float(t) for t in theta_full]

    def parts(mx, my):
        mu = mx if my is None else mx + my
        a = 1.0 + alpha * mu
        b = kappa * kappa + mu
        return mu, a, b, 1.0 / (a * a * b * b)

    phys = _mode_sum(dim, N, lambda mx, my: parts(mx, my)[3], obs)
    n = phys.shape[0]
    K = sigma2 * phys + tau2 * np.eye(n)
    dKs = []
    for name in free:
        if name == "kappa":
            d = sigma2 * _mode_sum(dim, N, lambda mx, my: -4.0 * kappa * parts(mx, my)[3] / parts(mx, my)[2], obs)
        elif name == "alpha":
            def wa(mx, my):
                mu, a, b, lam = parts(mx, my)
                return -2.0 * mu * lam / a
            d = sigma2 * _mode_sum(dim, N, wa, obs)
        elif name == "tau2":
            d = np.eye(n)
        elif name == "sigma2":
            d = phys.copy()
        else:
            raise ValueError(name)
        dKs.append(0.5 * (d + d.T))
    return 0.5 * (K + K.T), dKs


def grid_coords(dim: int, N: int, obs) -> np.ndarray:
    """Coordinates (node indices) of the selected grid points: (n,) in 1D, (n, 2) = (x, y) in 2D."""
    obs = np.asarray(obs, dtype=np.int64)
    if dim == 1:
        return obs.astype(np.float64)
    return np.stack([obs % N, obs // N], axis=1).astype(np.float64)
