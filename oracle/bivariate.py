"""Bivariate co-kriging covariance on the stencil grid (oracle side; test infrastructure only).

Two fields driven by one latent white noise w on the Dirichlet grid (the 2 x 2 block
covariance of co-located variables, the in-scope analogue of Sec. 5.2's bivariate wind
model, eq. "kphichi"; each block follows the cov model of Sec. 2.1 with the stencil
operators of Sec. 5.1):
    y1 = sigma B^{-1} w + tau1 eps1,   y2 = sigma A^{-1} B^{-1} w + tau2 eps2,
    K = sigma2 [[C, C A^{-T}], [A^{-1} C, A^{-1} C A^{-T}]] + diag(tau2_1 I, tau2_2 I),
    C = B^{-1} B^{-T},  B = kappa^2 I + T,  A = I + alpha T,  T = -Laplacian,
with theta_full = (kappa, alpha, tau2_1, sigma2, tau2_2) and the observation vector
stacked variable by variable, y = (y1; y2) (natural index v n_loc + g).

Co-located variables stay together in the ordering: the tree bisects the locations
(PairTree) and every location contributes its two rows, variable 1 first.

Parity: pinned against the per-mode 2 x 2 closed form in the sine basis, the
univariate model's marginals, alpha = 0 and central differences
(tests/test_oracle_bivariate.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle.model import _solve_dense, neg_laplacian

PARAMS = ("kappa", "alpha", "tau2", "sigma2", "tau2_2")


def bivariate_covariance(dim: int, N: int, theta_full, free=PARAMS):
    """(K, [dK/dtheta_j for j in free]) in natural order (variable-major), dense."""
    kappa, alpha, tau2a, sigma2, tau2b = [float(t) for t in theta_full]
    T = neg_laplacian(dim, N)
    nl = T.shape[0]
    eye = sp.identity(nl, format="csc")
    A = (eye + alpha * T).tocsc()
    B = (kappa * kappa * eye + T).tocsc()
    I = np.eye(nl)
    Mb = _solve_dense(B, I)                 # B^{-1}
    Ai = _solve_dense(A, I)                 # A^{-1}
    C = Mb @ Mb.T

    def blocks(Cm, Am, dCm=None, dAm=None):
        """sigma2-free physics blocks; with tangents, their derivative (product rule)."""
        if dCm is None and dAm is None:
            return np.block([[Cm, Cm @ Am.T], [Am @ Cm, Am @ Cm @ Am.T]])
        dC = dCm if dCm is not None else np.zeros_like(Cm)
        dA = dAm if dAm is not None else np.zeros_like(Am)
        return np.block([[dC, dC @ Am.T + Cm @ dA.T],
                         [dA @ Cm + Am @ dC, dA @ Cm @ Am.T + Am @ dC @ Am.T + Am @ Cm @ dA.T]])

    phys = blocks(C, Ai)
    nug1 = np.diag(np.r_[np.ones(nl), np.zeros(nl)])
    nug2 = np.diag(np.r_[np.zeros(nl), np.ones(nl)])
    K = sigma2 * phys + tau2a * nug1 + tau2b * nug2
    dKs = []
    for name in free:
        if name == "kappa":
            dMb = -2.0 * kappa * Mb @ Mb            # d B^{-1} / d kappa = -B^{-1} (2 kappa) B^{-1}
            d = sigma2 * blocks(C, Ai, dCm=dMb @ Mb.T + Mb @ dMb.T)
        elif name == "alpha":
            dAi = -_solve_dense(A, T @ Ai)          # d A^{-1} / d alpha = -A^{-1} T A^{-1}
            d = sigma2 * blocks(C, Ai, dAm=dAi)
        elif name == "tau2":
            d = nug1.copy()
        elif name == "tau2_2":
            d = nug2.copy()
        elif name == "sigma2":
            d = phys.copy()
        else:
            raise ValueError(name)
        dKs.append(0.5 * (d + d.T))
    return 0.5 * (K + K.T), dKs


class PairTree:
    """A location tree with nv co-located rows per location: nodes[d] = (offset, size)
    of the base tree's nodes scaled by nv; perm[nv i + v] = v n_loc + base.perm[i]."""

    def __init__(self, base, n_loc: int, nv: int = 2):
        self.levels = base.levels
        self.nodes = [[(nv * off, nv * sz) for off, sz in lst] for lst in base.nodes]
        self.perm = (np.asarray(base.perm, dtype=np.int64)[:, None] + n_loc * np.arange(nv)[None, :]).ravel()
        self.n = self.perm.size

    def rows(self, d: int, i: int) -> slice:
        off, sz = self.nodes[d][i]
        return slice(off, off + sz)

    @property
    def leaves(self):
        return self.nodes[-1]


def grid_locations(dim: int, N: int) -> np.ndarray:
    """Node coordinates of the whole grid (index y N + x in 2D), for the location KD-tree."""
    if dim == 1:
        return np.arange(N, dtype=np.float64)
    g = np.arange(N * N)
    return np.stack([g % N, g // N], axis=1).astype(np.float64)
