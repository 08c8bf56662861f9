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


def spectral_quantities(dim: int, N: int, theta_full, y: np.ndarray, free=PARAMS):
    """Exact L, NLL gradient and Fisher matrix of the bivariate model at any size.

    In the orthonormal sine basis every mode e is an independent 2 x 2 block
        Kh_e = sigma2 / b^2 [[1, r], [r, r^2]] + diag(tau2_1, tau2_2),  r = 1/a,
    (a = 1 + alpha mu, b = kappa^2 + mu), so with yh_e = (S y1, S y2)_e
        L = -n/2 log 2 pi - 1/2 sum log det Kh_e - 1/2 sum yh_e^T Kh_e^-1 yh_e,
        g_j = 1/2 sum tr(Kh^-1 dKh_j) - 1/2 sum yh^T Kh^-1 dKh_j Kh^-1 yh,
        I_ij = 1/2 sum tr(Kh^-1 dKh_i Kh^-1 dKh_j)."""
    import math

    import scipy.fft as sfft

    kappa, alpha, t1, s2, t2 = [float(t) for t in theta_full]
    h = 1.0 / (N + 1)
    mu1 = (4.0 / (h * h)) * np.sin(np.arange(1, N + 1) * math.pi * h / 2.0) ** 2
    mu = mu1 if dim == 1 else (mu1[None, :] + mu1[:, None]).ravel()
    nl = mu.size
    a = 1.0 + alpha * mu
    b = kappa * kappa + mu
    r = 1.0 / a
    q = 1.0 / (b * b)

    def dst(v):
        return sfft.dst(v, type=1, norm="ortho") if dim == 1 else sfft.dstn(v.reshape(N, N), type=1,
                                                                             norm="ortho").ravel()

    y = np.asarray(y, dtype=np.float64)
    u, v = dst(y[:nl]), dst(y[nl:])
    # blocks as (p11, p12, p22) per mode
    K = (s2 * q + t1, s2 * q * r, s2 * q * r * r + t2)
    dr = -mu * r * r
    dq = -4.0 * kappa * q / b
    dK = {"kappa": (s2 * dq, s2 * dq * r, s2 * dq * r * r),
          "alpha": (0.0 * mu, s2 * q * dr, s2 * q * 2.0 * r * dr),
          "tau2": (np.ones(nl), 0.0 * mu, 0.0 * mu),
          "sigma2": (q, q * r, q * r * r),
          "tau2_2": (0.0 * mu, 0.0 * mu, np.ones(nl))}
    det = K[0] * K[2] - K[1] * K[1]
    Ki = (K[2] / det, -K[1] / det, K[0] / det)

    def mul(A, B):       # 2 x 2 symmetric-input products per mode, general result (11, 12, 21, 22)
        return (A[0] * B[0] + A[1] * B[1], A[0] * B[1] + A[1] * B[2],
                A[1] * B[0] + A[2] * B[1], A[1] * B[1] + A[2] * B[2])

    z1, z2 = Ki[0] * u + Ki[1] * v, Ki[1] * u + Ki[2] * v      # Kh^-1 yh
    ll = -0.5 * 2 * nl * math.log(2.0 * math.pi) - 0.5 * float(np.sum(np.log(det))) \
        - 0.5 * float(np.sum(u * z1 + v * z2))
    M = {}
    g = []
    for f in free:
        d = dK[f]
        P = mul(Ki, d)                                           # Kh^-1 dKh
        M[f] = P
        quad = z1 * (d[0] * z1 + d[1] * z2) + z2 * (d[1] * z1 + d[2] * z2)
        g.append(0.5 * float(np.sum(P[0] + P[3])) - 0.5 * float(np.sum(quad)))
    p = len(free)
    fim = np.empty((p, p))
    for i, fi in enumerate(free):
        for j, fj in enumerate(free):
            A, B = M[fi], M[fj]
            tr = A[0] * B[0] + A[1] * B[2] + A[2] * B[1] + A[3] * B[3]
            fim[i, j] = 0.5 * float(np.sum(tr))
    return {"loglik": ll, "grad_nll": np.array(g), "fim": fim}


def apply_bivariate(dim: int, N: int, theta_full, X: np.ndarray, which: str = "K") -> np.ndarray:
    """K X or dK/dtheta X (which in "K", "kappa", "alpha") by sparse solves, natural order,
    X of shape (2 n_loc,) or (2 n_loc, c).  With u = B^{-2}(x1 + A^{-1} x2) (A, B symmetric):
        K_op x = (u, A^{-1} u);
        d/dkappa: u -> -4 kappa B^{-3}(x1 + A^{-1} x2) in both blocks;
        d/dalpha: with dA^{-1} = -A^{-1} T A^{-1}, v = x1 + A^{-1} x2,
            (B^{-2} dA^{-1} x2,  dA^{-1} B^{-2} v + A^{-1} B^{-2} dA^{-1} x2)."""
    import scipy.sparse.linalg as spla

    kappa, alpha, t1, s2, t2 = [float(t) for t in theta_full]
    T = neg_laplacian(dim, N)
    nl = T.shape[0]
    eye = sp.identity(nl, format="csc")
    A = spla.splu((eye + alpha * T).tocsc())
    B = spla.splu((kappa * kappa * eye + T).tocsc())
    X = np.asarray(X, dtype=np.float64)
    x1, x2 = X[:nl], X[nl:]
    Ai2 = A.solve(x2)
    v = x1 + Ai2
    if which == "K":
        u = B.solve(B.solve(v))
        return np.concatenate([s2 * u + t1 * x1, s2 * A.solve(u) + t2 * x2])
    if which == "kappa":
        u = -4.0 * kappa * B.solve(B.solve(B.solve(v)))
        return s2 * np.concatenate([u, A.solve(u)])
    if which == "alpha":
        dAi2 = -A.solve(T @ Ai2)
        y1 = B.solve(B.solve(dAi2))
        w = B.solve(B.solve(v))
        y2 = -A.solve(T @ A.solve(w)) + A.solve(y1)
        return s2 * np.concatenate([y1, y2])
    raise ValueError(which)
