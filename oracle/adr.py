"""Dense covariance of the advection-diffusion-reaction model (oracle side).

Sec. 5.3 (eqs. "ad1", "ad2"): the observed field u solves L u = phi with
    L u = -kd Lap u + v . grad u + c u,
and the latent source phi has the Matern covariance of the SPDE representation
(Sec. 5.1, eq. "latent covariance" with the mass matrix lumped to I): B^{-2},
B = kappa^2 I - Lap, kappa = 1 / length scale.  With a nugget,
    K = sigma2 L^{-1} B^{-2} L^{-T} + tau2 I,     theta = (kappa, c, tau2, sigma2).
In-scope reading: constant coefficients, central differences on the unit square with
Dirichlet boundary (h = 1/(N+1)) instead of the paper's finite elements and Neumann
boundary; L is not symmetric (v != 0), so L^{-1} and L^{-T} are different solves.

K is assembled by applying the solve chain to unit vectors (sparse LU of L, with the
transposed LU solve for L^{-T}); the derivatives follow the chain rule:
    dB/dkappa = 2 kappa I,   dL/dc = I.
Parity: pinned by central differences, symmetry / positive definiteness and the
non-normality of L (tests/test_oracle_adr.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .model import neg_laplacian


def central_gradient(N: int) -> sp.csc_matrix:
    """1D central difference (u[i+1] - u[i-1]) / (2h), Dirichlet (zero outside)."""
    h = 1.0 / (N + 1)
    off = np.ones(N - 1) / (2 * h)
    return sp.diags([-off, off], [-1, 1], format="csc")


def adr_operator(N: int, kd: float, vx: float, vy: float, c: float) -> sp.csc_matrix:
    """L = kd (-Lap) + vx d/dx + vy d/dy + c I on the N x N grid (index y N + x)."""
    T = neg_laplacian(2, N)
    G = central_gradient(N)
    eye = sp.identity(N, format="csc")
    Gx = sp.kron(eye, G)          # x fastest
    Gy = sp.kron(G, eye)
    return (kd * T + vx * Gx + vy * Gy + c * sp.identity(N * N, format="csc")).tocsc()


def dense_adr_covariance(N: int, kd: float, vx: float, vy: float, theta_full, free):
    """(K, [dK_j for j in free]) in natural grid order; free names: kappa, c, tau2, sigma2
    (c is the second parameter slot)."""
    kappa, c, tau2, sigma2 = [float(t) for t in theta_full]
    n = N * N
    L = spla.splu(adr_operator(N, kd, vx, vy, c))
    B = (kappa * kappa * sp.identity(n, format="csc") + neg_laplacian(2, N)).tocsc()
    Bf = spla.splu(B)
    I = np.eye(n)
    Binv = Bf.solve(I)
    M = L.solve(Binv)                      # L^{-1} B^{-1}
    Kphys = M @ M.T
    K = sigma2 * Kphys + tau2 * I
    K = 0.5 * (K + K.T)
    out = []
    for name in free:
        if name in ("kappa",):
            dM = L.solve(-2.0 * kappa * Bf.solve(Binv))      # L^{-1} (-2 kappa B^{-2})
            d = sigma2 * (dM @ M.T + M @ dM.T)
        elif name in ("c", "alpha"):
            dM = -L.solve(M)                                  # d(L^{-1})/dc = -L^{-1} L^{-1}
            d = sigma2 * (dM @ M.T + M @ dM.T)
        elif name == "tau2":
            d = I.copy()
        elif name == "sigma2":
            d = Kphys.copy()
        else:
            raise ValueError(name)
        out.append(0.5 * (d + d.T))
    return K, out


def apply_adr_covariance(N, kd, vx, vy, theta_full, X):
    """K X by sparse solves (L^{-T} by the transposed LU solve); X grid order (n,) or (n, c)."""
    kappa, c, tau2, sigma2 = [float(t) for t in theta_full]
    n = N * N
    L = spla.splu(adr_operator(N, kd, vx, vy, c))
    B = spla.splu((kappa * kappa * sp.identity(n, format="csc") + neg_laplacian(2, N)).tocsc())
    X = np.asarray(X, dtype=np.float64)
    v = L.solve(X, trans="T")
    v = B.solve(B.solve(v))
    return sigma2 * L.solve(v) + tau2 * X
