"""Dense covariance operators given by a kernel function on scattered points (the
oracle side of a caller-supplied operator; Sec. 2.1: any covariance reached only
through products K v and dK/dtheta_j v).

matern32(coords, ell, a): the Matern covariance of smoothness 3/2,
    k(d) = (1 + sqrt(3) d / ell) exp(-sqrt(3) d / ell),
with an anisotropic distance d = sqrt(dx^2 + (a dy)^2) (a = 1: isotropic), and its
derivatives in ell and a, written from differentiating k:
    with r = sqrt(3) d / ell:   dk/dell = r^2 exp(-r) / ell,
                                dk/da   = -3 a dy^2 exp(-r) / ell^2.
Parity: pinned by central differences and by symmetry / positive semidefiniteness
(tests/test_oracle_operators.py).
"""
from __future__ import annotations

import numpy as np


def matern32(coords, ell: float, a: float):
    """(K, dK/dell, dK/da) for the points coords (n x dim), in the points' order."""
    xy = np.asarray(coords, dtype=np.float64)
    if xy.ndim == 1:
        xy = xy[:, None]
    dx = xy[:, None, 0] - xy[None, :, 0]
    dy = (xy[:, None, 1] - xy[None, :, 1]) if xy.shape[1] == 2 else np.zeros_like(dx)
    d = np.sqrt(dx * dx + (a * dy) ** 2)
    r = np.sqrt(3.0) * d / ell
    e = np.exp(-r)
    K = (1.0 + r) * e
    dK_ell = r * r * e / ell
    dK_a = -3.0 * a * dy * dy * e / (ell * ell)
    return K, dK_ell, dK_a
