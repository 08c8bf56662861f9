"""Gaussian log-likelihood, NLL gradient and Fisher information from their definitions.

Sec. 2.2:  L = -n/2 log(2 pi) - 1/2 log|K| - 1/2 y^T K^{-1} y         (eq. "log-like")
           S_j = -1/2 tr(K^{-1} K_j) + 1/2 y^T K^{-1} K_j K^{-1} y    (eq. "score")
           I_ij = 1/2 tr(K^{-1} K_i K^{-1} K_j)                       (eq. "fisher info")
The gradient returned is that of the negative log-likelihood, g = -S.
Works for the exact K (Sec. 2) and, unchanged, for the HODLR approximation K~
(Sec. 4, eqs. "log-like approximated", "score approximated", "fisher info
approximated"), since those are the same definitions with K replaced by K~.

Parity: pinned by the spectral closed form, finite differences and brute-force
traces (tests/test_oracle_model.py).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


def loglik_terms(K: np.ndarray, y: np.ndarray):
    """(loglik, logdet, z = K^{-1} y) via a dense Cholesky factorisation."""
    n = K.shape[0]
    c = sla.cho_factor(K, lower=True)
    logdet = 2.0 * float(np.sum(np.log(np.diag(c[0]))))
    z = sla.cho_solve(c, y)
    ll = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * float(y @ z)
    return ll, logdet, z


def likelihood_gradient_fisher(K: np.ndarray, dKs, y: np.ndarray):
    """Return dict(loglik, logdet, z, grad_nll[p], fim[p,p]) from dense K and dK_j."""
    n = K.shape[0]
    c = sla.cho_factor(K, lower=True)
    logdet = 2.0 * float(np.sum(np.log(np.diag(c[0]))))
    z = sla.cho_solve(c, y)
    ll = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * float(y @ z)
    Ms = [sla.cho_solve(c, dK) for dK in dKs]          # M_j = K^{-1} K_j
    p = len(dKs)
    grad = np.array([0.5 * np.trace(Ms[j]) - 0.5 * float(z @ (dKs[j] @ z)) for j in range(p)])
    fim = np.empty((p, p))
    for i in range(p):
        for j in range(p):
            # tr(M_i M_j) = sum_ab (M_i)_ab (M_j)_ba
            fim[i, j] = 0.5 * float(np.sum(Ms[i] * Ms[j].T))
    return dict(loglik=ll, logdet=logdet, z=z, grad_nll=grad, fim=fim)


def trace_of_product_bruteforce(A: np.ndarray, B: np.ndarray) -> float:
    """tr(AB) by the plain double sum; used to pin the vectorised form above."""
    n = A.shape[0]
    s = 0.0
    for a in range(n):
        for b in range(n):
            s += A[a, b] * B[b, a]
    return s
