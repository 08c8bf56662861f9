"""Maximum-likelihood estimate by Fisher scoring on the dense likelihood (test
infrastructure only: tests/ may import this module; the library never does).

The estimator is the root of the score equations (Sec. 2, eq. "score"); its
asymptotic covariance is the inverse expected Fisher information (Sec. 2, eqs.
"fisher info" and "CLT"), so 95% intervals are theta_j +- 1.96 sqrt((I^{-1})_jj).
The paper leaves the optimiser open (it names quasi-Newton methods and uses MATLAB's);
this oracle takes the plain Fisher-scoring iteration in log-parameters
phi = log(theta), where the score is theta_j S_j and the information
theta_i theta_j I_ij, with step halving until the log-likelihood does not decrease
(beyond rounding).

Parity: pinned by tests/test_oracle_mle.py (the converged score vanishes, two
starting points agree, and an independent quasi-Newton minimiser (scipy's L-BFGS-B on
-L) finds the same point).
"""
from __future__ import annotations

import numpy as np

from oracle.exact import likelihood_gradient_fisher
from oracle.model import PARAMS, dense_covariance


def exact_evaluator(dim, N, theta_full, free, y):
    """theta (free entries) -> (loglik, grad_nll, fim) of the exact covariance."""
    idx = [PARAMS.index(f) for f in free]
    base = np.array(theta_full, dtype=np.float64)

    def evaluate(theta_free):
        th = base.copy()
        th[idx] = theta_free
        K, dKs = dense_covariance(dim, N, th, free)
        r = likelihood_gradient_fisher(K, dKs, y)
        return r["loglik"], np.asarray(r["grad_nll"]), np.asarray(r["fim"])

    return evaluate


def spectral_evaluator(dim, N, theta_full, free, y):
    """theta (free entries) -> (loglik, grad_nll, fim) of the exact covariance in its
    closed form (DST-I eigenbasis; oracle/spectral.py)."""
    from oracle.spectral import spectral_quantities

    idx = [PARAMS.index(f) for f in free]
    base = np.array(theta_full, dtype=np.float64)

    def evaluate(theta_free):
        th = base.copy()
        th[idx] = theta_free
        r = spectral_quantities(dim, N, th, y, free)
        return r["loglik"], np.asarray(r["grad_nll"]), np.asarray(r["fim"])

    return evaluate


def fisher_scoring(evaluate, theta0, max_iter=100, tol=1e-9):
    """Fisher scoring in log-parameters until the scoring decrement sqrt(S^T I^{-1} S)
    (the step in standard errors, the same in any parametrisation) is below tol.
    Returns dict(theta, loglik, grad_nll, fim, se, ci95, decrement, iterations); se and
    ci95 in theta units."""
    phi = np.log(np.asarray(theta0, dtype=np.float64))
    ll, g, fim = evaluate(np.exp(phi))
    it, dec = 0, np.inf
    while it < max_iter:
        th = np.exp(phi)
        score = -g * th                       # dL/dphi
        info = fim * np.outer(th, th)         # information in phi
        step = np.linalg.solve(info, score)
        dec = float(np.sqrt(max(score @ step, 0.0)))
        if dec < tol:
            break
        it += 1
        t = 1.0
        while True:
            cand = phi + t * step
            ll_c, g_c, fim_c = evaluate(np.exp(cand))
            if ll_c >= ll - 1e-13 * abs(ll) or t < 1e-6:
                break
            t *= 0.5
        phi, ll, g, fim = cand, ll_c, g_c, fim_c
    th = np.exp(phi)
    se = np.sqrt(np.diag(np.linalg.inv(fim)))
    return dict(theta=th, loglik=ll, grad_nll=g, fim=fim, se=se,
                ci95=np.stack([th - 1.96 * se, th + 1.96 * se], axis=1), decrement=dec, iterations=it)
