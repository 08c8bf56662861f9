"""Maximum-likelihood fit over the library, on the HODLR likelihood L~.

The estimate is the root of the approximate score equations (Sec. 4.3, eq. "score
approximated"); every evaluation is one `hm_iteration` (L~, its gradient and the
expected Fisher matrix of eq. "fisher info approximated" in one pass).  Intervals
follow the asymptotic normality of the estimator (Sec. 2, eq. "CLT"):
theta_j +- 1.96 sqrt((I~^{-1})_jj).

The paper leaves the optimiser open (quasi-Newton methods in the text, MATLAB's in the
experiments).  This driver works in log-parameters phi = log(theta) (the score there is
theta_j S_j and the information theta_i theta_j I_ij): a quasi-Newton (BFGS) iteration
whose curvature model starts at the expected information I~ (the first step is a
Fisher-scoring step) and is updated with the score differences, since I~ can differ from
the curvature of L~ enough to stall plain scoring.  Each step is capped to a change of
max_log_step in any log-parameter and, far from the optimum, halved until L~ does not
decrease; the fit stops when the scoring decrement sqrt(S^T I~^{-1} S), the distance to
the optimum in standard errors, is below tol.  The sketches stay those of the HMatrix's
Sketch (fixed across iterations, Sec. 3.3).  Only the p x p step solve runs on the host.
"""
from __future__ import annotations

import time

import numpy as np

from .hmle import PARAM_NAMES, HmleError


def fit(H, y, theta_full, max_iter=200, tol=1e-6, max_log_step=2.0, min_step=2.0 ** -20, local=0.1):
    """Fit the free parameters of H (those it was created with) starting from theta_full.

    H: an HMatrix; y: device vector (grid order, as for H.iteration); theta_full: the
    four model parameters, the free ones being the starting point.  Stops when the
    scoring decrement sqrt(S^T I~^{-1} S) (the step length in standard errors) is below
    tol.  Far from the optimum (decrement >= local) a trial step is accepted when L~ does
    not decrease; closer, where the quadratic model holds and changes of L~ approach its
    rounding, the full scoring step is taken.  Returns a dict with theta (free), theta_full, loglik, grad_nll, fim,
    se, ci95 (free x 2), decrement, converged, iterations, evaluations, seconds and
    history (per accepted step: theta, loglik, step length)."""
    idx = list(H.free_idx)
    free = [PARAM_NAMES[i] for i in idx]
    base = np.array(theta_full, dtype=np.float64)
    if np.any(base[idx] <= 0):
        raise ValueError("the free parameters must start positive")

    def full(phi):
        th = base.copy()
        th[idx] = np.exp(phi)
        return th

    evals = 0

    def evaluate(phi):
        nonlocal evals
        evals += 1
        return H.iteration(full(phi), y)

    t0 = time.perf_counter()
    phi = np.log(base[idx])
    ll, g, fim = evaluate(phi)
    history = [dict(theta=np.exp(phi), loglik=ll, step=0.0)]
    x = np.exp(phi)
    score = -g * x                      # dL~/dphi
    B = fim * np.outer(x, x)            # curvature model, started at the information
    it, dec, converged = 0, np.inf, False
    while it < max_iter:
        info = fim * np.outer(x, x)
        dec = float(np.sqrt(max(score @ np.linalg.solve(info, score), 0.0)))
        if dec < tol:
            converged = True
            break
        it += 1
        step = np.linalg.solve(B, score)
        big = np.max(np.abs(step))
        if big > max_log_step:
            step *= max_log_step / big
        t = 1.0
        accepted = False
        while t >= min_step:
            cand = phi + t * step
            try:
                ll_c, g_c, fim_c = evaluate(cand)
            except HmleError:   # e.g. a trial point where K~ is not positive definite
                t *= 0.5
                continue
            if ll_c >= ll or dec < local:
                accepted = True
                break
            t *= 0.5
        if not accepted:
            break
        x_c = np.exp(cand)
        score_c = -g_c * x_c
        # BFGS update of the curvature with the secant pair (step, change of -score);
        # without positive curvature along the step, restart from the information
        sv, yv = cand - phi, score - score_c
        sy = float(sv @ yv)
        if sy > 1e-12 * float(np.linalg.norm(sv) * np.linalg.norm(yv)):
            Bs = B @ sv
            B = B - np.outer(Bs, Bs) / float(sv @ Bs) + np.outer(yv, yv) / sy
        else:
            B = fim_c * np.outer(x_c, x_c)
        phi, ll, g, fim, x, score = cand, ll_c, g_c, fim_c, x_c, score_c
        history.append(dict(theta=x, loglik=ll, step=t))
    th = np.exp(phi)
    se = np.sqrt(np.diag(np.linalg.inv(fim)))
    return dict(theta=th, theta_full=full(phi), free=free, loglik=ll, grad_nll=g, fim=fim, se=se,
                ci95=np.stack([th - 1.96 * se, th + 1.96 * se], axis=1), decrement=dec, converged=converged,
                iterations=it, evaluations=evals, seconds=time.perf_counter() - t0, history=history)


def fit_schedule(model, omega, y, theta_full, free, ranks, oversample, rank_tol=None, **fit_kw):
    """Fits at increasing off-diagonal ranks, each stage starting from the previous
    estimate with its sketch re-created there (sketch refresh): cheap low-rank
    iterations far from the optimum, the target rank near it (the strategy the paper
    suggests for its experiments).

    model: Model; omega: device tensor (levels, ell_max, n) of N(0,1) draws with
    ell_max >= max(ranks) + oversample (stage r uses its first r + oversample columns);
    y: device vector; theta_full: starting parameters; free: parameter names.  Returns
    the last stage's fit with "stages" (per stage: rank, kept panel width, seconds of
    sketch creation, the fit) and "seconds" (all stages, sketch creation included)."""
    from .hmle import HMatrix, Sketch

    theta = np.array(theta_full, dtype=np.float64)
    stages, total, res = [], 0.0, None
    for r in ranks:
        ell = r + oversample
        if ell > omega.shape[1]:
            raise ValueError("omega has fewer columns than rank + oversample")
        t0 = time.perf_counter()
        om = omega[:, :ell, :].contiguous()
        s = Sketch(model, om, r, oversample, theta, rank_tol)
        del om
        H = HMatrix(s, free)
        t_sketch = time.perf_counter() - t0
        try:
            res = fit(H, y, theta, **fit_kw)
        finally:
            H.close()
            kc = s.ranks()[1]
            s.close()
        theta = res["theta_full"]
        total += t_sketch + res["seconds"]
        stages.append(dict(rank=r, kc=kc, sketch_seconds=t_sketch, fit=res))
    out = dict(res)
    out["stages"] = stages
    out["seconds"] = total
    return out
