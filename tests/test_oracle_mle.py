"""Oracle maximum-likelihood fits (CPU): oracle/mle.py against what fixes the MLE
independently of the scoring iteration.

* At the fit the score vanishes: the scoring decrement is below 1e-8 and central
  differences of L in log-parameters (step 1e-4, no gradient formula involved) are
  zero to their truncation and rounding error; L there is not below L at the start or
  at the generating parameters.
* Two starting points reach the same point, and so does an independent minimiser
  (scipy's L-BFGS-B on -L).
* The closed-form (spectral) likelihood and the dense one give the same fit on a grid
  small enough for both, which pins the spectral fits used at 128^2 and 256^2."""
import numpy as np
import pytest

from tests._cases import CASES, oracle_mle


def _evaluator(key, kind="dense"):
    from oracle.mle import exact_evaluator, spectral_evaluator
    from synth import sample_y

    w = CASES[key]
    make = exact_evaluator if kind == "dense" else spectral_evaluator
    return w, make(w.dim, w.N, w.theta_full, w.free, sample_y(w))


def test_fit_is_a_stationary_maximum():
    r = oracle_mle("1d_mle")
    assert r["decrement"] < 1e-8
    w, ev = _evaluator("1d_mle")
    phi = np.log(r["theta"])
    h = 1e-4
    fd = np.empty(len(phi))
    for j in range(len(phi)):
        e = np.zeros(len(phi))
        e[j] = h
        fd[j] = (ev(np.exp(phi + e))[0] - ev(np.exp(phi - e))[0]) / (2 * h)
    info_phi = r["fim"] * np.outer(r["theta"], r["theta"])
    # score in standard-error units; truncation ~h^2 L''' and rounding ~1e-13 |L| / h
    assert np.max(np.abs(fd) / np.sqrt(np.diag(info_phi))) < 1e-4
    assert r["loglik"] >= ev(np.asarray(w.theta))[0]
    assert r["loglik"] >= ev(np.asarray(w.theta) * 1.3)[0]


def test_two_starts_agree():
    a = oracle_mle("1d_mle", 1.3)
    b = oracle_mle("1d_mle", 0.7)
    assert np.max(np.abs(a["theta"] - b["theta"]) / a["se"]) < 1e-6


def test_quasi_newton_agrees():
    from scipy.optimize import minimize

    r = oracle_mle("1d_mle")
    w, ev = _evaluator("1d_mle")

    def f(phi):
        ll, g, _ = ev(np.exp(phi))
        return -ll, g * np.exp(phi)

    res = minimize(f, np.log(np.asarray(w.theta) * 1.3), jac=True, method="L-BFGS-B",
                   options=dict(maxiter=200, gtol=1e-10, ftol=1e-15))
    assert np.max(np.abs(np.exp(res.x) - r["theta"]) / r["se"]) < 1e-3


def test_spectral_fit_matches_dense():
    d = oracle_mle("2d_mle_32", evaluator="dense")
    s = oracle_mle("2d_mle_32", evaluator="spectral")
    assert d["decrement"] < 1e-8 and s["decrement"] < 1e-8
    assert np.max(np.abs(d["theta"] - s["theta"]) / d["se"]) < 1e-6
    assert np.max(np.abs(d["se"] / s["se"] - 1)) < 1e-6
