"""Stored oracle values (tests/golden/oracle_*.json, written by make_golden.py from
oracle/ only).

CPU: the oracle still reproduces them (a change to its arithmetic shows up here and
must name the passage that justifies it), and on the 1D case, whose off-diagonal
blocks have rank 4 < the sketch rank, the HODLR values equal the exact ones.
GPU: one iteration of the library on the same seeded inputs matches the stored
HODLR values to the parity tolerances (log-likelihood 1e-9; score per entry in units of
its standard deviation sqrt(I_jj) 1e-9, Fisher per entry in correlation units 1e-10)."""
import json
import os

import numpy as np
import pytest

from tests._cases import CASES, fim_err_corr, gpu_case, grad_err_sd, oracle_case

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KEYS = ("1d_n1024", "2d_n1024")


def _stored(key):
    with open(os.path.join(HERE, f"oracle_{key}.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("key", KEYS)
def test_oracle_reproduces_stored(key):
    g = _stored(key)
    r = oracle_case(key)["res"]
    assert g["n"] == CASES[key].n and g["params"] == list(CASES[key].free)
    assert abs(r["loglik"] - g["hodlr"]["loglik"]) <= 1e-11 * abs(g["hodlr"]["loglik"])
    assert abs(r["logdet"] - g["hodlr"]["logdet"]) <= 1e-11 * abs(g["hodlr"]["logdet"])
    fim = np.array(g["hodlr"]["fim"])
    assert grad_err_sd(r["grad_nll"], np.array(g["hodlr"]["grad_nll"]), fim) < 1e-9
    assert fim_err_corr(r["fim"], fim) < 1e-9


def test_rank_sufficient_case_is_exact():
    g = _stored("1d_n1024")
    h, e = g["hodlr"], g["exact"]
    assert abs(h["loglik"] - e["loglik"]) <= 1e-11 * abs(e["loglik"])
    fim = np.array(e["fim"])
    assert grad_err_sd(np.array(h["grad_nll"]), np.array(e["grad_nll"]), fim) < 1e-8
    assert fim_err_corr(np.array(h["fim"]), fim) < 1e-8


@pytest.mark.gpu
@pytest.mark.parametrize("key", KEYS)
def test_library_matches_stored(key):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from synth import sample_y
    print(f"\n[golden {key}]", flush=True)
    g = _stored(key)["hodlr"]
    w, m, s, H = gpu_case(key)
    y = torch.from_numpy(sample_y(w)).cuda()   # grid order, as the oracle's input
    ll, grad, fim = H.iteration(w.theta_full, y)
    H.close(); s.close(); m.close()
    ref = np.array(g["fim"])
    eg, ei = grad_err_sd(grad, np.array(g["grad_nll"]), ref), fim_err_corr(fim, ref)
    print(f"[golden {key}] gradient {eg:.2e} sd, Fisher {ei:.2e} corr")
    assert abs(ll - g["loglik"]) <= 1e-9 * abs(g["loglik"])
    assert eg < 1e-9
    assert ei < 1e-10
