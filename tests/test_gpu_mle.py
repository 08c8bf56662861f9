"""GPU: maximum-likelihood fits with the library (paper_2303_10102_amd/mle.py).

* 1D, (kappa, tau2) free: K~ = K there (off-diagonal rank 4 < the sketch rank), so
  the fit must land on the oracle's exact MLE: within 1e-5 standard errors, with
  standard errors equal to 1e-5 relative.
* A rank schedule (8 then 16) with the sketch re-created at the first estimate reaches
  the same point, the second stage starting at the optimum.
* 128^2 in a physics-dominated regime, (kappa, tau2, sigma2) free: the fit of L~
  converges (decrement < 1e-6) and is compared with the exact MLE from the closed-form
  likelihood; the shift is the rank-32 approximation's (measured 0.83 standard errors
  at most), bounded here by 1.5."""
import numpy as np
import pytest

from tests._cases import CASES, gpu_case, oracle_mle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _fit(key):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2303_10102_amd.mle import fit
    from synth import sample_y
    print(f"\n[mle {key}]", flush=True)
    w, m, s, H = gpu_case(key)
    y = torch.from_numpy(sample_y(w)).cuda()
    th0 = w.theta_full.copy()
    th0[list(w.free_idx)] *= 1.3
    r = fit(H, y, th0)
    H.close(); s.close(); m.close()
    print(key, "iterations", r["iterations"], "evaluations", r["evaluations"], f"{r['seconds']:.3f} s",
          "theta", r["theta"], "se", r["se"], "decrement", r["decrement"], flush=True)
    return w, r


def test_fit_matches_oracle_1d():
    w, r = _fit("1d_mle")
    o = oracle_mle("1d_mle")
    assert r["converged"]
    assert np.max(np.abs(r["theta"] - o["theta"]) / o["se"]) < 1e-5
    assert np.max(np.abs(r["se"] / o["se"] - 1)) < 1e-5


def test_fit_128_against_exact_mle():
    w, r = _fit("2d_mle_128")
    o = oracle_mle("2d_mle_128", evaluator="spectral")
    shift = (r["theta"] - o["theta"]) / o["se"]
    print("exact MLE", o["theta"], "se", o["se"], "shift in standard errors", shift, flush=True)
    assert r["converged"] and r["decrement"] < 1e-6
    assert np.max(np.abs(shift)) < 1.5


def test_rank_schedule_with_refresh_1d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2303_10102_amd import hmle
    from paper_2303_10102_amd.mle import fit_schedule
    from synth import sample_y, sketch_draws
    w = CASES["1d_mle"]
    print("\n[mle schedule 1d_mle]", flush=True)
    m = hmle.Model(w.dim, w.N, w.leaf)
    om = torch.from_numpy(sketch_draws(w)).cuda()
    y = torch.from_numpy(sample_y(w)).cuda()
    th0 = w.theta_full.copy()
    th0[list(w.free_idx)] *= 1.3
    r = fit_schedule(m, om, y, th0, w.free, ranks=(8, w.rank), oversample=w.oversample)
    m.close()
    o = oracle_mle("1d_mle")
    print([(st["rank"], st["kc"], st["fit"]["iterations"]) for st in r["stages"]], r["theta"], flush=True)
    assert [st["rank"] for st in r["stages"]] == [8, w.rank]
    assert r["converged"]
    # the second stage starts at the first stage's estimate: few iterations remain
    assert r["stages"][1]["fit"]["iterations"] <= 3
    assert np.max(np.abs(r["theta"] - o["theta"]) / o["se"]) < 1e-5
