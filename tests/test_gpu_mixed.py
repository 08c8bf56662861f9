"""GPU: the mixed-precision policy (FP32 MFMA panel products, FP64 elsewhere).

Accuracy is judged against the exact closed form (oracle.spectral) with the
acceptance rule for the mixed path: each metric's error is at most twice the FP64
H-path's error, or below a floor of 1e-8 relative for L~ and 1e-6 for the gradient
and the Fisher matrix, whichever is larger.  Gradient errors are measured per
component in units of sqrt(I_jj) and Fisher errors in correlation units
I_ij / sqrt(I_ii I_jj) (the entries span twelve orders of magnitude).
"""
import numpy as np
import pytest

from tests._cases import CASES, gpu_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FLOOR = {"L": 1e-8, "g": 1e-6, "I": 1e-6}
# BF16 keeps 8 significand bits: unit roundoff u = 2^-9.  Each trace panel entry carries a
# relative error of about 2u from its two rounded operands, averaged down over the panel's
# columns; the bounds allow 8u on a score (in sd) and 2u on a Fisher entry (in corr).
BF16_U = 2.0 ** -9
BF16_G_SD, BF16_I_CORR = 8 * BF16_U, 2 * BF16_U


def _metrics(ll, g, fim, ex):
    d = np.sqrt(np.diag(ex["fim"]))
    return {"L": abs(ll - ex["loglik"]) / abs(ex["loglik"]),
            "g": float(np.max(np.abs(g - ex["grad_nll"]) / d)),
            "I": float(np.max(np.abs(fim - ex["fim"]) / np.outer(d, d)))}


@pytest.mark.parametrize("key", ["1d_n1024", "2d_n4096", "2d_n16384", "2d_n65536"])
def test_mixed_accuracy(key):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from oracle.spectral import spectral_quantities
    from synth import WORKLOADS, sample_y
    w = CASES.get(key) or WORKLOADS[key]
    print(f"\n[mixed {key}]", flush=True)
    _, m, s, H = gpu_case(w)
    y = sample_y(w)
    yd = torch.from_numpy(y).cuda()
    ex = spectral_quantities(w.dim, w.N, w.theta_full, y, w.free)
    res = {}
    for prec in ("fp64", "mixed32"):
        H.set_precision(prec)
        ll, g, fim = H.iteration(w.theta_full, yd)
        res[prec] = _metrics(ll, g, fim, ex)
        d = np.sqrt(np.abs(np.diag(fim)))
        asym = float(np.max(np.abs(fim - fim.T) / np.outer(d, d)))
        print(prec, res[prec], "asymmetry", asym)
        # each (i, j) is computed independently: symmetric to the path's rounding
        assert asym <= (1e-12 if prec == "fp64" else FLOOR["I"])
    for k in ("L", "g", "I"):
        assert res["mixed32"][k] <= max(2.0 * res["fp64"][k], FLOOR[k]), k
    H.close(); s.close(); m.close()


@pytest.mark.parametrize("key", ["2d_n4096", "2d_n65536"])
def test_mixed_bf16_trace_panels(key):
    """Policy 2 changes only the trace panels: L~ is policy 1's exactly; the scores and
    the Fisher matrix carry BF16 rounding (unit roundoff 2^-9 of each operand), bounded
    here against the FP64 H path per entry."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from synth import WORKLOADS, sample_y
    w = CASES.get(key) or WORKLOADS[key]
    print(f"\n[mixed bf16 {key}]", flush=True)
    _, m, s, H = gpu_case(w)
    yd = torch.from_numpy(sample_y(w)).cuda()
    out = {}
    for prec in ("fp64", "mixed32", "mixedbf16"):
        H.set_precision(prec)
        out[prec] = H.iteration(w.theta_full, yd)
    H.set_precision("fp64")
    (l64, g64, f64), (l32, _, _), (lbf, gbf, fbf) = out["fp64"], out["mixed32"], out["mixedbf16"]
    assert lbf == l32
    d = np.sqrt(np.diag(f64))
    eg = float(np.max(np.abs(gbf - g64) / d))
    ei = float(np.max(np.abs(fbf - f64) / np.outer(d, d)))
    print(f"bf16 trace panels vs FP64 H: score {eg:.2e} sd, Fisher {ei:.2e} corr")
    assert np.all(np.isfinite(gbf)) and np.all(np.isfinite(fbf))
    assert eg < BF16_G_SD and ei < BF16_I_CORR
    H.close(); s.close(); m.close()
