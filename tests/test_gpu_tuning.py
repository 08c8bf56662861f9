"""GPU: the panel-kernel autotuner.

The variants it chooses between (one or two 16-row blocks per wavefront and four or
eight wavefronts per workgroup in the expand, two or four wavefronts per leaf in the
reduce) compute the same sums in a
different order, so an iteration after tuning agrees with one under each forced
variant to rounding; the tuned choice is one of the timed variants and can be read
back and copied to another model."""
import numpy as np
import pytest

from tests._cases import fim_err_corr, gpu_case, grad_err_sd, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", params=["2d_n65536"])
def tuned(request):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from synth import WORKLOADS, sample_y
    w = WORKLOADS[request.param]
    print(f"\n[autotune {w.name}]", flush=True)
    w, m, s, H = gpu_case(w)
    yd = torch.from_numpy(sample_y(w)).cuda()
    yield w, m, s, H, yd
    H.close(); s.close(); m.close()


def test_autotune_report(tuned):
    w, m, s, H, yd = tuned
    _, kc = s.ranks()
    rep = m.autotune(kc)
    print(rep)
    times = list(rep["expand_ms"].values()) + list(rep["reduce_ms"].values())
    assert all(np.isfinite(t) and t > 0 for t in times)
    assert rep["expand_variant"] == min(rep["expand_ms"], key=rep["expand_ms"].get)
    thr = {"never": 0, "below_1024": 1024, "always": 1 << 40}
    assert rep["reduce_split_below"] == thr[min(rep["reduce_ms"], key=rep["reduce_ms"].get)]
    assert m.tuning() == (rep["expand_variant"], rep["reduce_split_below"])


def test_variants_agree(tuned):
    w, m, s, H, yd = tuned
    saved = m.tuning()
    out = {}
    try:
        for rb in (1, 2, 3):
            for thr in (0, 1 << 40):
                m.tuning(rb, thr)
                out[(rb, thr)] = H.iteration(w.theta_full, yd)
    finally:
        m.tuning(*saved)
    ll0, g0, f0 = H.iteration(w.theta_full, yd)
    for key, (ll, g, fim) in out.items():
        assert rel_err(ll, ll0) <= 1e-12, key
        # per entry: rounding order only
        assert grad_err_sd(g, g0, f0) <= 1e-9, key
        assert fim_err_corr(fim, f0) <= 1e-10, key


def test_tuning_rejects_bad_values(tuned):
    from paper_2303_10102_amd import hmle
    w, m, s, H, yd = tuned
    with pytest.raises(hmle.HmleError):
        m.tuning(4, 0)
    with pytest.raises(hmle.HmleError):
        m.autotune(0)
