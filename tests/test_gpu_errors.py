"""GPU: error paths of the library, forced from the host (every kernel still
completes normally; failures are reported through the device status flags)."""
import numpy as np
import pytest

from tests._cases import gpu_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def test_not_spd_is_reported():
    # The 64 x 64 workload with a physics scale far above what rank 48 resolves
    # (unit marginal variance, sigma2 ~ 5e8): the fixed-rank K~ is indefinite, so the
    # factorisation must stop with HM_E_NOT_SPD instead of returning numbers.
    _need_gpu()
    from dataclasses import replace

    from paper_2303_10102_amd import hmle
    from synth import WORKLOADS, sample_y
    w = replace(WORKLOADS["2d_n4096"], sigma2=5.3e8)
    _, m, s, H = gpu_case(w)
    y = torch.from_numpy(sample_y(w)).cuda()
    with pytest.raises(hmle.HmleError) as ei:
        H.iteration(w.theta_full, y)
    assert ei.value.status == "HM_E_NOT_SPD"
    # the handle stays usable at a valid theta
    ok = replace(w, sigma2=1.0)
    ll, g, fim = H.iteration(ok.theta_full, y)
    assert np.isfinite(ll) and np.all(np.isfinite(fim))
    H.close(); s.close(); m.close()


def test_state_and_argument_errors():
    _need_gpu()
    from paper_2303_10102_amd import hmle
    from tests._cases import CASES
    w, m, s, H = gpu_case(CASES["1d_n1024"])
    with pytest.raises(hmle.HmleError) as ei:
        H.fisher()                      # before build / factor
    assert ei.value.status == "HM_E_STATE"
    bad = np.array(w.theta_full)
    bad[2] = -1.0                       # tau2 <= 0
    with pytest.raises(hmle.HmleError) as ei:
        H.build(bad)
    assert ei.value.status == "HM_E_INVAL"
    bad[2] = np.nan
    with pytest.raises(hmle.HmleError) as ei:
        H.build(bad)
    assert ei.value.status == "HM_E_NONFINITE"
    H.close(); s.close(); m.close()
