"""GPU: the kernel-family timing hooks used for the roofline figures.

Timing a family must not change what the iteration computes (the expand family is
timed by events that its own launches set, the others by events recorded around
their launches), and every family issued by an iteration reports launches, a positive
time no larger than the iteration's, and the algorithmic flops and bytes that the
host counts for those launches; switching the hooks off drops the records."""
import time

import numpy as np
import pytest

from tests._cases import gpu_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from synth import sample_y
    print("\n[case 2d_n4096 profile]", flush=True)
    w, m, s, H = gpu_case("2d_n4096")
    yd = torch.from_numpy(sample_y(w)).cuda()
    yield w, m, s, H, yd
    H.close(); s.close(); m.close()


@pytest.mark.parametrize("family", ["expand", "reduce", "dst", "leaf_gemm"])
def test_family_timing(case, family):
    w, m, s, H, yd = case
    ll0, g0, f0 = H.iteration(w.theta_full, yd)
    torch.cuda.synchronize()
    m.profile_enable(family)
    t = time.perf_counter()
    ll1, g1, f1 = H.iteration(w.theta_full, yd)
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t)
    p = m.profile_read()
    m.profile_enable(None)
    print(family, p, f"iteration {wall_ms:.2f} ms", flush=True)
    # identical results with the hooks on (same kernels, same order)
    assert ll1 == ll0
    assert np.array_equal(g1, g0) and np.array_equal(f1, f0)
    assert p["launches"] > 0
    assert 0.0 < p["ms"] <= wall_ms
    assert p["bytes"] > 0 and p["flops"] > 0
    # switching the hooks off drops the records, and nothing more is recorded
    H.iteration(w.theta_full, yd)
    torch.cuda.synchronize()
    assert m.profile_read()["launches"] == 0
