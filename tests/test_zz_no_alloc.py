"""GPU: hm_kapply_noalloc (fixed per-device scratch, no allocation) against hm_kapply.

Both run the same transform kernels; only the scratch and the column block size
differ, and every column is computed on its own, so the outputs agree to rounding
(bound 1e-14 relative to the largest entry of each column).  Two calls in a row share
the fixed scratch, the second with a smaller input (another model, fewer columns),
so a stale scratch from the first would show up in the second.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _call(fn, model, theta, X, which):
    from paper_2303_10102_amd import hmle
    c, n = X.shape
    Y = torch.full_like(X, float("nan"))
    st = getattr(hmle.lib(), fn)(model._h, hmle._theta(theta), C.c_void_p(X.data_ptr()), n, c,
                                 C.c_void_p(Y.data_ptr()), n, which)
    assert st == 0, hmle.lib().hm_last_error()
    return Y


def _colwise_rel(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return float(np.max(np.max(np.abs(a - b), axis=1) / np.max(np.abs(b), axis=1)))


def test_noalloc_kapply_matches_kapply():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2303_10102_amd import hmle
    from synth import WORKLOADS
    rng = np.random.default_rng(3)
    for key, c, which in (("2d_n16384", 70, 0), ("2d_n4096", 5, 2)):
        w = WORKLOADS[key]
        print(f"\n[noalloc {key} c={c} which={which}]", flush=True)
        m = hmle.Model(w.dim, w.N, w.leaf)
        X = torch.from_numpy(rng.standard_normal((c, w.n))).cuda()
        ref = _call("hm_kapply", m, w.theta_full, X, which)
        got = _call("hm_kapply_noalloc", m, w.theta_full, X, which)
        torch.cuda.synchronize()
        e = _colwise_rel(got, ref)
        print(f"column-wise relative difference {e:.2e}")
        assert e <= 1e-14
        m.close()


def test_noalloc_rejects_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2303_10102_amd import hmle
    from synth import WORKLOADS
    w = WORKLOADS["2d_n4096"]
    m = hmle.Model(w.dim, w.N, w.leaf)
    X = torch.zeros((2, w.n), dtype=torch.float64, device="cuda")
    L = hmle.lib()
    assert L.hm_kapply_noalloc(m._h, hmle._theta(w.theta_full), C.c_void_p(X.data_ptr()), w.n - 1, 2,
                               C.c_void_p(X.data_ptr()), w.n, 0) == 1
    assert L.hm_kapply_noalloc(m._h, hmle._theta(w.theta_full), C.c_void_p(X.data_ptr()), w.n, 2,
                               C.c_void_p(X.data_ptr()), w.n, 3) == 1
    m.close()
