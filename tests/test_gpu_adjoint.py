"""GPU: the reverse-mode (adjoint) gradient and its torch.autograd wrapper.

The adjoint differentiates the same L~(theta) (fixed sketches) as the forward-mode
gradient of hm_loglik_grad, so the two agree up to rounding: per entry to 1e-9
relative (and 1e-9 of the score's standard deviation sqrt(I~_jj)), on the parity cases
and at full size (observed: 2e-13 and 2.3e-10 relative).  Both are also checked
against the oracle's gradient of its own peeling replay on the parity cases, per entry
in units of sqrt(I~_jj).  Two choices keep the rounding this small: the test matrices
of a level carry a common column scale that keeps the sketch QRs' R, which Alg. 2 and
its transpose divide by, well conditioned, and the nugget is added to K X row by row
instead of through the sine transforms.
"""
import math

import numpy as np
import pytest

from tests._cases import gpu_case, grad_err_sd, oracle_case, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.mark.parametrize("key", ["1d_n1024", "2d_n1024", "2d_n4096", "2d_n2025"])
def test_adjoint_matches_oracle_and_forward(key):
    _need_gpu()
    print(f"\n[adjoint {key}]", flush=True)
    o = oracle_case(key)
    w, m, s, H = gpu_case(key)
    y = torch.from_numpy(o["y"]).cuda()
    ll_a, g_a = H.loglik_grad_adjoint(w.theta_full, y)
    ll_f, g_f, fim = H.iteration(w.theta_full, y)
    r = o["res"]
    print("adjoint", g_a, "forward", g_f, "oracle", r["grad_nll"])
    assert abs(ll_a - ll_f) <= 1e-13 * abs(ll_f)
    eo = grad_err_sd(g_a, r["grad_nll"], r["fim"])
    ef = grad_err_sd(g_a, g_f, fim)
    erel = float(np.max(np.abs(g_a - g_f) / np.abs(g_f)))
    print(f"[{key}] adjoint vs oracle {eo:.2e} sd; vs forward {ef:.2e} sd, {erel:.2e} relative")
    assert abs(ll_a - r["loglik"]) <= 1e-9 * abs(r["loglik"])
    assert eo < 1e-9
    assert ef < 1e-9
    assert erel < 1e-9
    H.close(); s.close(); m.close()


def test_adjoint_full_size_and_state_guard():
    _need_gpu()
    from paper_2303_10102_amd import hmle
    from synth import WORKLOADS, sample_y
    w = WORKLOADS["2d_n65536"]
    print(f"\n[adjoint full size {w.name}]", flush=True)
    _, m, s, H = gpu_case(w)
    y = torch.from_numpy(sample_y(w)).cuda()
    ll_f, g_f, fim = H.iteration(w.theta_full, y)
    ll_a, g_a = H.loglik_grad_adjoint(w.theta_full, y)
    std = np.sqrt(np.diag(fim))
    dev = np.abs(g_a - g_f) / std
    rel = np.abs(g_a - g_f) / np.abs(g_f)
    print("adjoint", g_a, "\nforward", g_f, "\n|diff|/sqrt(I_jj)", dev, "\n|diff|/|g|", rel)
    assert abs(ll_a - ll_f) <= 1e-13 * abs(ll_f)
    assert np.max(dev) < 1e-9
    assert np.max(rel) < 1e-9
    # derivative matrices were not built by the adjoint call
    with pytest.raises(hmle.HmleError) as ei:
        H.fisher()
    assert ei.value.status == "HM_E_STATE"
    H.build(w.theta_full)
    H.factor()
    H.fisher()
    H.close(); s.close(); m.close()


def test_autograd_function():
    _need_gpu()
    from paper_2303_10102_amd import hmle
    key = "2d_n4096"
    o = oracle_case(key)
    w, m, s, H = gpu_case(key)
    y = torch.from_numpy(o["y"]).cuda().requires_grad_(True)
    theta = torch.tensor([w.theta_full[k] for k in H.free_idx], dtype=torch.float64, requires_grad=True)
    ll = hmle.HLogLik.apply(H, theta, y, w.theta_full)
    (2.0 * ll).backward()
    assert abs(ll.item() - o["res"]["loglik"]) <= 1e-9 * abs(o["res"]["loglik"])
    # d L~/d theta = -grad_nll; d L~/d y = -K~^{-1} y
    assert grad_err_sd(theta.grad.numpy(), -2.0 * o["res"]["grad_nll"], 4.0 * o["res"]["fim"]) < 1e-9
    zt = o["res"]["z"]
    zg = y.grad.detach().cpu().numpy()[o["tree"].perm]
    assert rel_err(zg, -2.0 * zt) < 1e-8
    H.close(); s.close(); m.close()
