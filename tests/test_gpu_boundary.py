"""GPU: the boundary's context, statistics, multi-right-hand-side solve and the
forward / backward split of the likelihood.

* Device memory: a model created with a torch-backed context (the binding's default)
  takes every device buffer of its sketches and H handles from torch's caching
  allocator, so torch.cuda.memory_allocated() covers them and falls back on release;
  the results equal those of a context that lets the library call hipMalloc.
* hm_stats: one iteration does one construction with derivative matrices, one
  factorisation, one likelihood with gradient and one Fisher evaluation, and applies
  K to levels (2 + r) kc + n_leaf columns and dK/dtheta_j to 2 levels r kc + r n_leaf
  (r real parameters; two K-applies per level, the second also on the r tangent test
  matrices, then the stacked identities); every phase has device time.
* The autograd function's forward pass builds K~ without derivative matrices and runs
  no reverse sweep; backward runs exactly one and gives the adjoint gradient.
* hm_solve with several right-hand sides and a leading dimension > n equals the
  one-column solves, and the first column equals the oracle's K~^{-1} y.
"""
import ctypes as C

import numpy as np
import pytest

from tests._cases import CASES, gpu_case, oracle_case, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def test_torch_allocator_holds_the_device_memory():
    _need_gpu()
    from paper_2303_10102_amd import hmle
    from synth import sample_y, sketch_draws
    w = CASES["2d_n4096"]
    print("\n[allocator]", flush=True)
    torch.cuda.synchronize()
    a0 = torch.cuda.memory_allocated()
    w, m, s, H = gpu_case(w)
    torch.cuda.synchronize()
    a1 = torch.cuda.memory_allocated()
    held = H.stats()["device_bytes"]
    print(f"torch allocated {a1 - a0} bytes; H holds {held}")
    assert held > 0 and a1 - a0 >= held
    y = torch.from_numpy(sample_y(w)).cuda()
    res_torch = H.iteration(w.theta_full, y)
    H.close(); s.close(); m.close()
    torch.cuda.synchronize()
    a2 = torch.cuda.memory_allocated()
    assert a1 - a2 >= held
    # the same iteration with the library's own hipMalloc
    m2 = hmle.Model(w.dim, w.N, w.leaf, allocator="hip")
    om = torch.from_numpy(sketch_draws(w)).cuda()
    s2 = hmle.Sketch(m2, om, w.rank, w.oversample, w.theta_full)
    H2 = hmle.HMatrix(s2, w.free)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - a2 < held / 4   # only the sample and the draws
    res_hip = H2.iteration(w.theta_full, y)
    H2.close(); s2.close(); m2.close()
    assert res_torch[0] == res_hip[0]
    assert np.array_equal(res_torch[1], res_hip[1]) and np.array_equal(res_torch[2], res_hip[2])


def test_stats_count_the_iteration():
    _need_gpu()
    from synth import sample_y
    w, m, s, H = gpu_case("2d_n4096")
    y = torch.from_numpy(sample_y(w)).cuda()
    H.stats_reset()
    H.iteration(w.theta_full, y)
    st = H.stats()
    print("\n", st)
    _, kc = s.ranks()
    nr = sum(f in ("kappa", "alpha") for f in w.free)
    assert (st["builds"], st["deriv_builds"], st["factors"]) == (1, 1, 1)
    assert (st["loglik_evals"], st["grad_evals"], st["fisher_evals"], st["reverse_sweeps"]) == (1, 1, 1, 0)
    assert st["kapply_columns"] == m.levels * (2 + nr) * kc + m.leaf
    assert st["kapply_deriv_columns"] == 2 * m.levels * nr * kc + nr * m.leaf
    for ph in ("ms_build", "ms_factor", "ms_loglik", "ms_fisher"):
        assert st[ph] > 0.0, ph
    H.stats_reset()
    assert H.stats()["builds"] == 0
    H.close(); s.close(); m.close()


def test_forward_pass_runs_no_reverse_sweep():
    _need_gpu()
    from paper_2303_10102_amd import hmle
    key = "2d_n1024"
    o = oracle_case(key)
    w, m, s, H = gpu_case(key)
    y = torch.from_numpy(o["y"]).cuda().requires_grad_(True)
    theta = torch.tensor([w.theta_full[k] for k in H.free_idx], dtype=torch.float64, requires_grad=True)
    H.stats_reset()
    ll = hmle.HLogLik.apply(H, theta, y, w.theta_full)
    st = H.stats()
    assert (st["builds"], st["deriv_builds"], st["reverse_sweeps"], st["grad_evals"]) == (1, 0, 0, 0)
    ll.backward()
    st = H.stats()
    assert (st["builds"], st["reverse_sweeps"]) == (1, 1)
    g_adj = H.loglik_grad_adjoint(w.theta_full, y.detach())[1]
    assert np.array_equal(theta.grad.numpy(), -g_adj)
    # another evaluation between forward and backward: backward re-evaluates first
    ll2 = hmle.HLogLik.apply(H, theta.detach().clone().requires_grad_(True), y.detach(), w.theta_full)
    H.iteration(1.1 * np.asarray(w.theta_full), y.detach())
    theta3 = theta.detach().clone().requires_grad_(True)
    ll3 = hmle.HLogLik.apply(H, theta3, y.detach(), w.theta_full)
    H.iteration(1.1 * np.asarray(w.theta_full), y.detach())
    ll3.backward()
    assert np.array_equal(theta3.grad.numpy(), -g_adj)
    assert ll2.item() == ll.item()
    H.close(); s.close(); m.close()


def test_solve_many_right_hand_sides():
    _need_gpu()
    from paper_2303_10102_amd import hmle
    key = "2d_n4096"
    o = oracle_case(key)
    w, m, s, H = gpu_case(key)
    H.build(w.theta_full)
    H.factor()
    nrhs, ld = 21, w.n + 5
    rng = np.random.default_rng(4)
    Yh = np.zeros((nrhs, ld))
    Yh[:, :w.n] = rng.standard_normal((nrhs, w.n))
    Yh[0, :w.n] = o["y"]
    Y = torch.from_numpy(Yh).cuda()
    X = torch.full_like(Y, 7.0)
    st = hmle.lib().hm_solve(H._h, C.c_void_p(Y.data_ptr()), C.c_void_p(X.data_ptr()), nrhs, ld)
    assert st == 0, hmle.lib().hm_last_error()
    Xh = X.cpu().numpy()
    assert np.all(Xh[:, w.n:] == 7.0)                       # padding rows untouched
    for j in (0, 1, 15, 16, 20):
        xj = H.solve(Y[j, :w.n].contiguous()).cpu().numpy()
        assert rel_err(Xh[j, :w.n], xj) <= 1e-13, j
    zt = o["res"]["z"]
    assert rel_err(Xh[0, :w.n][o["tree"].perm], zt) < 1e-10
    assert hmle.lib().hm_solve(H._h, None, None, 0, 0) == 0   # nothing to do
    H.close(); s.close(); m.close()
