"""GPU: observed subsets of the stencil field (hm_model_create_spde with obs_idx).

The observation operator is a selection of grid nodes (Sec. 5.1, eq. "projection"):
K_obs = sigma2 Phi M M^T Phi^T + tau2 I with the physics on the full grid.  Cases:
  * sel_n4096: the 256^2 headline field (rank 48, leaf 256, theta = (kappa, alpha, tau2,
    sigma2)) observed on its regular 64 x 64 subgrid of nodes 4 s + 1 -- the dense
    oracle check of the 256^2 workload at a 64 x 64 subgrid;
  * sel_n1500: 1500 random nodes of a 48 x 48 grid (irregular, partial observations);
  * sel1d_n700: 700 random points of a 1000-point line.
The oracle assembles K_obs and its derivatives from sine-transform mode sums
(oracle/selection.py, pinned to the sparse-solve assembly), builds its own KD-tree of
the observed nodes (oracle/model.py PointTree) and replays the construction with the
same sketch draws.  Checked: the tree exactly; K-apply and both derivatives (1e-12
relative); K~, K~_j; L~, score per entry (sd) and Fisher per entry (correlation units);
the densified representation; the reverse-mode gradient against the forward mode.
"""
import functools

import numpy as np
import pytest

from tests._cases import dense_derivatives, densify, fim_err_corr, grad_err_sd, real_rows, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@functools.lru_cache(maxsize=None)
def _oracle(key):
    from oracle import peeling
    from oracle.exact import likelihood_gradient_fisher
    from oracle.model import PointTree, to_tree_order
    from oracle.selection import grid_coords, selected_covariance
    from synth import SEL_WORKLOADS, sketch_draws
    w = SEL_WORKLOADS[key]
    obs = w.obs()
    K, dKl = selected_covariance(w.dim, w.N, w.theta_full, obs)
    dK = dict(zip(("kappa", "alpha", "tau2", "sigma2"), dKl))
    xy = grid_coords(w.dim, w.N, obs)
    tree = PointTree(xy, w.levels)
    Kt = to_tree_order(tree, K)
    dKt = [to_tree_order(tree, dK[f]) for f in w.free]
    om = sketch_draws(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    rep = peeling.build(Kt, dKt, tree, om, V)
    y = w.sample()
    res = likelihood_gradient_fisher(rep["Kt"], rep["dKts"], to_tree_order(tree, y))
    return dict(w=w, obs=obs, tree=tree, K=K, dK=dK, rep=rep, y=y, res=res)


@pytest.fixture(scope="module", params=["sel_n1500", "sel1d_n700", "sel_n4096"])
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2303_10102_amd import hmle
    from synth import sketch_draws
    key = request.param
    print(f"\n[selection {key}]", flush=True)
    o = _oracle(key)
    w = o["w"]
    m = hmle.Model(w.dim, w.N, w.leaf, obs=o["obs"])
    s = hmle.Sketch(m, torch.from_numpy(sketch_draws(w)).cuda(), w.rank, w.oversample, w.theta_full)
    H = hmle.HMatrix(s, w.free)
    yield key, o, w, m, s, H
    H.close(); s.close(); m.close()


def test_observation_tree(case):
    key, o, w, m, s, H = case
    perm = m.perm()
    assert m.n == o["obs"].size
    assert np.array_equal(perm[real_rows(perm)], o["tree"].perm.astype(np.int32))
    assert m.leaf == (max(sz for _, sz in o["tree"].leaves) + 3) // 4 * 4


@pytest.mark.parametrize("which", [0, 1, 2])
def test_kapply(case, which):
    key, o, w, m, s, H = case
    from oracle.model import to_tree_order
    rng = np.random.default_rng(5)
    X = rng.standard_normal((m.rows, 6))
    Y = m.kapply(w.theta_full, torch.from_numpy(np.ascontiguousarray(X.T)).cuda(), which).cpu().numpy().T
    idx = real_rows(m.perm())
    op = o["K"] if which == 0 else o["dK"][("kappa", "alpha")[which - 1]]
    ref = to_tree_order(o["tree"], op) @ X[idx]
    e = rel_err(Y[idx], ref)
    print(f"K-apply {which}: {e:.2e}")
    assert e < 1e-12
    assert np.all(np.delete(Y, idx, axis=0) == 0.0)


def test_construction_and_likelihood(case):
    key, o, w, m, s, H = case
    from oracle.exact import likelihood_gradient_fisher
    yd = torch.from_numpy(o["y"]).cuda()
    ll, g, fim = H.iteration(w.theta_full, yd)
    _, kc = s.ranks()
    idx = real_rows(m.perm())
    ix = np.ix_(idx, idx)
    F = H.export(0).cpu().numpy()
    Kd = densify(F, H.export(10).cpu().numpy(), m.levels, kc, m.rows)[ix]
    ek = rel_err(Kd, o["rep"]["Kt"])
    real = [f for f in w.free if f in ("kappa", "alpha")]
    dK = {}
    for j, name in enumerate(real):
        dK[name] = densify(F, H.export(11 + j).cpu().numpy(), m.levels, kc, m.rows,
                           dF=H.export(1 + j).cpu().numpy())[ix]
        ej = rel_err(dK[name], o["rep"]["dKts"][list(w.free).index(name)])
        print(f"dK~/d{name} rel err {ej:.2e}")
        assert ej < 1e-9
    r = o["res"]
    eg, ei = grad_err_sd(g, r["grad_nll"], r["fim"]), fim_err_corr(fim, r["fim"])
    print(f"K~ {ek:.2e}; loglik {ll!r} vs {r['loglik']!r}; gradient {eg:.2e} sd, Fisher {ei:.2e} corr")
    assert ek < 1e-11
    assert abs(ll - r["loglik"]) <= 1e-9 * abs(r["loglik"])
    assert eg < 1e-9 and ei < 1e-10
    rd = likelihood_gradient_fisher(Kd, dense_derivatives(w, Kd, dK), o["y"][o["tree"].perm])
    egd, eid = grad_err_sd(g, rd["grad_nll"], rd["fim"]), fim_err_corr(fim, rd["fim"])
    print(f"densified: loglik {abs(ll - rd['loglik']) / abs(rd['loglik']):.2e} rel, gradient {egd:.2e} sd, "
          f"Fisher {eid:.2e} corr")
    assert abs(ll - rd["loglik"]) <= 1e-12 * abs(rd["loglik"])
    assert egd < 1e-9 and eid < 1e-10


def test_adjoint_gradient(case):
    key, o, w, m, s, H = case
    yd = torch.from_numpy(o["y"]).cuda()
    ll_f, g_f, fim = H.iteration(w.theta_full, yd)
    ll_a, g_a = H.loglik_grad_adjoint(w.theta_full, yd)
    rel = np.max(np.abs(g_a - g_f) / np.abs(g_f))
    esd = grad_err_sd(g_a, g_f, fim)
    print(f"adjoint {g_a} forward {g_f}: {rel:.2e} relative, {esd:.2e} sd")
    assert ll_a == ll_f or abs(ll_a - ll_f) <= 1e-13 * abs(ll_f)
    assert esd < 1e-9
