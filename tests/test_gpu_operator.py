"""GPU: the general operator interface (hm_model_create_op).

A caller-supplied covariance operator on scattered points -- here an anisotropic
Matern-3/2 kernel applied as a dense product by the caller's own torch code on the
model's stream -- replaces the built-in stencil K-apply; the tree is the KD-tree of the
points.  The oracle evaluates the same kernel densely (oracle/operators.py), builds
its own point KD-tree (oracle/model.py PointTree) and replays the construction
(oracle/peeling.py) with the same sketch draws.  Checked: the tree permutation
exactly, the K-apply and its two parameter derivatives (1e-12 relative), K~ and K~_j,
L~, the score per entry (standard deviations) and the Fisher matrix per entry
(correlation units) against the oracle, the densified representation (pin P4), and
the reverse-mode gradient against the forward mode (bounds: 1e-9 sd for scores, 1e-10
correlation units for Fisher entries, 1e-9 relative between the two gradients).
"""
import functools

import numpy as np
import pytest

from tests._cases import dense_derivatives, densify, fim_err_corr, grad_err_sd, real_rows, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _matern_op(coords):
    """The caller's operator: dense anisotropic Matern-3/2 products in torch."""
    xy = torch.from_numpy(np.asarray(coords, dtype=np.float64)).cuda()
    if xy.dim() == 1:
        xy = xy[:, None]
    cache = {}

    def kernel(theta):
        key = (theta[0], theta[1])
        if key not in cache:
            ell, a = theta[0], theta[1]
            dx = xy[:, None, 0] - xy[None, :, 0]
            dy = (xy[:, None, 1] - xy[None, :, 1]) if xy.shape[1] == 2 else torch.zeros_like(dx)
            r = (3.0 ** 0.5) * torch.sqrt(dx * dx + (a * dy) ** 2) / ell
            e = torch.exp(-r)
            cache.clear()
            cache[key] = ((1.0 + r) * e, r * r * e / ell, -3.0 * a * dy * dy * e / (ell * ell))
        return cache[key]

    def op(which, theta, X, Y):
        Y.copy_(X @ kernel(theta)[which])     # X, Y: (c, n); every kernel matrix is symmetric

    return op


@functools.lru_cache(maxsize=None)
def _oracle(key):
    from oracle import peeling
    from oracle.exact import likelihood_gradient_fisher
    from oracle.model import PointTree, to_tree_order
    from oracle.operators import matern32
    from synth import OP_WORKLOADS, sketch_draws
    w = OP_WORKLOADS[key]
    xy = w.coords()
    Kop, d0, d1 = matern32(xy, w.theta0, w.theta1)
    K = w.sigma2 * Kop + w.tau2 * np.eye(w.n)
    dK = {"kappa": w.sigma2 * d0, "alpha": w.sigma2 * d1, "tau2": np.eye(w.n), "sigma2": Kop}
    tree = PointTree(xy, w.levels)
    Kt = to_tree_order(tree, K)
    dKt = [to_tree_order(tree, dK[f]) for f in w.free]
    om = sketch_draws(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    rep = peeling.build(Kt, dKt, tree, om, V)
    y = w.sample()
    res = likelihood_gradient_fisher(rep["Kt"], rep["dKts"], to_tree_order(tree, y))
    return dict(w=w, xy=xy, tree=tree, K=K, dK=dK, V=V, rep=rep, y=y, res=res)


@pytest.fixture(scope="module", params=["op2d_n1500", "op1d_n1000"])
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2303_10102_amd import hmle
    from synth import sketch_draws
    key = request.param
    print(f"\n[operator {key}]", flush=True)
    o = _oracle(key)
    w = o["w"]
    m = hmle.OpModel(o["xy"], w.leaf, _matern_op(o["xy"]))
    s = hmle.Sketch(m, torch.from_numpy(sketch_draws(w)).cuda(), w.rank, w.oversample, w.theta_full)
    H = hmle.HMatrix(s, w.free)
    yield key, o, w, m, s, H
    H.close(); s.close(); m.close()


def test_point_tree(case):
    key, o, w, m, s, H = case
    perm = m.perm()
    assert np.array_equal(perm[real_rows(perm)], o["tree"].perm.astype(np.int32))
    assert m.leaf == (max(sz for _, sz in o["tree"].leaves) + 3) // 4 * 4


@pytest.mark.parametrize("which", [0, 1, 2])
def test_kapply(case, which):
    key, o, w, m, s, H = case
    rng = np.random.default_rng(5)
    X = rng.standard_normal((m.rows, 6))
    Y = m.kapply(w.theta_full, torch.from_numpy(np.ascontiguousarray(X.T)).cuda(), which).cpu().numpy().T
    idx = real_rows(m.perm())
    from oracle.model import to_tree_order
    op = o["K"] if which == 0 else o["dK"][("kappa", "alpha")[which - 1]]
    ref = to_tree_order(o["tree"], op) @ X[idx]
    assert rel_err(Y[idx], ref) < 1e-12
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
        dK[name] = densify(F, H.export(11 + j).cpu().numpy(), m.levels, kc, m.rows, dF=H.export(1 + j).cpu().numpy())[ix]
        ej = rel_err(dK[name], o["rep"]["dKts"][list(w.free).index(name)])
        print(f"dK~/d{name} rel err {ej:.2e}")
        assert ej < 1e-9
    r = o["res"]
    eg, ei = grad_err_sd(g, r["grad_nll"], r["fim"]), fim_err_corr(fim, r["fim"])
    print(f"K~ {ek:.2e}; loglik {ll!r} vs {r['loglik']!r}; gradient {eg:.2e} sd, Fisher {ei:.2e} corr")
    assert ek < 1e-11
    assert abs(ll - r["loglik"]) <= 1e-9 * abs(r["loglik"])
    assert eg < 1e-9 and ei < 1e-10
    # densified representation: the H operations are exact for the library's own K~
    rd = likelihood_gradient_fisher(Kd, dense_derivatives(w, Kd, dK), o["y"][o["tree"].perm])
    egd, eid = grad_err_sd(g, rd["grad_nll"], rd["fim"]), fim_err_corr(fim, rd["fim"])
    print(f"densified: loglik {abs(ll - rd['loglik']) / abs(rd['loglik']):.2e} rel, gradient {egd:.2e} sd, "
          f"Fisher {eid:.2e} corr")
    # (1D: close points make K~ ill conditioned, cond ~ 1e7; the scores carry its rounding)
    assert abs(ll - rd["loglik"]) <= 1e-12 * abs(rd["loglik"])
    assert egd < 1e-9 and eid < 1e-10


def test_adjoint_gradient(case):
    key, o, w, m, s, H = case
    yd = torch.from_numpy(o["y"]).cuda()
    ll_f, g_f, fim = H.iteration(w.theta_full, yd)
    ll_a, g_a = H.loglik_grad_adjoint(w.theta_full, yd)
    rel = np.max(np.abs(g_a - g_f) / np.abs(g_f))
    print(f"adjoint {g_a} forward {g_f}: {rel:.2e} relative, {grad_err_sd(g_a, g_f, fim):.2e} sd")
    assert ll_a == ll_f or abs(ll_a - ll_f) <= 1e-13 * abs(ll_f)
    assert rel < 1e-9 and grad_err_sd(g_a, g_f, fim) < 1e-9
