"""GPU: the bivariate co-kriging model (hm_model_create_spde with nvars = 2).

Two variables per grid node driven by one latent noise, y1 = B^-1 w + nugget 1,
y2 = A^-1 B^-1 w + nugget 2, theta_full = (kappa, alpha, tau2_1, sigma2, tau2_2), a
5 x 5 Fisher matrix.  The oracle assembles K and its five derivatives from sparse
solves (oracle/bivariate.py, pinned by the per-mode 2 x 2 closed form), orders the rows
by its own KD-tree of the nodes with each node's two rows together (PairTree), and
replays the construction with the same sketch draws.  Checked: the tree exactly; the
K-apply and its two derivatives (1e-12 relative); K~, K~_j; L~, the score per entry
(sd) and the Fisher matrix per entry (correlation units); the densified
representation (pin P4, with the two nugget derivatives diagonal masks); the
reverse-mode gradient (the two nuggets' sums split by variable) against the forward mode.
"""
import functools

import numpy as np
import pytest

from tests._cases import densify, fim_err_corr, grad_err_sd, real_rows, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@functools.lru_cache(maxsize=None)
def _oracle(key):
    from oracle import peeling
    from oracle.bivariate import PairTree, bivariate_covariance, grid_locations
    from oracle.exact import likelihood_gradient_fisher
    from oracle.model import PointTree, to_tree_order
    from synth import BIV_WORKLOADS, sketch_draws
    w = BIV_WORKLOADS[key]
    K, dKl = bivariate_covariance(w.dim, w.N, w.theta_full)
    dK = dict(zip(("kappa", "alpha", "tau2", "sigma2", "tau2_2"), dKl))
    tree = PairTree(PointTree(grid_locations(w.dim, w.N), w.levels), w.n_loc)
    Kt = to_tree_order(tree, K)
    dKt = [to_tree_order(tree, dK[f]) for f in w.free]
    om = sketch_draws(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    rep = peeling.build(Kt, dKt, tree, om, V)
    y = w.sample()
    res = likelihood_gradient_fisher(rep["Kt"], rep["dKts"], to_tree_order(tree, y))
    return dict(w=w, tree=tree, K=K, dK=dK, rep=rep, y=y, res=res)


def _dense_derivatives(w, tree, Kt, dK_real):
    """Derivative matrices of a dense bivariate K~ (tree order) for w's free parameters:
    kappa, alpha given; tau2_v: the diagonal mask of variable v's rows; sigma2:
    (K~ - T) / sigma2 with T the nugget diagonal."""
    first = (np.asarray(tree.perm) < w.n_loc).astype(np.float64)
    T = np.diag(w.tau2 * first + w.tau2_2 * (1.0 - first))
    out = []
    for name in w.free:
        if name in ("kappa", "alpha"):
            out.append(dK_real[name])
        elif name == "tau2":
            out.append(np.diag(first))
        elif name == "tau2_2":
            out.append(np.diag(1.0 - first))
        else:
            out.append((Kt - T) / w.sigma2)
    return out


@pytest.fixture(scope="module", params=["biv_n1152", "biv_n882", "biv1d_n1000"])
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2303_10102_amd import hmle
    from synth import sketch_draws
    key = request.param
    print(f"\n[bivariate {key}]", flush=True)
    o = _oracle(key)
    w = o["w"]
    m = hmle.Model(w.dim, w.N, w.leaf, nvars=2)
    s = hmle.Sketch(m, torch.from_numpy(sketch_draws(w)).cuda(), w.rank, w.oversample, w.theta_full)
    H = hmle.HMatrix(s, w.free)
    yield key, o, w, m, s, H
    H.close(); s.close(); m.close()


def test_pair_tree(case):
    key, o, w, m, s, H = case
    perm = m.perm()
    assert m.n == w.n
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
    assert fim.shape == (len(w.free), len(w.free))
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
    print(f"grad {g}\noracle {r['grad_nll']}")
    assert ek < 1e-11
    assert abs(ll - r["loglik"]) <= 1e-9 * abs(r["loglik"])
    assert eg < 1e-9 and ei < 1e-10
    rd = likelihood_gradient_fisher(Kd, _dense_derivatives(w, o["tree"], Kd, dK), o["y"][o["tree"].perm])
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
    esd = grad_err_sd(g_a, g_f, fim)
    print(f"adjoint {g_a} forward {g_f}: {esd:.2e} sd")
    assert ll_a == ll_f or abs(ll_a - ll_f) <= 1e-13 * abs(ll_f)
    assert esd < 1e-9
