"""GPU: ranks chosen per block by a truncation tolerance (hm_sketch_create_tol).

On the 32^2 parity case with rank_tol = 1e-2 the kept ranks vary per block (7..16; the
closest singular-value ratio lies 3% from the threshold, so rounding cannot flip a
decision).  The library's ranks equal the oracle's block by block, and K~, K~_j and
the likelihood terms match the oracle's replay with those ranks to the parity
tolerances."""
import numpy as np
import pytest

from tests._cases import CASES, densify, fim_err_corr, grad_err_sd, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-2


def test_adaptive_ranks_match_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from oracle import peeling
    from oracle.exact import likelihood_gradient_fisher
    from oracle.model import Tree, dense_covariance, to_tree_order
    from paper_2303_10102_amd import hmle
    from synth import sample_y, sketch_draws

    w = CASES["2d_n1024"]
    print(f"\n[rank_tol {TOL} {w.name}]", flush=True)
    K, dKs = dense_covariance(w.dim, w.N, w.theta_full, w.free)
    tree = Tree(w.dim, w.N, w.levels)
    Kt = to_tree_order(tree, K)
    dKt = [to_tree_order(tree, d) for d in dKs]
    om = sketch_draws(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank, TOL)
    rep = peeling.build(Kt, dKt, tree, om, V)
    y = sample_y(w)
    res = likelihood_gradient_fisher(rep["Kt"], rep["dKts"], to_tree_order(tree, y))
    ranks_o = [Vb.shape[1] for Vs in V for Vb in Vs]
    assert min(ranks_o) < w.rank   # the tolerance is active

    m = hmle.Model(w.dim, w.N, w.leaf)
    s = hmle.Sketch(m, torch.from_numpy(om).cuda(), w.rank, w.oversample, w.theta_full, rank_tol=TOL)
    H = hmle.HMatrix(s, w.free)
    k, kc = s.ranks()
    print("ranks", list(k), "oracle", ranks_o, flush=True)
    assert list(k) == ranks_o and kc == max(ranks_o)
    H.build(w.theta_full)
    Kt_g = densify(H.export(0).cpu().numpy(), H.export(10).cpu().numpy(), m.levels, kc, w.n)
    assert rel_err(Kt_g, rep["Kt"]) < 1e-11
    for j, name in enumerate([f for f in w.free if f in ("kappa", "alpha")]):
        dKt_g = densify(H.export(0).cpu().numpy(), H.export(11 + j).cpu().numpy(), m.levels, kc, w.n,
                        dF=H.export(1 + j).cpu().numpy())
        assert rel_err(dKt_g, rep["dKts"][list(w.free).index(name)]) < 1e-9
    ll, g, fim = H.iteration(w.theta_full, torch.from_numpy(y).cuda())
    H.close(); s.close(); m.close()
    eg, ei = grad_err_sd(g, res["grad_nll"], res["fim"]), fim_err_corr(fim, res["fim"])
    print(f"gradient {eg:.2e} sd, Fisher {ei:.2e} corr")
    assert abs(ll - res["loglik"]) <= 1e-9 * abs(res["loglik"])
    assert eg < 1e-9
    assert ei < 1e-10
