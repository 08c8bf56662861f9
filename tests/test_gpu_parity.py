"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Tolerances (FP64, from the rounding of each step's arithmetic):
  K-apply                      1e-11 relative to max |K X|  (direct solves, O(N) rounding)
  K~, leaves and panels        TOL_KT relative to max |K~|
  K~_j                         TOL_DKT relative to max |K~_j| (Alg. 2 divides by the sketch
                               QRs' R, kept well conditioned by the common column scale of
                               each level's test matrix; observed <= 1.3e-11)
  log-likelihood               1e-9 relative
  gradient                     TOL_G_SD per entry, in units of the score's standard
                               deviation sqrt(I_jj) (entries span many orders of magnitude;
                               observed <= 1.2e-11)
  Fisher                       TOL_I_CORR per entry, in correlation units
                               |dI_ij| / sqrt(I_ii I_jj) (observed <= 5e-13)
The densified check (the library's own K~ and K~_j exported, densified on the host and
run through the oracle's dense likelihood, score and Fisher) pins the factorisation,
log-determinant, solve and exact traces apart from the construction: there both sides
evaluate the same matrices, so only rounding separates them (TOL_EXACT_*).
"""
import numpy as np
import pytest

from tests._cases import (CASES, dense_derivatives, densify, fim_err_corr, gpu_case, grad_err_sd, oracle_case,
                          real_rows, rel_err)

pytestmark = pytest.mark.gpu

TOL_KT = 1e-11
TOL_DKT = 1e-9
TOL_G_SD = 1e-9
TOL_I_CORR = 1e-10
TOL_EXACT_L = 1e-12
TOL_EXACT_G_SD = 1e-10
TOL_EXACT_I_CORR = 1e-10

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.fixture(scope="module", params=["1d_n1024", "2d_n1024", "2d_n4096", "2d_n2304", "2d_n2025", "1d_n1023",
                                        "1d_n1000", "2d_n2601"])
def case(request):
    _need_gpu()
    key = request.param
    print(f"\n[case {key}]", flush=True)
    o = oracle_case(key)
    w, m, s, H = gpu_case(key)
    yield key, o, w, m, s, H
    H.close()
    s.close()
    m.close()


def test_tree_permutation(case):
    key, o, w, m, s, H = case
    perm = m.perm()
    idx = real_rows(perm)
    assert np.array_equal(perm[idx], o["tree"].perm.astype(np.int32))
    # padded layout: leaves stored at the largest leaf's size rounded up to a multiple of
    # four, padding rows at the end of a leaf
    sizes = [sz for _, sz in o["tree"].leaves]
    assert m.leaf == (max(sizes) + 3) // 4 * 4 and m.rows == m.leaf << m.levels and len(idx) == w.n
    for L, sz in enumerate(sizes):
        blk = perm[L * m.leaf:(L + 1) * m.leaf]
        assert np.all(blk[:sz] >= 0) and np.all(blk[sz:] == -1)


@pytest.mark.parametrize("which", [0, 1, 2])
def test_kapply(case, which):
    key, o, w, m, s, H = case
    from oracle.model import dense_covariance, to_tree_order
    names = ("kappa", "alpha")
    K, dKs = dense_covariance(w.dim, w.N, w.theta_full, names)
    ref_op = to_tree_order(o["tree"], K if which == 0 else dKs[which - 1])
    rng = np.random.default_rng(11)
    X = rng.standard_normal((m.rows, 7))          # padding rows hold values too: ignored
    Xt = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    Y = m.kapply(w.theta_full, Xt, which).cpu().numpy().T
    idx = real_rows(m.perm())
    pad = np.setdiff1d(np.arange(m.rows), idx)
    assert np.all(Y[pad] == 0.0)
    ref = ref_op @ X[idx]
    assert rel_err(Y[idx], ref) < 1e-11


def test_sketch_ranks(case):
    key, o, w, m, s, H = case
    k, kc = s.ranks()
    ref = [V.shape[1] for Vs in o["V"] for V in Vs]
    assert list(k) == ref
    assert kc == max(ref)


def test_construction(case):
    key, o, w, m, s, H = case
    H.build(w.theta_full)
    _, kc = s.ranks()
    F = H.export(0).cpu().numpy()
    D = H.export(10).cpu().numpy()
    idx = real_rows(m.perm())
    Kfull = densify(F, D, m.levels, kc, m.rows)
    pad = np.setdiff1d(np.arange(m.rows), idx)
    # padding: zero panel rows, identity leaf block uncoupled from the real rows
    assert np.all(F[:, pad] == 0.0)
    assert np.array_equal(Kfull[np.ix_(pad, pad)], np.eye(len(pad))) and np.all(Kfull[np.ix_(idx, pad)] == 0.0)
    Kt = Kfull[np.ix_(idx, idx)]
    ref = o["rep"]["Kt"]
    e = rel_err(Kt, ref)
    print(f"K~ rel err {e:.3e}")
    assert e < TOL_KT
    real = [f for f in w.free if f in ("kappa", "alpha")]
    for j, name in enumerate(real):
        dF = H.export(1 + j).cpu().numpy()
        dD = H.export(11 + j).cpu().numpy()
        dfull = densify(F, dD, m.levels, kc, m.rows, dF=dF)
        assert np.all(dfull[pad] == 0.0)
        dKt = dfull[np.ix_(idx, idx)]
        refj = o["rep"]["dKts"][list(w.free).index(name)]
        ej = rel_err(dKt, refj)
        print(f"dK~/d{name} rel err {ej:.3e}")
        assert ej < TOL_DKT


def test_likelihood_gradient_fisher(case):
    key, o, w, m, s, H = case
    y = torch.from_numpy(o["y"]).cuda()
    ll, g, fim = H.iteration(w.theta_full, y)
    r = o["res"]
    print(f"loglik {ll!r} vs {r['loglik']!r}")
    print("grad", g, r["grad_nll"])
    print("fim", fim, r["fim"], sep="\n")
    eg, ei = grad_err_sd(g, r["grad_nll"], r["fim"]), fim_err_corr(fim, r["fim"])
    asym = fim_err_corr(fim, fim.T)
    print(f"[{key}] per entry: gradient {eg:.2e} sd, Fisher {ei:.2e} corr, asymmetry {asym:.2e}")
    assert abs(ll - r["loglik"]) <= 1e-9 * abs(r["loglik"])
    assert eg < TOL_G_SD
    assert ei < TOL_I_CORR
    # (i, j) and (j, i) are computed independently: symmetric to rounding
    assert asym < TOL_I_CORR


def test_densified_representation(case):
    """The library's L~, score and Fisher equal the dense definitions evaluated on its
    own exported K~ and K~_j (factorisation, log-determinant, solve and the exact traces
    of App. B are exact for a given HODLR matrix)."""
    key, o, w, m, s, H = case
    from oracle.exact import likelihood_gradient_fisher
    y = torch.from_numpy(o["y"]).cuda()
    ll, g, fim = H.iteration(w.theta_full, y)
    _, kc = s.ranks()
    F = H.export(0).cpu().numpy()
    ix = np.ix_(real_rows(m.perm()), real_rows(m.perm()))
    Kd = densify(F, H.export(10).cpu().numpy(), m.levels, kc, m.rows)[ix]
    real = [f for f in w.free if f in ("kappa", "alpha")]
    dK = {name: densify(F, H.export(11 + j).cpu().numpy(), m.levels, kc, m.rows,
                        dF=H.export(1 + j).cpu().numpy())[ix]
          for j, name in enumerate(real)}
    r = likelihood_gradient_fisher(Kd, dense_derivatives(w, Kd, dK), o["y"][o["tree"].perm])
    eg, ei = grad_err_sd(g, r["grad_nll"], r["fim"]), fim_err_corr(fim, r["fim"])
    el = abs(ll - r["loglik"]) / abs(r["loglik"])
    print(f"[{key}] densified: loglik {el:.2e} rel, gradient {eg:.2e} sd, Fisher {ei:.2e} corr")
    assert el < TOL_EXACT_L
    assert eg < TOL_EXACT_G_SD
    assert ei < TOL_EXACT_I_CORR


def test_logdet_and_solve(case):
    key, o, w, m, s, H = case
    H.build(w.theta_full)
    H.factor()
    ld = H.logdet()
    assert abs(ld - o["res"]["logdet"]) <= 1e-9 * abs(o["res"]["logdet"]) + 1e-9
    y = torch.from_numpy(o["y"]).cuda()
    x = H.solve(y).cpu().numpy()
    zt = o["res"]["z"]           # tree order
    xt = x[o["tree"].perm]
    assert rel_err(xt, zt) < 1e-8
