"""Pins of the oracle's peeling replay (Sec. 3.2-3.3) on the CPU.

Fixed independently of the replay code by:
  * exactness when every off-diagonal block has rank <= k: the 1D stencil
    covariance has off-diagonal rank <= 4 (banded inverse factors), and on
    tiny 2D grids a rank at least the block size makes every block exact;
  * Alg. 2 against finite differences of numpy's QR (sign-fixed);
  * the construction's forward-mode derivative against central finite
    differences of the whole construction with the sketch held fixed;
  * the exact parameter structure: dK~/dtau2 = I and
    dK~/dsigma2 = (K~ - tau2 I)/sigma2 (homogeneity of the construction),
    and the Euler identities they imply for the likelihood quantities;
  * the level-1 block equals the randomized range finder's Q Q^T B (Alg. 1).
"""
import numpy as np
import pytest

from oracle import peeling
from oracle.exact import likelihood_gradient_fisher
from oracle.model import Tree, dense_covariance, to_tree_order
from synth import WORKLOADS, sample_y, sketch_draws, small_workload


def _setup(w, free=None):
    free = w.free if free is None else free
    K, dKs = dense_covariance(w.dim, w.N, w.theta_full, free)
    tree = Tree(w.dim, w.N, w.levels)
    Kt = to_tree_order(tree, K)
    dKt = [to_tree_order(tree, d) for d in dKs]
    om = sketch_draws(w)
    return Kt, dKt, tree, om


def test_1d_workload_is_exact():
    w = WORKLOADS["1d_n1024"]
    Kt, dKt, tree, om = _setup(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    assert all(v.shape[1] == 4 for vs in V for v in vs)   # numerical rank of every block
    r = peeling.build(Kt, dKt, tree, om, V)
    assert np.max(np.abs(r["Kt"] - Kt)) <= 1e-13 * np.max(np.abs(Kt))
    for j in range(len(dKt)):
        assert np.max(np.abs(r["dKts"][j] - dKt[j])) <= 1e-9 * np.max(np.abs(dKt[j]))
    y = to_tree_order(tree, sample_y(w))
    a = likelihood_gradient_fisher(r["Kt"], r["dKts"], y)
    b = likelihood_gradient_fisher(Kt, dKt, y)
    assert abs(a["loglik"] - b["loglik"]) <= 1e-12 * abs(b["loglik"])
    assert np.max(np.abs(a["grad_nll"] - b["grad_nll"]) / np.abs(b["grad_nll"])) <= 1e-8
    assert np.max(np.abs(a["fim"] - b["fim"])) <= 1e-8 * np.max(np.abs(b["fim"]))


def test_2d_full_rank_is_exact():
    # n = 64, leaf 8, 3 levels; level-1 blocks are 32 x 32 and rank 32 keeps them whole
    w = small_workload(N=8, leaf=8, rank=32, oversample=4, sigma2=300.0)
    Kt, dKt, tree, om = _setup(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    r = peeling.build(Kt, dKt, tree, om, V)
    assert np.max(np.abs(r["Kt"] - Kt)) <= 1e-11 * np.max(np.abs(Kt))
    for j in range(len(dKt)):
        assert np.max(np.abs(r["dKts"][j] - dKt[j])) <= 1e-7 * np.max(np.abs(dKt[j]))


def test_2d_full_rank_is_exact_on_an_odd_grid():
    # n = 81 (9 x 9), leaf 8, 3 levels: 9 -> 4 | 5 along x, then y: leaves of 8 to 15 points
    # (the left child takes floor(side / 2)); rank 45 keeps every off-diagonal block whole
    w = small_workload(N=9, leaf=8, rank=45, oversample=4, sigma2=300.0)
    Kt, dKt, tree, om = _setup(w)
    sizes = sorted({sz for _, sz in tree.leaves})
    assert len(sizes) > 1 and sum(sz for _, sz in tree.leaves) == 81
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    r = peeling.build(Kt, dKt, tree, om, V)
    assert np.max(np.abs(r["Kt"] - Kt)) <= 1e-11 * np.max(np.abs(Kt))
    for j in range(len(dKt)):
        assert np.max(np.abs(r["dKts"][j] - dKt[j])) <= 1e-7 * np.max(np.abs(dKt[j]))


def test_qr_tangent_matches_finite_differences():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((30, 6))
    dB = rng.standard_normal((30, 6))
    Q, R = peeling.qr_positive(B)
    dQ = peeling.qr_tangent(Q, R, dB)
    h = 1e-6
    Qp, _ = peeling.qr_positive(B + h * dB)
    Qm, _ = peeling.qr_positive(B - h * dB)
    fd = (Qp - Qm) / (2 * h)
    assert np.max(np.abs(fd - dQ)) <= 1e-7
    # Q^T dQ is skew (orthonormality is preserved to first order)
    S = Q.T @ dQ
    assert np.max(np.abs(S + S.T)) <= 1e-12


def test_qr_positive_gauge():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((12, 5))
    Q, R = peeling.qr_positive(Y)
    assert np.all(np.diag(R) > 0)
    assert np.allclose(Q @ R, Y) and np.allclose(Q.T @ Q, np.eye(5))


def test_compress_rank_and_sign():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 9))
    V = peeling.compress(A, rank=6)
    assert V.shape == (9, 3)
    for j in range(3):
        i = np.argmax(np.abs(V[:, j]))
        assert V[i, j] > 0
    # the kept directions span the row space
    assert np.linalg.norm(A - A @ V @ V.T) <= 1e-12 * np.linalg.norm(A)
    assert peeling.compress(A, rank=2).shape == (9, 2)


def test_construction_derivative_matches_finite_differences():
    w = small_workload(N=16, leaf=16, rank=8, oversample=4, sigma2=500.0)
    Kt, dKt, tree, om = _setup(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    r = peeling.build(Kt, dKt, tree, om, V)
    theta = w.theta_full
    for j, name in enumerate(w.free):
        k = ("kappa", "alpha", "tau2", "sigma2").index(name)
        h = 1e-6 * theta[k]
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        Kp = to_tree_order(tree, dense_covariance(w.dim, w.N, tp, ())[0])
        Km = to_tree_order(tree, dense_covariance(w.dim, w.N, tm, ())[0])
        fd = (peeling.build(Kp, [], tree, om, V)["Kt"] - peeling.build(Km, [], tree, om, V)["Kt"]) / (2 * h)
        err = np.max(np.abs(fd - r["dKts"][j])) / np.max(np.abs(r["dKts"][j]))
        assert err <= 1e-5, (name, err)


def test_scale_parameter_structure():
    w = small_workload(N=16, leaf=16, rank=8, oversample=4, sigma2=500.0)
    Kt, dKt, tree, om = _setup(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    r = peeling.build(Kt, dKt, tree, om, V)
    n = w.n
    j_tau, j_sig = w.free.index("tau2"), w.free.index("sigma2")
    assert np.max(np.abs(r["dKts"][j_tau] - np.eye(n))) <= 1e-13
    ref = (r["Kt"] - w.tau2 * np.eye(n)) / w.sigma2
    assert np.max(np.abs(r["dKts"][j_sig] - ref)) <= 1e-12 * np.max(np.abs(ref))
    # Euler identities of the homogeneous scale pair (sigma2, tau2)
    y = to_tree_order(tree, sample_y(w))
    q = likelihood_gradient_fisher(r["Kt"], r["dKts"], y)
    ts = np.array([w.sigma2 if f == "sigma2" else w.tau2 if f == "tau2" else 0.0 for f in w.free])
    yz = float(y @ q["z"])
    assert abs(ts @ q["grad_nll"] - (n / 2 - yz / 2)) <= 1e-10 * n
    assert abs(ts @ q["fim"] @ ts - n / 2) <= 1e-10 * n
    kj = w.free.index("kappa")
    trace_k = 2 * q["grad_nll"][kj] + float(q["z"] @ (r["dKts"][kj] @ q["z"]))
    assert abs((q["fim"] @ ts)[kj] - 0.5 * trace_k) <= 1e-9 * abs(trace_k)


def test_level1_block_is_range_finder_projection():
    w = small_workload(N=16, leaf=32, rank=10, oversample=0, sigma2=500.0)
    Kt, dKt, tree, om = _setup(w, free=())
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    r = peeling.build(Kt, [], tree, om, V)
    a, b = tree.rows(1, 0), tree.rows(1, 1)
    Q = r["Q"][0][0]
    B = Kt[a, b]
    # Alg. 1: B^ = Q (Q^T B) with Q an orthonormal basis of B Omega'
    assert np.allclose(r["Kt"][a, b], Q @ (Q.T @ B), atol=1e-14 * np.abs(B).max())
    Om = om[0][:, b].T @ V[0][0]
    Qref, _ = peeling.qr_positive(B @ Om)
    assert np.allclose(np.abs(Q.T @ Qref), np.eye(Q.shape[1]), atol=1e-10)


def test_compress_tolerance_keeps_the_leading_directions():
    # a sample with prescribed singular values: Y = U diag(s) W^T (orthonormal U, W);
    # the tolerance keeps the directions with s_i > tol s_1 (capped at the rank), and
    # they span the leading right singular vectors W[:, :k]
    rng = np.random.default_rng(5)
    s = np.array([1.0, 0.5, 0.2, 0.05, 0.012, 0.008, 1e-3, 1e-5])
    U, _ = np.linalg.qr(rng.standard_normal((40, s.size)))
    W, _ = np.linalg.qr(rng.standard_normal((s.size, s.size)))
    Y = U @ np.diag(s) @ W.T
    for tol, rank, k in ((1e-2, 8, 5), (1e-2, 3, 3), (1e-4, 8, 7), (0.0, 8, 8), (0.3, 8, 2)):
        V = peeling.compress(Y, rank, tol)
        assert V.shape == (s.size, k)
        # same subspace: the projector onto span(V) equals the one onto W[:, :k]
        P1, P2 = V @ V.T, W[:, :k] @ W[:, :k].T
        assert np.max(np.abs(P1 - P2)) < 1e-12


def test_level_scale_whitens_alike_blocks():
    # hand case: geometric mean over the blocks that keep each column
    d = peeling.level_scale([np.array([1.0, 0.1, 0.05]), np.array([2.0, 0.02, 1e-3])], [2, 3])
    assert np.allclose(d, [1.0, np.sqrt(10.0 * 100.0), 2000.0], rtol=1e-14)
    # blocks with one spectrum: Y V d = s_1 U (orthogonal columns of equal norm s_1),
    # so the sample's R is s_1 I; rounding of Y (u |Y|) grows by s_1 / s_5 = 3e6
    rng = np.random.default_rng(8)
    s = np.array([3.0, 1.0, 1e-2, 1e-4, 1e-6])
    Ys = []
    for _ in range(2):
        U, _ = np.linalg.qr(rng.standard_normal((30, s.size)))
        W, _ = np.linalg.qr(rng.standard_normal((7, s.size)))
        Ys.append(U @ np.diag(s) @ W.T)
    Vs = [peeling.compress(Y, rank=5) for Y in Ys]
    d = peeling.level_scale([peeling.sample_spectrum(Y) for Y in Ys], [5, 5])
    assert np.allclose(d, s[0] / s, rtol=1e-6)
    for Y, V in zip(Ys, Vs):
        G = (Y @ V * d).T @ (Y @ V * d)
        assert np.max(np.abs(G - s[0] ** 2 * np.eye(5))) <= 1e-8 * s[0] ** 2
        _, R = peeling.qr_positive(Y @ V * d)
        assert np.linalg.cond(R) < 1 + 1e-6


def test_scaled_compression_leaves_the_construction_unchanged():
    # a positive column scale common to the blocks of a level gives the same sample up
    # to that scale in every block, hence the same Q (diag R > 0): K~ and K~_j are the
    # same matrices (up to the rounding of the unscaled, worse-conditioned R)
    w = small_workload(N=16, leaf=16, rank=8, oversample=4, sigma2=500.0)
    Kt, dKt, tree, om = _setup(w)
    V1 = peeling.sketch_create(Kt, tree, om, w.rank, scaled=True)
    V0 = peeling.sketch_create(Kt, tree, om, w.rank, scaled=False)
    r1 = peeling.build(Kt, dKt, tree, om, V1)
    r0 = peeling.build(Kt, dKt, tree, om, V0)
    assert np.max(np.abs(r1["Kt"] - r0["Kt"])) <= 1e-12 * np.max(np.abs(r0["Kt"]))
    for j in range(len(w.free)):
        assert np.max(np.abs(r1["dKts"][j] - r0["dKts"][j])) <= 1e-7 * np.max(np.abs(r0["dKts"][j]))
