"""Shared test cases: seeded workloads, oracle results (CPU) and GPU handles.

Oracle values come only from oracle/ applied to synth/ inputs; GPU values only
from the HIP library.  The two meet only in the comparisons of the tests.
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

from synth import WORKLOADS, small_workload, sample_y, sketch_draws

CASES = {
    # the 1D workload itself (n = 1024, leaf 64, 4 levels, rank 16 + 10)
    "1d_n1024": WORKLOADS["1d_n1024"],
    # 2D 32x32, leaf 64 (4 levels, 16 leaves), rank 16 + 10, physics-dominated scale
    "2d_n1024": small_workload(N=32, leaf=64, rank=16, sigma2=1.0e3, name="2d_n1024"),
    # 2D 64x64 with the headline workload's leaf size and rank
    "2d_n4096": WORKLOADS["2d_n4096"],
    # 2D 48x48, leaf 6x6 (6 levels): leaf extents and split widths that are not powers
    # of two (the transforms' closed-form tree index and axis maps divide by 6, 12, 24)
    "2d_n2304": small_workload(N=48, leaf=36, rank=12, sigma2=1.0e3, name="2d_n2304"),
    # the 1D workload with sigma2 = 1e4 and (kappa, tau2) free: a finite, well-separated
    # maximum of L (kappa is not identifiable at sigma2 = 1), and K~ = K since the
    # off-diagonal blocks have rank 4 < the sketch rank
    "1d_mle": dataclasses.replace(WORKLOADS["1d_n1024"], sigma2=1.0e4, name="1d_mle"),
    # the 128^2 workload in a physics-dominated regime (sigma2 = 1.6e4: the field's mean
    # variance about 0.12 of the nugget's, as in the 32^2 parity case) with
    # (kappa, tau2, sigma2) free; the exact likelihood has a finite maximum there
    "2d_mle_128": dataclasses.replace(WORKLOADS["2d_n16384"], sigma2=1.6e4, free=("kappa", "tau2", "sigma2"),
                                      name="2d_mle_128"),
    # 2D 32^2 with (kappa, tau2) free: small enough for the dense exact likelihood
    "2d_mle_32": small_workload(N=32, leaf=64, rank=16, sigma2=1.0e3, free=("kappa", "tau2"), name="2d_mle_32"),
    # odd sides: 45 x 45 (n = 2025, leaf 64, 4 levels): 45 -> 22 | 23 -> 11 | 11, 11 | 12,
    # leaves of 121 to 144 points, stored padded to 144 rows
    "2d_n2025": small_workload(N=45, leaf=64, rank=16, sigma2=1.0e3, name="2d_n2025"),
    # 1D with 1000 points (leaf 64, 3 levels): equal leaves of 125 points, stored padded to
    # 128 rows (leaf rows come in groups of four)
    "1d_n1000": small_workload(dim=1, N=1000, leaf=64, rank=16, kappa=10.0, alpha=0.01, tau2=1e-4, sigma2=1.0e4,
                               free=("kappa", "alpha", "tau2", "sigma2"), name="1d_n1000"),
    # 2D 51 x 51 with leaves above 512 rows (leaf 600, 2 levels): 51 -> 25 | 26 on both axes,
    # leaves of 625 to 676 points, stored padded to 676 rows; the leaf Cholesky takes its
    # narrow-block path (16-column block columns, a ragged last one of 4)
    "2d_n2601": small_workload(N=51, leaf=600, rank=16, sigma2=1.0e3, name="2d_n2601"),
    # 1D with 1023 points (leaf 64, 3 levels): leaves of 127 and 128 points
    "1d_n1023": small_workload(dim=1, N=1023, leaf=64, rank=16, kappa=10.0, alpha=0.01, tau2=1e-4, sigma2=1.0e4,
                               free=("kappa", "alpha", "tau2", "sigma2"), name="1d_n1023"),
}


def real_rows(perm):
    """Rows of the library's tree-ordered layout that hold grid points (padding rows,
    perm = -1, are dropped); in order they are the oracle's tree rows."""
    return np.nonzero(np.asarray(perm) >= 0)[0]


@functools.lru_cache(maxsize=None)
def oracle_case(key):
    from oracle import peeling
    from oracle.exact import likelihood_gradient_fisher
    from oracle.model import Tree, dense_covariance, to_tree_order

    w = CASES[key]
    y = sample_y(w)
    K, dKs = dense_covariance(w.dim, w.N, w.theta_full, w.free)
    tree = Tree(w.dim, w.N, w.levels)
    Kt = to_tree_order(tree, K)
    dKt = [to_tree_order(tree, d) for d in dKs]
    om = sketch_draws(w)
    V = peeling.sketch_create(Kt, tree, om, w.rank)
    rep = peeling.build(Kt, dKt, tree, om, V)
    res = likelihood_gradient_fisher(rep["Kt"], rep["dKts"], to_tree_order(tree, y))
    return dict(w=w, y=y, Kt=Kt, dKt=dKt, tree=tree, om=om, V=V, rep=rep, res=res)


def densify(F, leaves, levels, kc, n, dF=None):
    """Dense matrix of a HODLR representation exported by the library.

    F, dF: (levels*kc, n) tensors/arrays (column c of the n x levels*kc panel set);
    leaves: (nleaves, nl, nl) with leaves[L] the column-major block (so block = leaves[L].T).
    Off-diagonal block of sibling pair (a, b) at depth l: F_a F_b^T, or
    dF_a F_b^T + F_a dF_b^T for a derivative matrix.
    """
    F = np.asarray(F).T
    dFm = None if dF is None else np.asarray(dF).T
    K = np.zeros((n, n))
    for l in range(1, levels + 1):
        blk = F[:, (l - 1) * kc:l * kc]
        dblk = None if dFm is None else dFm[:, (l - 1) * kc:l * kc]
        sz = n >> l
        for P in range(1 << (l - 1)):
            a = slice(2 * P * sz, (2 * P + 1) * sz)
            b = slice((2 * P + 1) * sz, (2 * P + 2) * sz)
            if dblk is None:
                m = blk[a] @ blk[b].T
            else:
                m = dblk[a] @ blk[b].T + blk[a] @ dblk[b].T
            K[a, b] = m
            K[b, a] = m.T
    lv = np.asarray(leaves)
    nl = lv.shape[1]
    for L in range(lv.shape[0]):
        K[L * nl:(L + 1) * nl, L * nl:(L + 1) * nl] = lv[L].T
    return K


def gpu_case(key):
    import torch

    from paper_2303_10102_amd import hmle

    w = CASES[key] if isinstance(key, str) else key
    m = hmle.Model(w.dim, w.N, w.leaf)
    om = torch.from_numpy(sketch_draws(w)).to("cuda")
    s = hmle.Sketch(m, om, w.rank, w.oversample, w.theta_full)
    del om
    H = hmle.HMatrix(s, w.free)
    return w, m, s, H


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def grad_err_sd(g, ref, fim_ref):
    """Per-entry gradient error in units of the score's standard deviation:
    max_j |g_j - ref_j| / sqrt(I_jj).  The entries of g span many orders of magnitude
    (the scale parameters' scores dwarf kappa's), so an error relative to the largest
    entry would not see the small ones; this unit is scale free per parameter."""
    g, ref = np.asarray(g, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    sd = np.sqrt(np.diag(np.asarray(fim_ref, dtype=np.float64)))
    return float(np.max(np.abs(g - ref) / sd))


def fim_err_corr(fim, ref):
    """Per-entry Fisher error in correlation units: max_ij |I_ij - ref_ij| / sqrt(ref_ii ref_jj)."""
    fim, ref = np.asarray(fim, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    d = np.sqrt(np.diag(ref))
    return float(np.max(np.abs(fim - ref) / np.outer(d, d)))


def dense_derivatives(w, Kt, dK_real):
    """Derivative matrices of a dense K~ for the free parameters of workload w, in its
    order: kappa, alpha from dK_real (dict name -> matrix); tau2: I; sigma2:
    (K~ - tau2 I) / sigma2 (K~ is linear in tau2 and homogeneous in sigma2)."""
    n = Kt.shape[0]
    out = []
    for name in w.free:
        if name in ("kappa", "alpha"):
            out.append(dK_real[name])
        elif name == "tau2":
            out.append(np.eye(n))
        else:
            out.append((Kt - w.tau2 * np.eye(n)) / w.sigma2)
    return out


def hmatvec(F, leaves, levels, kc, x, dF=None, dleaves=None):
    """K~ x (or K~_j x when dF, dleaves are given) from an exported representation.

    Plain NumPy on the host, in tree order; x has shape (n,) or (n, c).  Used where
    a dense matrix would not fit: the off-diagonal block of sibling pair (a, b) at
    depth l is F_a F_b^T (or dF_a F_b^T + F_a dF_b^T), the diagonal blocks are the leaves.
    """
    F = np.asarray(F).T
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    X = x.reshape(x.shape[0], -1)
    n = X.shape[0]
    Y = np.zeros_like(X)
    dFm = None if dF is None else np.asarray(dF).T
    for l in range(1, levels + 1):
        sz = n >> l
        P = 1 << (l - 1)
        blk = F[:, (l - 1) * kc:l * kc].reshape(P, 2, sz, kc)
        Xb = X.reshape(P, 2, sz, -1)
        Yb = Y.reshape(P, 2, sz, -1)
        # F_b^T x_b and F_a^T x_a for every pair
        tb = np.einsum("psk,psc->pkc", blk[:, 1], Xb[:, 1])
        ta = np.einsum("psk,psc->pkc", blk[:, 0], Xb[:, 0])
        if dFm is None:
            Yb[:, 0] += np.einsum("psk,pkc->psc", blk[:, 0], tb)
            Yb[:, 1] += np.einsum("psk,pkc->psc", blk[:, 1], ta)
        else:
            dblk = dFm[:, (l - 1) * kc:l * kc].reshape(P, 2, sz, kc)
            dtb = np.einsum("psk,psc->pkc", dblk[:, 1], Xb[:, 1])
            dta = np.einsum("psk,psc->pkc", dblk[:, 0], Xb[:, 0])
            # rows of a: (dF_a F_b^T + F_a dF_b^T) x_b ; rows of b: the transpose applied to x_a
            Yb[:, 0] += np.einsum("psk,pkc->psc", dblk[:, 0], tb) + np.einsum("psk,pkc->psc", blk[:, 0], dtb)
            Yb[:, 1] += np.einsum("psk,pkc->psc", blk[:, 1], dta) + np.einsum("psk,pkc->psc", dblk[:, 1], ta)
    lv = np.asarray(leaves if dleaves is None else dleaves)
    nb, nl = lv.shape[0], lv.shape[1]
    Xl = X.reshape(nb, nl, -1)
    # lv[L] is the column-major block, i.e. its transpose as a row-major array
    Y += np.einsum("Lji,Ljc->Lic", lv, Xl).reshape(n, -1)
    return Y[:, 0] if vec else Y


@functools.lru_cache(maxsize=None)
def oracle_mle(key, start_factor=1.3, evaluator="dense"):
    """The oracle's maximum-likelihood fit of case `key` on the exact likelihood, from
    theta_true scaled by start_factor in every free parameter; evaluator "dense"
    (assembled K, any grid) or "spectral" (closed form in the DST-I eigenbasis, 2D/1D
    Dirichlet grids of any size)."""
    from oracle.mle import exact_evaluator, fisher_scoring, spectral_evaluator

    w = CASES[key]
    y = sample_y(w)
    make = exact_evaluator if evaluator == "dense" else spectral_evaluator
    ev = make(w.dim, w.N, w.theta_full, w.free, y)
    th0 = np.asarray(w.theta, dtype=np.float64) * start_factor
    return fisher_scoring(ev, th0)
