"""Dense replay of the matrix-free HODLR construction and of its derivative.

Sec. 3.2 ("Construction from matrix-vector products"): level by level, a patterned
Gaussian block supported on the right children is multiplied by K minus all
coarser off-diagonal approximations; the rows of the left children give a sample
of the block's column space (Alg. 1 steps 1-2, eqs. "lvl1 sample1", "lvl2
sample1"); its QR factor Q (Alg. 1 step 3) is placed on the left-children rows,
multiplied again, and the right-children rows give C = B^T Q (Alg. 1 step 4,
eqs. "lvl1 sample2", "lvl2 sample2").  The block is Q C^T (eqs. "lowrnkB11",
"lowrnkB212").  Leaves come from stacked identities (eq. "leaf sample").

Sec. 3.3 ("Differentiating the HODLR approximation"): with the sampling
matrices held fixed, the same steps are differentiated in forward mode:
dY = (K_j - dH) X_R (eq. "db1r1", eq. "lvl2 sample1 diff"); dQ from Alg. 2;
dC = (K_j - dH) X_S + (K - H) [dQ; 0] restricted to the right rows (eqs.
"prod-rule-2", "lvl2 sample2 diff", "tmp2"); the derivative block is
dQ C^T + Q dC^T (eqs. "diff low-rank", "lvl2 block1 diff"); leaves by eq. "diag diff".

Here K and K_j are dense and "K - H" is formed explicitly: that is the plain
definition of what the matrix-free products compute.

Readings (the paper is silent or loose on these):
  * Alg. 1's Omega has q rows (the block's column count), not p.
  * Oversampling and truncation: when the sketch state is created, each block is
    sketched with ell = r + p_os columns, the right singular vectors V of that
    sample are computed, and V keeps k = min(r, #{sigma_i > 1e-10 sigma_1})
    columns, each signed so that its entry of largest magnitude is positive.
    Column j of every block of a level is scaled by one common factor (the
    geometric mean of s_1 / s_j over the level's blocks that keep it).  Omega V is
    then the block's fixed test matrix for every later theta (the paper's "draw
    once and keep fixed"), so Alg. 1 and Alg. 2 apply with k columns and R is
    invertible.  The common scale changes no block of K~ or K~_j (Q is that of the
    unscaled sample) and keeps R well conditioned where the blocks' spectra are alike.
  * QR sign gauge: diag(R) > 0.
  * Leaf blocks read from the stacked-identity sample are symmetrised, (D + D^T)/2.
  * Columns of all blocks at one level share one patterned matrix (one batched
    product per pass), as in eqs. "lvl2 sample1/2"; block P's columns beyond its
    k_P are zero.

Parity: pinned by exactness where the off-diagonal blocks have rank <= k
(1D stencil, and tiny 2D grids with full rank), by finite differences of the
construction with the sketch held fixed, and by Alg. 2 against finite
differences of a QR factorisation (tests/test_oracle_peeling.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .model import Tree


def qr_positive(Y: np.ndarray):
    """Thin QR with diag(R) > 0 (Alg. 1 step 3; sign gauge fixed)."""
    Q, R = np.linalg.qr(Y, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def qr_tangent(Q: np.ndarray, R: np.ndarray, dB: np.ndarray) -> np.ndarray:
    """Alg. 2: derivative of the thin-QR factor Q1 of B given dB.

    Y = Q1^T dB R^{-1};  Y = dOmega + dR R^{-1} with dOmega skew and dR R^{-1}
    upper triangular, so dOmega's strictly lower part is that of Y;
    dQ1 = Q1 dOmega + (I - Q1 Q1^T) dB R^{-1}.
    """
    QtdB = Q.T @ dB
    W = sla.solve_triangular(R, QtdB.T, trans="T", lower=False).T      # Q^T dB R^{-1}
    L = np.tril(W, -1)
    dOmega = L - L.T
    resid = dB - Q @ QtdB
    return Q @ dOmega + sla.solve_triangular(R, resid.T, trans="T", lower=False).T


def compress(Yl: np.ndarray, rank: int, tol: float = 1e-10) -> np.ndarray:
    """Frozen compression of an oversampled sketch (reading of Alg. 1 step 3): the
    kept right singular vectors of the sample (orthonormal columns)."""
    _, s, Vt = np.linalg.svd(Yl, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((Yl.shape[1], 0))
    k = int(min(rank, np.count_nonzero(s > tol * s[0])))
    V = Vt[:k].T.copy()
    for j in range(k):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V


def sample_spectrum(Yl: np.ndarray) -> np.ndarray:
    """Singular values of a block's oversampled sketch, decreasing."""
    return np.linalg.svd(Yl, compute_uv=False)


def level_scale(spectra, ks) -> np.ndarray:
    """Column scale shared by every block of one level: d_j = exp(mean over the blocks
    that keep column j of log(s_1 / s_j)).  The blocks of a level share the columns of
    one patterned test matrix, so only a scale common to all of them leaves every
    block's sample, and hence Q and K~, unchanged (a per-block scale would change the
    crosstalk between blocks, eqs. "lvl2 sample1/2"); it makes R well conditioned
    when the blocks' spectra are alike."""
    kmax = max(ks) if ks else 0
    d = np.ones(kmax)
    for j in range(kmax):
        logs = [np.log(s[0] / s[j]) for s, k in zip(spectra, ks) if k > j]
        d[j] = np.exp(np.mean(logs))
    return d


def _blocks(tree: Tree, l: int):
    """(parent index, rows of left child a, rows of right child b) at level l."""
    out = []
    for i in range(len(tree.nodes[l - 1])):
        out.append((i, tree.rows(l, 2 * i), tree.rows(l, 2 * i + 1)))
    return out


def patterned_right(tree: Tree, l: int, omega_l: np.ndarray, Vs) -> np.ndarray:
    """Level-l test matrix: rows of each right child b hold Omega_b V_P, others zero."""
    kcols = max([V.shape[1] for V in Vs] + [0])
    X = np.zeros((tree.n, kcols))
    for (i, a, b) in _blocks(tree, l):
        V = Vs[i]
        if V.shape[1]:
            X[b, :V.shape[1]] = omega_l[:, b].T @ V
    return X


def _level_step(Kr, tree, l, XR, ks, dKrs=()):
    """One level of value (and tangent) construction.  Returns per-block tuples."""
    n = tree.n
    kcols = XR.shape[1]
    Y = Kr @ XR
    dYs = [dKr @ XR for dKr in dKrs]
    XS = np.zeros((n, kcols))
    XdS = [np.zeros((n, kcols)) for _ in dKrs]
    QR = {}
    for (i, a, b) in _blocks(tree, l):
        k = ks[i]
        if k == 0:
            continue
        Q, R = qr_positive(Y[a, :k])
        QR[i] = (Q, R)
        XS[a, :k] = Q
        for j, dY in enumerate(dYs):
            XdS[j][a, :k] = qr_tangent(Q, R, dY[a, :k])
    Z = Kr @ XS
    dZs = [dKrs[j] @ XS + Kr @ XdS[j] for j in range(len(dKrs))]
    out = []
    for (i, a, b) in _blocks(tree, l):
        k = ks[i]
        if k == 0:
            out.append((i, a, b, None, None, [None] * len(dKrs), [None] * len(dKrs)))
            continue
        Q = QR[i][0]
        C = Z[b, :k]
        dQs = [XdS[j][a, :k] for j in range(len(dKrs))]
        dCs = [dZs[j][b, :k] for j in range(len(dKrs))]
        out.append((i, a, b, Q, C, dQs, dCs))
    return out


def sketch_create(K: np.ndarray, tree: Tree, omega: np.ndarray, rank: int, tol: float = 1e-10,
                  scaled: bool = True):
    """Create the frozen per-block compressions V[l-1][i] (ell x k_P) at theta_0
    (columns scaled by the level's common factors unless scaled=False; see level_scale)."""
    H = np.zeros_like(K)
    V_all = []
    for l in range(1, tree.levels + 1):
        Kr = K - H
        ell = omega.shape[1]
        full = [np.eye(ell)] * len(tree.nodes[l - 1])
        Yl = Kr @ patterned_right(tree, l, omega[l - 1], full)
        Vs = [compress(Yl[a], rank, tol) for (i, a, b) in _blocks(tree, l)]
        if scaled:
            d = level_scale([sample_spectrum(Yl[a]) for (i, a, b) in _blocks(tree, l)],
                            [V.shape[1] for V in Vs])
            Vs = [V * d[None, :V.shape[1]] for V in Vs]
        V_all.append(Vs)
        XR = patterned_right(tree, l, omega[l - 1], Vs)
        ks = [V.shape[1] for V in Vs]
        for (i, a, b, Q, C, _, _) in _level_step(Kr, tree, l, XR, ks):
            if Q is None:
                continue
            H[a, b] += Q @ C.T
            H[b, a] += C @ Q.T
    return V_all


def build(K: np.ndarray, dKs, tree: Tree, omega: np.ndarray, V_all):
    """Construct K~ and K~_j with the fixed sketch (omega, V_all).

    Returns dict with dense Kt, dKts (list), and the factors:
      Q[l-1][i], C[l-1][i], dQ[j][l-1][i], dC[j][l-1][i], D[leaf], dD[j][leaf].
    """
    n = tree.n
    p = len(dKs)
    H = np.zeros_like(K)
    dH = [np.zeros_like(K) for _ in range(p)]
    Qs, Cs = [], []
    dQs = [[] for _ in range(p)]
    dCs = [[] for _ in range(p)]
    for l in range(1, tree.levels + 1):
        Kr = K - H
        dKrs = [dKs[j] - dH[j] for j in range(p)]
        Vs = V_all[l - 1]
        XR = patterned_right(tree, l, omega[l - 1], Vs)
        ks = [V.shape[1] for V in Vs]
        res = _level_step(Kr, tree, l, XR, ks, dKrs)
        Qs.append([r[3] for r in res])
        Cs.append([r[4] for r in res])
        for j in range(p):
            dQs[j].append([r[5][j] for r in res])
            dCs[j].append([r[6][j] for r in res])
        for (i, a, b, Q, C, dQl, dCl) in res:
            if Q is None:
                continue
            H[a, b] += Q @ C.T
            H[b, a] += C @ Q.T
            for j in range(p):
                blk = dQl[j] @ C.T + Q @ dCl[j].T
                dH[j][a, b] += blk
                dH[j][b, a] += blk.T
    # leaf level: stacked identities
    leaves = tree.leaves
    nlmax = max(sz for _, sz in leaves)
    S = np.zeros((n, nlmax))
    for (off, sz) in leaves:
        S[off:off + sz, :sz] = np.eye(sz)
    Z = (K - H) @ S
    dZ = [(dKs[j] - dH[j]) @ S for j in range(p)]
    D, dD = [], [[] for _ in range(p)]
    Kt = H.copy()
    dKts = [dH[j].copy() for j in range(p)]
    for (off, sz) in leaves:
        blk = Z[off:off + sz, :sz]
        blk = 0.5 * (blk + blk.T)
        D.append(blk)
        Kt[off:off + sz, off:off + sz] = blk
        for j in range(p):
            db = dZ[j][off:off + sz, :sz]
            db = 0.5 * (db + db.T)
            dD[j].append(db)
            dKts[j][off:off + sz, off:off + sz] = db
    return dict(Kt=Kt, dKts=dKts, Q=Qs, C=Cs, dQ=dQs, dC=dCs, D=D, dD=dD)
