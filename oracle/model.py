"""Dense physics-based covariance and the spatial tree ordering (oracle side).

K(theta) = sigma2 * A^{-1} B^{-1} B^{-T} A^{-T} + tau2 * I, with
B = kappa^2 I + T, A = I + alpha T, T = -Laplacian (Dirichlet, h = 1/(N+1)).
This is the covariance model of Sec. 2.1 (eq. "cov model", exact for a linear
map y = L z with L = A^{-1}B^{-1} and K_z = I), with a nugget.

Parity: pinned against the spectral closed form (tests/test_oracle_model.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PARAMS = ("kappa", "alpha", "tau2", "sigma2")


def neg_laplacian(dim: int, N: int) -> sp.csc_matrix:
    """T = -Laplacian: (1/h^2) * 3-point (1D) or 5-point (2D) Dirichlet stencil.

    Grid index in 2D is iy*N + ix (x fastest).
    """
    h = 1.0 / (N + 1)
    main = np.full(N, 2.0)
    off = np.full(N - 1, -1.0)
    t1 = sp.diags([off, main, off], [-1, 0, 1], format="csc") / (h * h)
    if dim == 1:
        return t1
    eye = sp.identity(N, format="csc")
    return (sp.kron(eye, t1) + sp.kron(t1, eye)).tocsc()


def _solve_dense(op: sp.csc_matrix, rhs: np.ndarray) -> np.ndarray:
    lu = spla.splu(op.tocsc())
    return lu.solve(np.asarray(rhs, dtype=np.float64))


def dense_covariance(dim: int, N: int, theta_full, free=PARAMS):
    """Assemble K and dK/dtheta_j densely by applying the solve chain to unit vectors.

    Returns (K, [dK_j for j in free]) in natural grid order.
    M = A^{-1} B^{-1};  K = sigma2 M M^T + tau2 I.
      dM/dkappa = -A^{-1} B^{-1} (2 kappa I) B^{-1}
      dM/dalpha = -A^{-1} T A^{-1} B^{-1}          (dA/dalpha = T)
      dK/dtau2 = I,  dK/dsigma2 = M M^T
    """
    kappa, alpha, tau2, sigma2 = [float(t) for t in theta_full]
    T = neg_laplacian(dim, N)
    n = T.shape[0]
    eye = sp.identity(n, format="csc")
    A = (eye + alpha * T).tocsc()
    B = (kappa * kappa * eye + T).tocsc()
    I = np.eye(n)
    Binv = _solve_dense(B, I)              # B^{-1}
    M = _solve_dense(A, Binv)              # A^{-1} B^{-1}
    Kphys = M @ M.T
    K = sigma2 * Kphys + tau2 * I
    K = 0.5 * (K + K.T)
    dKs = []
    for name in free:
        if name == "kappa":
            dM = -2.0 * kappa * _solve_dense(A, _solve_dense(B, Binv))
            d = sigma2 * (dM @ M.T + M @ dM.T)
        elif name == "alpha":
            dM = -_solve_dense(A, T @ M)
            d = sigma2 * (dM @ M.T + M @ dM.T)
        elif name == "tau2":
            d = I.copy()
        elif name == "sigma2":
            d = Kphys.copy()
        else:
            raise ValueError(name)
        dKs.append(0.5 * (d + d.T))
    return K, dKs


def apply_covariance(dim: int, N: int, theta_full, X: np.ndarray, which="K") -> np.ndarray:
    """K X (or dK/dtheta_which X) by sparse solves, one right-hand side block at a time.

    Used where a dense K is too large: sampled columns at full size.
    X is in natural grid order, shape (n,) or (n, c).
    """
    kappa, alpha, tau2, sigma2 = [float(t) for t in theta_full]
    T = neg_laplacian(dim, N)
    n = T.shape[0]
    eye = sp.identity(n, format="csc")
    A = spla.splu((eye + alpha * T).tocsc())
    B = spla.splu((kappa * kappa * eye + T).tocsc())
    X = np.asarray(X, dtype=np.float64)
    # A, B symmetric: M^T x = B^{-1} A^{-1} x
    v1 = A.solve(X)
    v2 = B.solve(v1)
    v3 = B.solve(v2)
    v4 = A.solve(v3)
    if which == "K":
        return sigma2 * v4 + tau2 * X
    if which == "kappa":
        # d/dkappa of A^-1 B^-1 B^-1 A^-1 = -2 kappa A^-1 (B^-2 B^-1 + B^-1 B^-2) A^-1
        w = B.solve(v3)  # B^-3 A^-1 x
        return sigma2 * (-4.0 * kappa) * A.solve(w)
    if which == "alpha":
        # d/dalpha A^-1 B^-2 A^-1 = -A^-1 T A^-1 B^-2 A^-1 - A^-1 B^-2 A^-1 T A^-1
        t1 = A.solve(T @ v4)
        t2 = A.solve(B.solve(B.solve(A.solve(T @ v1))))
        return -sigma2 * (t1 + t2)
    if which == "tau2":
        return X.copy()
    if which == "sigma2":
        return v4
    raise ValueError(which)


# ---------------------------------------------------------------------------
# Spatial ordering: KD-tree-style recursive coordinate bisection (Sec. 5.2,
# "ordering of the observations is done by a KD-tree binary spatial
# partitioning"; leaf sizes Sec. 5.2 and 5.3).
# ---------------------------------------------------------------------------

class Tree:
    """Binary tree over tree-ordered rows.

    nodes[d] = list of (offset, size) of the 2^d nodes at depth d, left to right.
    perm[i] = natural grid index of tree position i.
    Rule: a node is a grid rectangle; split its longer side (x on ties); the
    left child receives floor(side/2) grid lines.  Leaves are listed depth-first,
    and points inside a leaf row-major (y outer, x inner).
    """

    def __init__(self, dim: int, N: int, levels: int):
        self.dim, self.N, self.levels = dim, N, levels
        rects = [(0, 0, N, N if dim == 2 else 1)]
        self.rects = [rects]
        for _ in range(levels):
            nxt = []
            for (x0, y0, w, h) in rects:
                if w >= h:
                    wl = w // 2
                    nxt += [(x0, y0, wl, h), (x0 + wl, y0, w - wl, h)]
                else:
                    hl = h // 2
                    nxt += [(x0, y0, w, hl), (x0, y0 + hl, w, h - hl)]
            rects = nxt
            self.rects.append(rects)
        self.nodes = []
        for rs in self.rects:
            off, lst = 0, []
            for (_, _, w, h) in rs:
                lst.append((off, w * h))
                off += w * h
            self.nodes.append(lst)
        perm = []
        for (x0, y0, w, h) in self.rects[-1]:
            for yy in range(y0, y0 + h):
                for xx in range(x0, x0 + w):
                    perm.append(yy * N + xx if dim == 2 else xx)
        self.perm = np.array(perm, dtype=np.int64)
        self.n = len(perm)

    def rows(self, d: int, i: int) -> slice:
        off, sz = self.nodes[d][i]
        return slice(off, off + sz)

    @property
    def leaves(self):
        return self.nodes[-1]


def to_tree_order(tree: Tree, M: np.ndarray) -> np.ndarray:
    """Permute a grid-ordered vector or matrix (rows and columns) into tree order."""
    p = tree.perm
    if M.ndim == 1:
        return M[p]
    if M.shape[0] == M.shape[1] == tree.n:
        return M[np.ix_(p, p)]
    return M[p]


class PointTree:
    """KD-tree of a scattered point set (Sec. 5.2, "KD-tree binary spatial
    partitioning"), with the interface of Tree: nodes[d] = (offset, size) of the 2^d
    nodes at depth d, perm[i] = point index of tree position i.

    Rule: a node's points are split along the longer side of their bounding box (x on
    ties); the floor(m/2) points with the smallest coordinate along it go left (ties:
    the other coordinate, then the point index).  Points inside a leaf are listed in
    increasing index.
    """

    def __init__(self, coords, levels: int):
        xy = np.asarray(coords, dtype=np.float64)
        if xy.ndim == 1:
            xy = xy[:, None]
        self.levels = levels
        groups = [np.arange(xy.shape[0])]
        self.groups = [groups]
        for _ in range(levels):
            nxt = []
            for g in groups:
                pts = xy[g]
                axis = 0
                if xy.shape[1] == 2 and len(g):
                    ext = pts.max(axis=0) - pts.min(axis=0)
                    axis = 1 if ext[1] > ext[0] else 0
                other = 1 - axis if xy.shape[1] == 2 else axis
                order = np.lexsort((g, pts[:, other], pts[:, axis]))   # last key is the primary one
                srt = g[order]
                half = len(g) // 2
                nxt += [srt[:half], srt[half:]]
            groups = nxt
            self.groups.append(groups)
        self.nodes = []
        for gs in self.groups:
            off, lst = 0, []
            for g in gs:
                lst.append((off, len(g)))
                off += len(g)
            self.nodes.append(lst)
        self.perm = np.concatenate([np.sort(g) for g in self.groups[-1]]).astype(np.int64)
        self.n = len(self.perm)

    def rows(self, d: int, i: int) -> slice:
        off, sz = self.nodes[d][i]
        return slice(off, off + sz)

    @property
    def leaves(self):
        return self.nodes[-1]
