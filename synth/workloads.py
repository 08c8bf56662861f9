"""Seeded synthetic workloads for the SPDE-driven covariance model.

This module only synthesises inputs: the grid and parameter configuration of
each workload, the observed sample y, and the Gaussian draws of the fixed
sketching test matrices.  It contains no step of the likelihood method
(no peeling, factorisation or trace); both the HIP library's tests and the
CPU oracle take their inputs from here.

Model (paper Sec. 2.1, eq. "cov model" with a linear map, so the linearised
covariance is exact):  y = sigma * A^{-1} B^{-1} w + tau * eps,
    B = kappa^2 I - Lap,   A = I - alpha Lap,
with Lap the 3-point (1D) or 5-point (2D) Dirichlet Laplacian on the open
unit interval/square, h = 1/(N+1), and w, eps ~ N(0, I).  B is the
finite-difference analogue of the Whittle operator (1/l^2 - Delta) of the
paper's Matern SPDE (Sec. 5.1, eq. "SPDE") with kappa = 1/l.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PARAM_NAMES = ("kappa", "alpha", "tau2", "sigma2")


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int            # 1 or 2
    N: int              # grid side (1D: number of points)
    leaf: int           # target leaf size; levels = floor(log2(n / leaf))
    rank: int           # off-diagonal target rank r
    oversample: int     # extra sketch columns used once, when the sketch is created
    kappa: float
    alpha: float
    tau2: float
    sigma2: float
    free: tuple         # free parameters, in gradient / Fisher order
    data_seed: int
    sketch_seed: int

    @property
    def n(self) -> int:
        return self.N if self.dim == 1 else self.N * self.N

    @property
    def h(self) -> float:
        return 1.0 / (self.N + 1)

    @property
    def levels(self) -> int:
        return int(math.floor(math.log2(self.n / self.leaf)))

    @property
    def ell(self) -> int:
        return self.rank + self.oversample

    @property
    def theta_full(self) -> np.ndarray:
        return np.array([self.kappa, self.alpha, self.tau2, self.sigma2], dtype=np.float64)

    @property
    def free_idx(self) -> tuple:
        return tuple(PARAM_NAMES.index(f) for f in self.free)

    @property
    def theta(self) -> np.ndarray:
        return self.theta_full[list(self.free_idx)]

    def with_theta(self, theta) -> "Workload":
        vals = dict(zip(self.free, [float(t) for t in theta]))
        return replace(self, **vals)


# sigma^2 of the 256^2 workload at the generating parameters.  The workload is
# the 128^2 model on a 256^2 grid "with K scaled by sigma^2", so its true value
# is the unscaled model's, 1.  (A unit-marginal-variance scaling, ~5.3e8, makes
# the rank-48 approximation indefinite on the 64^2 analogue.)
SIGMA2_256 = 1.0

WORKLOADS = {
    # 1D, n=1024: the small plain-FP64 case.
    "1d_n1024": Workload("1d_n1024", 1, 1024, 64, 16, 10, 10.0, 0.01, 1e-4, 1.0,
                         ("kappa", "tau2"), 1, 101),
    # 2D 128x128 (n=16384), theta = (kappa, alpha, tau2).
    "2d_n16384": Workload("2d_n16384", 2, 128, 256, 32, 10, 20.0, 2e-4, 1e-3, 1.0,
                          ("kappa", "alpha", "tau2"), 2, 102),
    # 2D 256x256 (n=65536), theta = (kappa, alpha, tau2, sigma2): the headline case.
    "2d_n65536": Workload("2d_n65536", 2, 256, 256, 48, 10, 20.0, 2e-4, 1e-3, SIGMA2_256,
                          ("kappa", "alpha", "tau2", "sigma2"), 3, 103),
    # Same model on a 64x64 grid (n=4096): the dense-oracle-sized companion.
    "2d_n4096": Workload("2d_n4096", 2, 64, 256, 48, 10, 20.0, 2e-4, 1e-3, SIGMA2_256,
                         ("kappa", "alpha", "tau2", "sigma2"), 3, 103),
}


def small_workload(dim=2, N=32, leaf=64, rank=16, oversample=10, free=("kappa", "alpha", "tau2", "sigma2"),
                   kappa=20.0, alpha=2e-4, tau2=1e-3, sigma2=1.0e3, data_seed=7, sketch_seed=70,
                   name=None) -> Workload:
    """A small workload with the shape of the headline one, for parity tests."""
    return Workload(name or f"{dim}d_N{N}_leaf{leaf}_r{rank}", dim, N, leaf, rank, oversample,
                    kappa, alpha, tau2, sigma2, tuple(free), data_seed, sketch_seed)


BATCH_SIDES = (64, 96, 128, 192, 256)


def batched_fields(count: int = 64, seed: int = 4, sides=BATCH_SIDES, leaf: int = 256, rank: int = 32,
                   oversample: int = 10) -> list:
    """Independent 2D fields of uneven size and parameters (the batched workload).

    Per field i = 0..count-1, drawn from numpy.random.default_rng(seed) in this
    order: grid side uniform over `sides`, kappa ~ U[5, 40], alpha ~ U[1e-4, 5e-4],
    log tau2 ~ U[log 1e-4, log 1e-2]; sigma2 = 1; theta = (kappa, alpha, tau2) free;
    data seed 1000 + i, sketch seed 2000 + i.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        side = int(sides[int(rng.integers(0, len(sides)))])
        kappa = float(rng.uniform(5.0, 40.0))
        alpha = float(rng.uniform(1e-4, 5e-4))
        tau2 = float(math.exp(rng.uniform(math.log(1e-4), math.log(1e-2))))
        out.append(Workload(f"field{i:02d}_N{side}", 2, side, leaf, rank, oversample, kappa, alpha, tau2, 1.0,
                            ("kappa", "alpha", "tau2"), 1000 + i, 2000 + i))
    return out


def _lap(dim: int, N: int) -> sp.csc_matrix:
    h = 1.0 / (N + 1)
    e = np.ones(N)
    t1 = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1]) / (h * h)
    if dim == 1:
        return t1.tocsc()
    i1 = sp.identity(N)
    # grid index = iy * N + ix  (x fastest)
    return (sp.kron(i1, t1) + sp.kron(t1, i1)).tocsc()


def sample_y(w: Workload) -> np.ndarray:
    """One draw y = sigma A^-1 B^-1 w + tau eps in natural grid order (x fastest).

    w then eps are drawn from numpy.random.default_rng(data_seed), in that order.
    """
    rng = np.random.default_rng(w.data_seed)
    wv = rng.standard_normal(w.n)
    ev = rng.standard_normal(w.n)
    T = _lap(w.dim, w.N)
    I = sp.identity(w.n, format="csc")
    A = (I + w.alpha * T).tocsc()
    B = (w.kappa ** 2 * I + T).tocsc()
    v = spla.spsolve(B, wv)
    v = spla.spsolve(A, v)
    return math.sqrt(w.sigma2) * v + math.sqrt(w.tau2) * ev


def sketch_draws(w: Workload) -> np.ndarray:
    """Gaussian draws for the fixed sketching matrices: shape (levels, ell, n).

    omega[l-1, j, i] is the draw for tree position i (rows in tree order), sketch
    column j, at level l.  Only rows of right children at depth l are used by the
    method; the others are ignored.  Drawn once from default_rng(sketch_seed).
    """
    rng = np.random.default_rng(w.sketch_seed)
    return rng.standard_normal((w.levels, w.ell, w.n))


def scattered_points(n: int, seed: int, dim: int = 2) -> np.ndarray:
    """n points drawn uniformly in the unit square (or interval), seeded (n x dim)."""
    return np.random.default_rng(seed).random((n, dim))


def scattered_sample(n: int, seed: int, scale: float) -> np.ndarray:
    """A seeded sample vector of n standard normals times scale (an observation vector
    for likelihood evaluations at scattered points)."""
    return scale * np.random.default_rng(seed).standard_normal(n)


@dataclass(frozen=True)
class OpWorkload:
    """A likelihood problem on scattered points with a caller-supplied covariance
    operator K = sigma2 K_op(theta0, theta1) + tau2 I (the operator itself is the
    caller's: here the anisotropic Matern-3/2 kernel, range theta0, y-stretch theta1)."""
    name: str
    dim: int
    n: int
    leaf: int
    rank: int
    oversample: int
    theta0: float
    theta1: float
    tau2: float
    sigma2: float
    free: tuple
    coord_seed: int
    data_seed: int
    sketch_seed: int

    @property
    def levels(self) -> int:
        return int(math.floor(math.log2(self.n / self.leaf)))

    @property
    def ell(self) -> int:
        return self.rank + self.oversample

    @property
    def theta_full(self) -> np.ndarray:
        return np.array([self.theta0, self.theta1, self.tau2, self.sigma2], dtype=np.float64)

    @property
    def free_idx(self) -> tuple:
        return tuple(PARAM_NAMES.index(f) for f in self.free)

    def coords(self) -> np.ndarray:
        return scattered_points(self.n, self.coord_seed, self.dim)

    def sample(self) -> np.ndarray:
        return scattered_sample(self.n, self.data_seed, math.sqrt(self.sigma2 + self.tau2))


OP_WORKLOADS = {
    # 1500 points uniform in the unit square, leaf 64 (4 levels), rank 24 + 10; range 0.3
    # and nugget 0.2 keep the rank-24 approximation positive definite
    "op2d_n1500": OpWorkload("op2d_n1500", 2, 1500, 64, 24, 10, 0.3, 1.3, 0.2, 1.0,
                             ("kappa", "alpha", "tau2", "sigma2"), 11, 12, 13),
    # 1000 points uniform on the unit interval, leaf 64 (3 levels)
    "op1d_n1000": OpWorkload("op1d_n1000", 1, 1000, 64, 16, 10, 0.05, 1.0, 1e-2, 2.0,
                             ("kappa", "tau2", "sigma2"), 21, 22, 23),
}


@dataclass(frozen=True)
class AdrWorkload:
    """The advection-diffusion-reaction model on an N x N grid of the unit square:
    K = sigma2 L^{-1} B^{-2} L^{-T} + tau2 I, L = -kd Lap + v . grad + c, B = kappa^2 - Lap,
    theta = (kappa, c, tau2, sigma2) in the slots of (theta0, theta1, tau2, sigma2)."""
    name: str
    N: int
    leaf: int
    rank: int
    oversample: int
    kd: float
    vx: float
    vy: float
    kappa: float
    c: float
    tau2: float
    sigma2: float
    free: tuple
    data_seed: int
    sketch_seed: int
    dim: int = 2

    @property
    def n(self) -> int:
        return self.N * self.N

    @property
    def levels(self) -> int:
        return int(math.floor(math.log2(self.n / self.leaf)))

    @property
    def ell(self) -> int:
        return self.rank + self.oversample

    @property
    def theta_full(self) -> np.ndarray:
        return np.array([self.kappa, self.c, self.tau2, self.sigma2], dtype=np.float64)

    def sample(self) -> np.ndarray:
        """y = sigma L^{-1} B^{-1} w + tau eps (w then eps from default_rng(data_seed)), by
        sparse solves on the host (grid order, x fastest)."""
        N, h = self.N, 1.0 / (self.N + 1)
        one = np.ones(N)
        T1 = sp.diags([-one[:-1], 2 * one, -one[:-1]], [-1, 0, 1]) / (h * h)
        G1 = sp.diags([-one[:-1], one[:-1]], [-1, 1]) / (2 * h)
        I1 = sp.identity(N)
        lap = sp.kron(I1, T1) + sp.kron(T1, I1)
        Lop = (self.kd * lap + self.vx * sp.kron(I1, G1) + self.vy * sp.kron(G1, I1)
               + self.c * sp.identity(N * N)).tocsc()
        Bop = (self.kappa ** 2 * sp.identity(N * N) + lap).tocsc()
        rng = np.random.default_rng(self.data_seed)
        w = rng.standard_normal(N * N)
        eps = rng.standard_normal(N * N)
        return math.sqrt(self.sigma2) * spla.spsolve(Lop, spla.spsolve(Bop, w)) + math.sqrt(self.tau2) * eps


ADR_WORKLOADS = {
    # 32 x 32 (n = 1024), leaf 64, rank 16 + 10; advection (2.5, 1) with kd = 1: cell Peclet
    # numbers 0.038 and 0.015; sigma2 gives unit mean physics variance, nugget 0.05
    "adr_n1024": AdrWorkload("adr_n1024", 32, 64, 16, 10, 1.0, 2.5, 1.0, 10.0, 1.0, 0.05, 5.0e9,
                             ("kappa", "alpha", "tau2", "sigma2"), 31, 32),
    # odd sides: 45 x 45 (leaves of 121-144 points)
    "adr_n2025": AdrWorkload("adr_n2025", 45, 64, 16, 10, 1.0, 2.5, 1.0, 10.0, 1.0, 0.05, 1.0e10,
                             ("kappa", "alpha", "tau2", "sigma2"), 33, 34),
    # 256 x 256 (n = 65536), leaf 256, rank 48 + 10: the headline grid with this model
    "adr_n65536": AdrWorkload("adr_n65536", 256, 256, 48, 10, 1.0, 2.5, 1.0, 20.0, 1.0, 0.05, 1.0e11,
                              ("kappa", "alpha", "tau2", "sigma2"), 35, 36),
}


@dataclass(frozen=True)
class SelWorkload:
    """Observations of a subset of the stencil field's grid points (the observation
    operator a selection): the physics on the full grid of side N, the nugget on the
    observations.  obs_kind "regular": nodes stride*s + offset on each axis (s = 0, 1, ...);
    "random": n_obs distinct nodes drawn with numpy.random.default_rng(obs_seed), sorted."""
    name: str
    dim: int
    N: int
    obs_kind: str
    stride: int
    offset: int
    n_obs: int
    obs_seed: int
    leaf: int
    rank: int
    oversample: int
    kappa: float
    alpha: float
    tau2: float
    sigma2: float
    free: tuple
    data_seed: int
    sketch_seed: int

    def obs(self) -> np.ndarray:
        """Observed grid indices (x fastest in 2D), in observation order."""
        if self.obs_kind == "regular":
            s = np.arange(self.offset, self.N, self.stride)
            if self.dim == 1:
                return s.astype(np.int64)
            return (s[None, :] + self.N * s[:, None]).ravel().astype(np.int64)   # y outer, x inner
        full = self.N ** self.dim
        rng = np.random.default_rng(self.obs_seed)
        return np.sort(rng.choice(full, size=self.n_obs, replace=False)).astype(np.int64)

    @property
    def n(self) -> int:
        return int(self.obs().size)

    @property
    def levels(self) -> int:
        return int(math.floor(math.log2(self.n / self.leaf)))

    @property
    def ell(self) -> int:
        return self.rank + self.oversample

    @property
    def theta_full(self) -> np.ndarray:
        return np.array([self.kappa, self.alpha, self.tau2, self.sigma2], dtype=np.float64)

    @property
    def free_idx(self) -> tuple:
        return tuple(PARAM_NAMES.index(f) for f in self.free)

    def field(self) -> Workload:
        """The full-grid workload with the same parameters and data seed."""
        return Workload(self.name + "_grid", self.dim, self.N, self.leaf, self.rank, self.oversample, self.kappa,
                        self.alpha, self.tau2, self.sigma2, self.free, self.data_seed, self.sketch_seed)

    def sample(self) -> np.ndarray:
        """A draw of the full field (sample_y) read at the observed nodes."""
        return sample_y(self.field())[self.obs()]


SEL_WORKLOADS = {
    # the 256^2 headline field observed on the regular 64 x 64 subgrid of nodes 4 s + 1
    # (n = 4096, leaf 256, 4 levels, rank 48 + 10; physics at 256^2)
    "sel_n4096": SelWorkload("sel_n4096", 2, 256, "regular", 4, 1, 0, 0, 256, 48, 10, 20.0, 2e-4, 1e-3, 1.0,
                             ("kappa", "alpha", "tau2", "sigma2"), 41, 42),
    # 1500 random nodes of a 48 x 48 grid (partial, irregular observations), leaf 64,
    # rank 16 + 10, physics-dominated scale
    "sel_n1500": SelWorkload("sel_n1500", 2, 48, "random", 0, 0, 1500, 43, 64, 16, 10, 20.0, 2e-4, 1e-3, 1.0e3,
                             ("kappa", "alpha", "tau2", "sigma2"), 44, 45),
    # 1D: 700 random points of a 1000-point line, leaf 64
    "sel1d_n700": SelWorkload("sel1d_n700", 1, 1000, "random", 0, 0, 700, 46, 64, 16, 10, 10.0, 0.01, 1e-4, 1.0e4,
                              ("kappa", "alpha", "tau2", "sigma2"), 47, 48),
}


BIV_PARAM_NAMES = ("kappa", "alpha", "tau2", "sigma2", "tau2_2")


@dataclass(frozen=True)
class BivWorkload:
    """Bivariate co-kriging on an N x N (or N) Dirichlet grid: y1 = sigma B^-1 w + tau1 eps1,
    y2 = sigma A^-1 B^-1 w + tau2 eps2 at every node, stacked y = (y1; y2);
    theta_full = (kappa, alpha, tau2_1, sigma2, tau2_2)."""
    name: str
    dim: int
    N: int
    leaf: int
    rank: int
    oversample: int
    kappa: float
    alpha: float
    tau2: float
    sigma2: float
    tau2_2: float
    free: tuple
    data_seed: int
    sketch_seed: int

    @property
    def n_loc(self) -> int:
        return self.N if self.dim == 1 else self.N * self.N

    @property
    def n(self) -> int:
        return 2 * self.n_loc

    @property
    def levels(self) -> int:
        return int(math.floor(math.log2(self.n / self.leaf)))

    @property
    def ell(self) -> int:
        return self.rank + self.oversample

    @property
    def theta_full(self) -> np.ndarray:
        return np.array([self.kappa, self.alpha, self.tau2, self.sigma2, self.tau2_2], dtype=np.float64)

    @property
    def free_idx(self) -> tuple:
        return tuple(BIV_PARAM_NAMES.index(f) for f in self.free)

    def sample(self) -> np.ndarray:
        """w, eps1, eps2 drawn from default_rng(data_seed) in that order (natural order)."""
        rng = np.random.default_rng(self.data_seed)
        wv = rng.standard_normal(self.n_loc)
        e1 = rng.standard_normal(self.n_loc)
        e2 = rng.standard_normal(self.n_loc)
        T = _lap(self.dim, self.N)
        I = sp.identity(self.n_loc, format="csc")
        A = (I + self.alpha * T).tocsc()
        B = (self.kappa ** 2 * I + T).tocsc()
        u = spla.spsolve(B, wv)
        v = spla.spsolve(A, u)
        s = math.sqrt(self.sigma2)
        return np.r_[s * u + math.sqrt(self.tau2) * e1, s * v + math.sqrt(self.tau2_2) * e2]


BIV_WORKLOADS = {
    # 24 x 24 locations x 2 variables (n = 1152), leaf 128 (3 levels), rank 16 + 10
    "biv_n1152": BivWorkload("biv_n1152", 2, 24, 128, 16, 10, 20.0, 2e-4, 1e-3, 2.0e3, 2e-3,
                             ("kappa", "alpha", "tau2", "sigma2", "tau2_2"), 51, 52),
    # odd sides: 21 x 21 x 2 (n = 882), leaf 96 (3 levels), uneven location leaves
    "biv_n882": BivWorkload("biv_n882", 2, 21, 96, 16, 10, 20.0, 2e-4, 1e-3, 2.0e3, 2e-3,
                            ("kappa", "alpha", "tau2", "sigma2", "tau2_2"), 53, 54),
    # 1D: 500 locations x 2 (n = 1000), leaf 64 (3 levels), two free nuggets and kappa
    "biv1d_n1000": BivWorkload("biv1d_n1000", 1, 500, 64, 16, 10, 10.0, 0.01, 1e-4, 1.0e4, 3e-4,
                               ("kappa", "tau2", "sigma2", "tau2_2"), 55, 56),
    # the co-kriging workload: 362 x 362 x 2 (n = 262088), leaf 512 (8 levels, leaves of up to
    # 2 x 529 rows), rank 64 + 10, theta = (kappa, alpha, tau2_1, sigma2, tau2_2)
    "biv_n262088": BivWorkload("biv_n262088", 2, 362, 512, 64, 10, 20.0, 2e-4, 1e-3, 1.0, 2e-3,
                               ("kappa", "alpha", "tau2", "sigma2", "tau2_2"), 57, 58),
}
