"""CPU pins of the oracle's operator-model pieces: the Matern-3/2 kernel and its
derivatives (oracle/operators.py) and the KD-tree of scattered points
(oracle/model.py PointTree)."""
import numpy as np

from oracle.model import PointTree, Tree
from oracle.operators import matern32
from synth import scattered_points


def test_matern32_values_and_derivatives():
    xy = scattered_points(60, 3)
    ell, a = 0.2, 1.4
    K, dl, da = matern32(xy, ell, a)
    assert np.allclose(np.diag(K), 1.0, rtol=0, atol=1e-15)
    assert np.array_equal(K, K.T)
    assert np.linalg.eigvalsh(K).min() > -1e-12
    # one entry by hand: k(d) = (1 + sqrt(3) d / ell) exp(-sqrt(3) d / ell)
    d = np.hypot(xy[3, 0] - xy[7, 0], a * (xy[3, 1] - xy[7, 1]))
    r = np.sqrt(3) * d / ell
    assert abs(K[3, 7] - (1 + r) * np.exp(-r)) <= 1e-15
    for j, (h, D) in enumerate(((1e-6 * ell, dl), (1e-6 * a, da))):
        args_p = (ell + h, a) if j == 0 else (ell, a + h)
        args_m = (ell - h, a) if j == 0 else (ell, a - h)
        fd = (matern32(xy, *args_p)[0] - matern32(xy, *args_m)[0]) / (2 * h)
        assert np.max(np.abs(fd - D)) <= 1e-8 * np.max(np.abs(D)), j
    # one dimension: no y term, the a-derivative vanishes
    K1, _, da1 = matern32(scattered_points(20, 4, dim=1), ell, a)
    assert np.all(da1 == 0.0) and np.linalg.eigvalsh(K1).min() > -1e-12


def test_point_tree_on_a_grid_equals_the_rectangle_tree():
    # even splits: the median-by-count rule and the rectangle rule give the same tree
    N = 16
    xs, ys = np.meshgrid(np.arange(N), np.arange(N))
    xy = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(float)   # index = y N + x
    for levels in (1, 2, 3, 4):
        assert np.array_equal(PointTree(xy, levels).perm, Tree(2, N, levels).perm)


def test_point_tree_rule_by_hand():
    # 7 points, 2 levels: root splits along x (extent 6 vs 2), 3 go left
    xy = np.array([[0, 0], [6, 1], [2, 2], [1, 0.5], [5, 2], [3, 1], [4, 0]], dtype=float)
    t = PointTree(xy, 2)
    assert t.nodes[1] == [(0, 3), (3, 4)]
    left = set(t.perm[:3])
    assert left == {0, 2, 3}            # x = 0, 2, 1
    # left child {0, 2, 3}: extents x 2, y 2 -> x on ties; 1 point left (x = 0)
    assert list(t.perm[:1]) == [0] and sorted(t.perm[1:3]) == [2, 3]
    # right child {1, 4, 5, 6}: extent x 3 > y 2: x = 3, 4 left
    assert sorted(t.perm[3:5]) == [5, 6] and sorted(t.perm[5:]) == [1, 4]
    # every leaf lists its points in increasing index
    for off, sz in t.leaves:
        assert list(t.perm[off:off + sz]) == sorted(t.perm[off:off + sz])


def test_point_tree_scattered():
    xy = scattered_points(1500, 11)
    t = PointTree(xy, 4)
    assert sorted(t.perm) == list(range(1500))
    sizes = [sz for _, sz in t.leaves]
    assert max(sizes) - min(sizes) <= 1 + 4 and sum(sizes) == 1500
