"""Host-side test helpers checked on the CPU: the H-matvec used by the full-size
GPU checks agrees with the dense matrix of the same representation."""
import numpy as np

from tests._cases import densify, hmatvec


def test_hmatvec_matches_densify():
    rng = np.random.default_rng(0)
    levels, kc, n = 3, 5, 64
    F = rng.standard_normal((levels * kc, n))
    dF = rng.standard_normal((levels * kc, n))
    nl = n >> levels
    lv = rng.standard_normal((1 << levels, nl, nl))
    dlv = rng.standard_normal((1 << levels, nl, nl))
    x = rng.standard_normal((n, 3))
    K = densify(F, lv, levels, kc, n)
    dK = densify(F, dlv, levels, kc, n, dF=dF)
    assert np.abs(hmatvec(F, lv, levels, kc, x) - K @ x).max() < 1e-12 * np.abs(K).max() * n
    assert np.abs(hmatvec(F, lv, levels, kc, x[:, 1]) - K @ x[:, 1]).max() < 1e-12 * np.abs(K).max() * n
    got = hmatvec(F, lv, levels, kc, x, dF=dF, dleaves=dlv)
    assert np.abs(got - dK @ x).max() < 1e-12 * np.abs(dK).max() * n


def test_densify_block_layout():
    # one level, kc = 1: the off-diagonal block is the outer product of the two halves
    n = 4
    F = np.array([[1.0, 2.0, 3.0, 4.0]])
    lv = np.zeros((2, 2, 2))
    K = densify(F, lv, 1, 1, n)
    assert np.array_equal(K[:2, 2:], np.outer([1.0, 2.0], [3.0, 4.0]))
    assert np.array_equal(K[2:, :2], np.outer([3.0, 4.0], [1.0, 2.0]))
