"""CPU pins of the observed-subset covariance (oracle/selection.py).

K_obs = sigma2 Phi M M^T Phi^T + tau2 I for a selection Phi of grid nodes (Sec. 5.1, eq.
"projection").  The oracle sums over the sine-transform modes; these checks hold it to
the sparse-solve dense assembly of the full-grid model (oracle.model.dense_covariance,
itself pinned to the spectral closed form) restricted to the selected rows and columns,
for random (irregular) and tensor-product (regular subgrid) selections, in 1D and 2D,
and for every parameter derivative.
"""
import numpy as np
import pytest

from oracle.model import dense_covariance
from oracle.selection import grid_coords, selected_covariance

THETA = (7.0, 3e-3, 0.01, 2.0)


def _check(dim, N, obs, theta=THETA):
    K, dK = selected_covariance(dim, N, theta, obs)
    Kf, dKf = dense_covariance(dim, N, theta)
    ix = np.ix_(obs, obs)
    assert np.abs(K - Kf[ix]).max() <= 1e-13 * np.abs(Kf).max()
    for a, b in zip(dK, dKf):
        assert np.abs(a - b[ix]).max() <= 1e-13 * np.abs(b).max()
    return K, dK


@pytest.mark.parametrize("dim,N,frac", [(2, 14, 0.4), (1, 40, 0.6)])
def test_random_selection_matches_dense_assembly(dim, N, frac):
    rng = np.random.default_rng(3)
    full = N ** dim
    obs = rng.choice(full, size=int(frac * full), replace=False)   # unsorted: any observation order
    _check(dim, N, obs)


def test_regular_subgrid_matches_dense_assembly_and_the_general_sum():
    N = 20
    s = np.arange(1, N, 3)
    obs = (s[None, :] + N * s[:, None]).ravel()          # tensor product, y outer
    K, dK = _check(2, N, obs)
    # the same nodes in another order take the general mode sum: the same matrix permuted
    p = np.random.default_rng(4).permutation(obs.size)
    K2, dK2 = selected_covariance(2, N, THETA, obs[p])
    assert np.abs(K2 - K[np.ix_(p, p)]).max() <= 1e-14 * np.abs(K).max()
    for a, b in zip(dK2, dK):
        assert np.abs(a - b[np.ix_(p, p)]).max() <= 1e-14 * np.abs(b).max()


def test_every_node_selected_is_the_full_model():
    N = 10
    obs = np.arange(N * N)
    K, _ = selected_covariance(2, N, THETA, obs)
    Kf, _ = dense_covariance(2, N, THETA)
    assert np.abs(K - Kf).max() <= 1e-13 * np.abs(Kf).max()


def test_nugget_on_observations_only_and_coordinates():
    N = 12
    obs = np.array([5, 17, 18, 100, 143])
    K, dK = selected_covariance(2, N, THETA, obs, free=("tau2", "sigma2"))
    assert np.array_equal(dK[0], np.eye(5))
    assert np.allclose(K - THETA[3] * dK[1], THETA[2] * np.eye(5), rtol=0, atol=1e-15)
    xy = grid_coords(2, N, obs)
    assert np.array_equal(xy[:, 0], obs % N) and np.array_equal(xy[:, 1], obs // N)
