"""Host logic of the maximum-likelihood driver (paper_2303_10102_amd/mle.py) on the CPU,
with a stand-in for the HMatrix whose log-likelihood is known in closed form:
L(phi) = -1/2 (phi - phi*)^T A (phi - phi*) in log-parameters phi = log(theta), with
an expected information that differs from A (as the HODLR information can differ from
the curvature of L~).  The driver must reach phi* to its tolerance, report the
intervals from the information it was given, recover from evaluations that fail, and
refuse a start that is not positive."""
import numpy as np
import pytest

from paper_2303_10102_amd.hmle import HmleError
from paper_2303_10102_amd.mle import fit


class QuadraticH:
    """iteration(theta_full, y) -> (L, grad of -L in theta, information in theta)."""

    def __init__(self, free_idx, phi_star, A, info_scale, fail_above=None):
        self.free_idx = tuple(free_idx)
        self.phi_star = np.asarray(phi_star, dtype=np.float64)
        self.A = np.asarray(A, dtype=np.float64)
        self.info_scale = np.asarray(info_scale, dtype=np.float64)
        self.fail_above = fail_above
        self.calls = 0
        self.failures = 0

    def iteration(self, theta_full, y):
        self.calls += 1
        th = np.asarray(theta_full, dtype=np.float64)[list(self.free_idx)]
        phi = np.log(th)
        if self.fail_above is not None and np.any(phi > self.fail_above):
            self.failures += 1
            raise HmleError("hm_iteration", "HM_E_NOT_SPD", "stand-in failure")
        d = phi - self.phi_star
        ll = -0.5 * float(d @ self.A @ d)
        g_theta = (self.A @ d) / th                          # -dL/dtheta
        info_phi = self.A * np.outer(self.info_scale, self.info_scale)
        fim = info_phi / np.outer(th, th)
        return ll, g_theta, fim


def _problem(**kw):
    A = np.array([[4.0, 1.2, 0.3], [1.2, 2.0, -0.4], [0.3, -0.4, 1.0]])
    phi_star = np.log([3.0, 0.02, 50.0])
    return QuadraticH((0, 2, 3), phi_star, A, info_scale=[1.3, 0.8, 1.1], **kw), phi_star, A


def test_reaches_the_maximum_with_a_mismatched_information():
    H, phi_star, A = _problem()
    theta0 = np.array([6.0, 1e-3, 0.005, 20.0])
    r = fit(H, None, theta0)
    assert r["converged"] and r["decrement"] < 1e-6
    # distance to phi* in the curvature's norm
    d = np.log(r["theta"]) - phi_star
    assert float(np.sqrt(d @ A @ d)) < 1e-5
    assert r["theta_full"][1] == theta0[1]              # the fixed parameter is untouched
    assert r["evaluations"] == H.calls and r["iterations"] < 30
    # intervals from the reported information (theta units)
    se = np.sqrt(np.diag(np.linalg.inv(r["fim"])))
    assert np.allclose(r["se"], se) and np.allclose(r["ci95"][:, 1] - r["ci95"][:, 0], 2 * 1.96 * se)


def test_recovers_from_failed_trial_points():
    # evaluations beyond log(theta) = 4.2 fail; the start's first steps overshoot there
    H, phi_star, A = _problem(fail_above=4.2)
    theta0 = np.array([0.05, 1e-3, 2.0, 60.0])
    r = fit(H, None, theta0, max_log_step=3.0)
    assert H.failures > 0 and r["converged"]
    d = np.log(r["theta"]) - phi_star
    assert float(np.sqrt(d @ A @ d)) < 1e-5


def test_rejects_a_start_that_is_not_positive():
    H, _, _ = _problem()
    with pytest.raises(ValueError):
        fit(H, None, np.array([3.0, 1e-3, -1.0, 50.0]))
