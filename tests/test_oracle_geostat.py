"""Pins of the oracle's geostatistical inversion (Algorithm 2) and Crank-Nicolson data:

* the covariance against its closed form at hand-computed distances, symmetry and
  positive definiteness;
* the saddle-point update of eq:inversion1 with a linear forward model against the textbook
  universal-kriging estimate with an unknown constant mean, and against the optimality
  conditions of the MAP objective (gradient in s and in beta zero);
* Crank-Nicolson heads converging to the Laplace-transform heads at second order.
"""
import numpy as np
import pytest

from oracle.contour import talbot_nodes  # noqa: F401  (contour used through heads)
from oracle.geostat import cell_centres, exp_covariance, saddle_update
from oracle.heads import heads
from oracle.timestep import crank_nicolson_heads
from workloads.configs import T_D, make_problem


def test_covariance_closed_form():
    n, h = (6, 5, 1), (0.1, 0.2, 1.0)
    Q = exp_covariance(n, h, 2.0, (0.3, 0.5, 1.0), 2)
    # cell (0, 0) against (3, 0): dx = 0.3 -> 0.3 / 0.3 = 1; against (0, 2): dy = 0.4 -> 0.8;
    # against (3, 2): sqrt(1 + 0.64)
    assert Q[0, 3] == pytest.approx(2.0 * np.exp(-1.0), rel=1e-14)
    assert Q[0, 12] == pytest.approx(2.0 * np.exp(-0.8), rel=1e-14)
    assert Q[0, 15] == pytest.approx(2.0 * np.exp(-np.sqrt(1.64)), rel=1e-14)
    assert np.array_equal(Q, Q.T) and np.all(np.diag(Q) == 2.0)
    assert np.linalg.eigvalsh(Q).min() > 0
    x = cell_centres(n, h, 2)
    assert np.allclose(x[7], [0.15, 0.3])  # cell (1, 1), x fastest


def _linear_case(seed=4, M=9, n=(7, 6, 1)):
    rng = np.random.default_rng(seed)
    h = (1.0 / n[0], 1.0 / n[1], 1.0)
    Q = exp_covariance(n, h, 1.3, (0.25, 0.25, 1.0), 2)
    N = Q.shape[0]
    H = rng.standard_normal((M, N)) / np.sqrt(N)
    y = rng.standard_normal(M)
    return H, Q, y, 1e-2, rng.standard_normal(N)


def test_saddle_update_is_universal_kriging_for_a_linear_model():
    H, Q, y, r, s0 = _linear_case()
    s1, xi, beta = saddle_update(H, H @ s0, y, s0, Q @ H.T, r)
    # textbook: Sigma = H Q H^T + R, beta = (1^T H^T Sigma^-1 H 1)^-1 1^T H^T Sigma^-1 y,
    # s = 1 beta + Q H^T Sigma^-1 (y - H 1 beta)
    M, N = H.shape
    one = np.ones(N)
    Si = np.linalg.inv(H @ Q @ H.T + r * np.eye(M))
    Hx = H @ one
    b_ref = (Hx @ Si @ y) / (Hx @ Si @ Hx)
    s_ref = one * b_ref + Q @ H.T @ Si @ (y - Hx * b_ref)
    assert beta == pytest.approx(b_ref, rel=1e-10)
    assert np.allclose(s1, s_ref, rtol=1e-10, atol=1e-12)
    # the result does not depend on the linearisation point for a linear model
    s1b, _, _ = saddle_update(H, H @ (2 * s0), y, 2 * s0, Q @ H.T, r)
    assert np.allclose(s1, s1b, rtol=1e-10, atol=1e-12)


def test_saddle_update_satisfies_the_map_optimality_conditions():
    # minimiser of 1/2 ||y - H s||^2 / r + 1/2 (s - X beta)^T Q^-1 (s - X beta) over s and beta
    H, Q, y, r, s0 = _linear_case(seed=9)
    s1, _, beta = saddle_update(H, H @ s0, y, s0, Q @ H.T, r)
    g = np.linalg.solve(Q, s1 - beta)  # Q^-1 (s - X beta)
    grad_s = H.T @ (H @ s1 - y) / r + g
    grad_beta = -g.sum()
    assert np.abs(grad_s).max() <= 1e-8 * (np.abs(H.T @ y).max() / r)
    assert abs(grad_beta) <= 1e-8 * np.abs(g).max() * g.size


def test_crank_nicolson_converges_to_the_transform_heads():
    p = make_problem("THT", n=(24, 24))
    times = p.times[:2]
    ref = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers[:6], times, 40, ndim=2)
    errs = []
    # (coarser steps leave the asymptotic range: the trapezoidal rule damps the stiff modes of
    # the step start poorly)
    for dt in (0.005 * T_D, 0.0025 * T_D):
        cn = crank_nicolson_heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers[:6], times, dt, ndim=2)
        errs.append(np.abs(cn - ref).max() / np.abs(ref).max())
    assert errs[1] < 1e-6
    assert 3.5 < errs[0] / errs[1] < 4.5  # second order in dt
