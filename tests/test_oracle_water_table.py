"""Pins for the oracle's linearised water-table boundary (eqn:timedomain,
third condition; the boundary term of M_ij in Section 2.1).

* One cell closed by no-flux walls and one water-table face: the head of a
  constant pumping rate q rises as q t / (S V + S_y A), the storage of the
  cell plus that of the face.
* A heterogeneous grid closed the same way: once the transient has died,
  every cell rises at the common rate q / (S Vol + S_y A_w), the domain's
  total storage capacity (mass balance; fixes the face area and that the
  face carries no conductive flux).
* S_y = 0 turns the face into a no-flux face.
* The storage sensitivity with a water table against central differences of
  the heads (the S_y A term does not depend on S).
"""
import numpy as np
import pytest

import workloads as wl
from oracle.fv import assemble, WATER_TABLE, NEUMANN0
from oracle.heads import heads
from oracle.jacobian import jacobian


@pytest.mark.parametrize("ndim,face", [(3, 5), (3, 0), (2, 3)])
def test_single_cell_rises_linearly(ndim, face):
    n = (1, 1, 1)
    h = (0.3, 0.5, 0.2) if ndim == 3 else (0.3, 0.5, 1.0)
    S, sy, q = 2e-3, 0.1, 0.7
    bc = [NEUMANN0] * 6
    bc[face] = WATER_TABLE
    area = h[0] * h[1] * h[2] / h[face // 2]
    times = np.array([0.01, 0.3, 2.0])
    phi = heads(n, h, [1.0], [S], [(0.1, 0.2, 0.1)], [(0.2, 0.3, 0.1)], times, 32, q=q,
                bc=tuple(bc), ndim=ndim, sy=sy)
    want = q * times / (S * h[0] * h[1] * h[2] + sy * area)
    np.testing.assert_allclose(phi[0, 0], want, rtol=1e-9)


@pytest.mark.parametrize("ndim", [2, 3])
def test_late_time_rate_is_total_capacity(ndim):
    n = (6, 5, 4) if ndim == 3 else (7, 5, 1)
    h = tuple(1.0 / a for a in n[:ndim]) + (1.0,) * (3 - ndim)
    kap = np.exp(wl.gaussian_random_field(n[:ndim], h[:ndim], (0.3,) * ndim, 0.5, 3)).flatten(order="F")
    S = np.full(kap.size, 1e-5)
    sy = 2e-5
    top = 2 * ndim - 1
    bc = [NEUMANN0] * 6
    bc[top] = WATER_TABLE
    vol = 1.0
    area_top = 1.0          # the unit square's top side or the unit cube's top face
    rate = 1.0 / (1e-5 * vol + sy * area_top)
    t1, t2 = 40 * wl.T_D, 60 * wl.T_D
    src = [(0.3, 0.4, 0.3)]
    rec = [(0.8, 0.2, 0.7), (0.1, 0.9, 0.2)]
    phi = heads(n, h, kap, S, src, rec, [t1, t2], 32, bc=tuple(bc), ndim=ndim, sy=sy)
    slope = (phi[0, :, 1] - phi[0, :, 0]) / (t2 - t1)
    np.testing.assert_allclose(slope, rate, rtol=1e-7)


def test_zero_specific_yield_is_no_flux():
    n = (4, 3, 3)
    h = (0.25, 1 / 3, 1 / 3)
    rng = np.random.default_rng(5)
    kap = np.exp(rng.standard_normal(36))
    S = np.exp(rng.standard_normal(36))
    K1, m1 = assemble(n, h, kap, S, (0, 0, 1, 2, 1, 2), sy=0.0)
    K2, m2 = assemble(n, h, kap, S, (0, 0, 1, 1, 1, 1))
    assert abs(K1 - K2).max() == 0.0
    np.testing.assert_array_equal(m1, m2)


def test_rejects_bad_water_table():
    with pytest.raises(ValueError):
        assemble((3, 3, 1), (1, 1, 1), np.ones(9), np.ones(9), (0, 0, 0, 0, 0, 2))
    with pytest.raises(ValueError):
        assemble((3, 3, 1), (1, 1, 1), np.ones(9), np.ones(9), (0, 0, 0, 2, 0, 0), sy=-1.0)


def test_storage_sensitivity_matches_central_differences():
    n = (4, 3, 3)
    h = (0.25, 1 / 3, 1 / 3)
    kap = np.exp(wl.gaussian_random_field(n, h, (0.3,) * 3, 1.0, 8)).flatten(order="F")
    S = 1e-5 * np.exp(0.3 * np.random.default_rng(8).standard_normal(kap.size))
    bc = (0, 0, 1, 1, 1, 2)
    sy = 5e-6
    src = [(0.5, 0.5, 0.5)]
    rec = [(0.25, 0.3, 0.8), (0.7, 0.75, 0.6)]
    times = wl.T_D * np.array([0.1, 0.6])
    JK, JS = jacobian(n, h, kap, S, src, rec, times, 16, bc=bc, sy=sy)
    eps = 1e-5
    N = kap.size
    for c in range(N):
        d = np.zeros(N)
        d[c] = eps
        fk = (heads(n, h, kap * np.exp(d), S, src, rec, times, 16, bc=bc, sy=sy)
              - heads(n, h, kap * np.exp(-d), S, src, rec, times, 16, bc=bc, sy=sy)) / (2 * eps)
        fs = (heads(n, h, kap, S * np.exp(d), src, rec, times, 16, bc=bc, sy=sy)
              - heads(n, h, kap, S * np.exp(-d), src, rec, times, 16, bc=bc, sy=sy)) / (2 * eps)
        np.testing.assert_allclose(JK[..., c], fk, rtol=0, atol=2e-7 * np.abs(JK).max())
        np.testing.assert_allclose(JS[..., c], fs, rtol=0, atol=2e-7 * np.abs(JS).max())
