"""Pins for the oracle's sensitivities (Section 5.2): central finite
differences of the oracle's own heads in ln(kappa_c) and ln(S_c) (a
different code path: re-assembly and re-solve, no adjoint), reciprocity,
and the mirror symmetry of the constant-field sensitivity map."""
import numpy as np
import pytest

import workloads as wl
from oracle.heads import heads
from oracle.jacobian import jacobian


def _setup(n, seed):
    nd = 3 if n[2] > 1 else 2
    h = tuple(1.0 / a for a in n[:nd]) + (1.0,) * (3 - nd)
    kap = np.exp(wl.gaussian_random_field(n[:nd], h[:nd], (0.3,) * nd, 1.0, seed)).flatten(order="F")
    S = 1e-5 * np.exp(0.3 * np.random.default_rng(seed).standard_normal(kap.size))
    return h, kap, S


@pytest.mark.parametrize("n", [(6, 5, 1), (4, 3, 3)])
def test_jacobian_matches_central_differences(n):
    h, kap, S = _setup(n, 21)
    src = [(0.5, 0.5, 0.5)]
    rec = [(0.25, 0.3, 0.3), (0.7, 0.75, 0.6)]
    times = wl.T_D * np.array([0.1, 0.6])
    JK, JS = jacobian(n, h, kap, S, src, rec, times, 16)
    eps = 1e-5
    N = kap.size
    for c in range(N):
        d = np.zeros(N)
        d[c] = eps
        fk = (heads(n, h, kap * np.exp(d), S, src, rec, times, 16)
              - heads(n, h, kap * np.exp(-d), S, src, rec, times, 16)) / (2 * eps)
        fs = (heads(n, h, kap, S * np.exp(d), src, rec, times, 16)
              - heads(n, h, kap, S * np.exp(-d), src, rec, times, 16)) / (2 * eps)
        sc = np.abs(JK).max()
        np.testing.assert_allclose(JK[..., c], fk, rtol=0, atol=2e-7 * sc)
        np.testing.assert_allclose(JS[..., c], fs, rtol=0, atol=2e-7 * np.abs(JS).max())


def test_jacobian_reciprocity():
    n = (7, 6, 1)
    h, kap, S = _setup(n, 4)
    a, b = (0.3, 0.4, 0.0), (0.7, 0.6, 0.0)
    times = wl.T_D * np.array([0.2])
    J1 = jacobian(n, h, kap, S, [a], [b], times, 16)
    J2 = jacobian(n, h, kap, S, [b], [a], times, 16)
    np.testing.assert_allclose(J1[0], J2[0], rtol=1e-11, atol=1e-14 * np.abs(J1[0]).max())
    np.testing.assert_allclose(J1[1], J2[1], rtol=1e-11, atol=1e-14 * np.abs(J1[1]).max())


def test_constant_field_map_is_mirror_symmetric():
    # The paper's example map (Section 5.2): constant field, source and
    # receiver on one horizontal line.  The map is symmetric about their
    # common line and, with the wells placed symmetrically about the domain
    # centre, about the perpendicular bisector (reciprocity + mirror).
    n = (10, 9, 1)
    h = (0.1, 1 / 9, 1.0)
    kap = np.ones(90)
    S = np.full(90, 1e-5)
    src, rec = (0.65, 0.5, 0.0), (0.35, 0.5, 0.0)
    JK, _ = jacobian(n, h, kap, S, [src], [rec], wl.T_D * np.array([0.3]), 20)
    Jm = JK[0, 0, 0].reshape(9, 10)
    np.testing.assert_allclose(Jm, Jm[::-1, :], rtol=1e-10, atol=1e-13 * np.abs(Jm).max())
    np.testing.assert_allclose(Jm, Jm[:, ::-1], rtol=1e-10, atol=1e-13 * np.abs(Jm).max())
