"""Pins for the oracle's Talbot contour (eq:talbot, eqn:quadrature, eqn:half)."""
import json
import os

import numpy as np
import pytest

from oracle.contour import talbot_nodes, talbot_full

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "talbot_rate.json")))
RATE = GOLD["rate_base"]


def _inv(F, nz, t):
    z, w = talbot_nodes(nz, t)
    return 2.0 * np.real(np.sum(w * F(z)))


@pytest.mark.parametrize("t", [1e-7, 0.3, 2.0, 50.0])
def test_scalar_transforms_converge_at_the_papers_rate(t):
    a = 0.7 / t
    cases = [(lambda z: 1.0 / z, 1.0),
             (lambda z: 1.0 / (z + a), np.exp(-a * t)),
             (lambda z: 1.0 / z ** 2, t)]
    for nz in (8, 12, 16, 20):
        bound = 10.0 * RATE ** (-nz) + 1e-13 * np.exp(0.171 * nz)
        for F, f in cases:
            scale = t if f == t else 1.0
            err = abs(_inv(F, nz, t) - f) / scale
            # 1/z^2 has a double pole: the same rate with a larger constant
            mult = 300.0 if f == t else 1.0
            assert err <= mult * bound, (nz, err, bound)


def test_rate_is_geometric():
    errs = [abs(_inv(lambda z: 1.0 / z, nz, 1.0) - 1.0) for nz in (8, 12, 16, 20)]
    for e0, e1 in zip(errs[:-1], errs[1:]):
        r = (e0 / e1) ** 0.25
        assert 3.5 < r < 4.3, r


def test_half_sum_equals_full_sum_and_layout():
    for nz in (16, 20, 24):
        z, w = talbot_nodes(nz, 0.5)
        zf, wf = talbot_full(nz, 0.5)
        assert len(z) == nz // 2 and np.all(z.imag > 0)
        # conjugate pairs
        np.testing.assert_allclose(np.sort_complex(zf[zf.imag < 0].conj()), np.sort_complex(z), rtol=1e-15)
        F = lambda s: 1.0 / (s * (s + 3.0))
        np.testing.assert_allclose(np.sum(wf * F(zf)).real, 2.0 * np.real(np.sum(w * F(z))), rtol=1e-13)
        assert abs(np.sum(wf * F(zf)).imag) < 1e-14


def test_nodes_scale_with_nz_over_t():
    z1, w1 = talbot_nodes(20, 1.0)
    z2, w2 = talbot_nodes(20, 4.0)
    np.testing.assert_allclose(z1, 4.0 * z2, rtol=1e-14)
    # the node nearest theta = 0 sits at (N/t) * 0.1709... on the right half plane
    zf, _ = talbot_full(2000, 1.0)
    assert abs(zf[np.argmin(abs(zf.imag))].real / 2000 - (-0.6122 + 0.5017 / 0.6407)) < 1e-5
