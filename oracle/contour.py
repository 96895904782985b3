"""Optimised Talbot contour and its trapezoid (midpoint) weights.

Oracle (test infrastructure only).

Section 2.2 (eq:talbot) inverts the Laplace transform on a modified Talbot
contour whose parameters are the optimised ones of Trefethen, Weideman and
Schmelzer (2006), scale with N_z / t, and give the error O(3.89^-N_z)
(Section 2.3).  That optimised contour is

    z(theta) = (N/t) * (-0.6122 + 0.5017 theta cot(0.6407 theta) + 0.2645 i theta),

for theta in (-pi, pi).  The trapezoid rule with spacing 2 pi / N
(eqn:quadrature) is taken at midpoints theta_k = -pi + (k - 1/2) 2 pi / N,
k = 1..N, so no node lies at theta = 0 or +-pi and the N nodes form N/2
conjugate pairs.  Approximating (1 / 2 pi i) int e^{zt} F(z) z'(theta) dtheta
gives the weights w_k = -(i / N) e^{z_k t} z'(theta_k) with

    f(t) ~= sum_{k=1..N} w_k F(z_k) = 2 Re sum_{Im z_k > 0} w_k F(z_k)

(eqn:half) when F(conj z) = conj F(z), as for the real symmetric pencil
(K, M).  The weight carries 1/N, not 1/(2N), because the half sum is
doubled by 2 Re.
"""
from __future__ import annotations

import numpy as np

_A0 = -0.6122
_A1 = 0.5017
_ALPHA = 0.6407
_NU = 0.2645


def _z_and_dz(theta, scale):
    at = _ALPHA * theta
    cot = np.cos(at) / np.sin(at)
    z = scale * (_A0 + _A1 * theta * cot + 1j * _NU * theta)
    dz = scale * (_A1 * (cot - at / np.sin(at) ** 2) + 1j * _NU)
    return z, dz


def talbot_full(nz, t):
    """All nz nodes and weights for time t (nz even)."""
    if nz % 2:
        raise ValueError("nz must be even")
    k = np.arange(1, nz + 1)
    theta = -np.pi + (k - 0.5) * 2.0 * np.pi / nz
    z, dz = _z_and_dz(theta, nz / t)
    w = -1j / nz * np.exp(z * t) * dz
    return z, w


def talbot_nodes(nz, t):
    """The nz/2 nodes with Im z > 0 and their weights; f ~ 2 Re sum w F(z)."""
    z, w = talbot_full(nz, t)
    keep = z.imag > 0
    return z[keep], w[keep]
