"""The quasi-linear geostatistical inversion (Section 5.1, Algorithm 2).

Oracle (test infrastructure only).

The unknowns are s = ln kappa per cell with the prior s ~ N(X beta, Q): X is a column of
ones (one unknown constant mean, the paper's X = [1, ..., 1]^T) and Q the exponential
covariance Q_ij = var exp(-|(x_i - x_j) / ell|) over the cell centres (the kernel of the
paper's rough field, per-axis lengths ell).  The measurements are y = h(s) + eps with
eps ~ N(0, r I): heads at the observation wells and times, ordered (well, receiver, time)
as heads() returns them.

One Gauss-Newton step at s_k: J = dh/ds at s_k (the adjoint sensitivities of
jacobian.py: d phi / d ln kappa), then the saddle-point system of eq:inversion1,

    [ J Q J^T + R   J X ] [ xi   ]   [ y - h(s_k) + J s_k ]
    [ (J X)^T       0   ] [ beta ] = [ 0                  ],

and s_{k+1} = X beta + Q J^T xi.  Q is formed densely here (its plain definition); the
paper's FFT and hierarchical-matrix products are faster ways of forming Q J^T.
"""
from __future__ import annotations

import numpy as np

from .heads import heads
from .jacobian import jacobian


def cell_centres(n, h, ndim):
    """Cell-centre coordinates [N, ndim], x fastest (the grid's storage order)."""
    n = tuple(int(a) for a in n)
    axes = [(np.arange(n[a]) + 0.5) * h[a] for a in range(ndim)]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel(order="F") for g in grids], axis=1)


def exp_covariance(n, h, var, ell, ndim):
    """Dense Q_ij = var exp(-|(x_i - x_j) / ell|) over the cell centres."""
    x = cell_centres(n, h, ndim) / np.asarray(ell[:ndim], dtype=np.float64)
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(axis=2))
    return var * np.exp(-d)


def saddle_update(J, hs, y, s, QJt, r):
    """s_{k+1}, xi, beta of eq:inversion1 from J [M, N], h(s_k) [M], y [M], s_k [N],
    Q J^T [N, M] and the error variance r (R = r I)."""
    M = J.shape[0]
    JX = J.sum(axis=1)  # J X with X a column of ones
    A = np.zeros((M + 1, M + 1))
    A[:M, :M] = J @ QJt + r * np.eye(M)
    A[:M, M] = JX
    A[M, :M] = JX
    rhs = np.zeros(M + 1)
    rhs[:M] = y - hs + J @ s
    sol = np.linalg.solve(A, rhs)
    xi, beta = sol[:M], sol[M]
    return beta + QJt @ xi, xi, beta


def measure(n, h, s, S, sources, receivers, times, nz, q=1.0, bc=(0,) * 6, ndim=None, workers=1):
    """h(s) [M] and J = dh/ds [M, N] at s = ln kappa (direct solves per shift)."""
    kappa = np.exp(np.asarray(s, dtype=np.float64))
    phi = heads(n, h, kappa, S, sources, receivers, times, nz, q=q, bc=bc, ndim=ndim, workers=workers)
    JK, _ = jacobian(n, h, kappa, S, sources, receivers, times, nz, q=q, bc=bc, workers=workers, ndim=ndim)
    return phi.ravel(), JK.reshape(-1, JK.shape[-1])


def gauss_newton_step(n, h, s, S, sources, receivers, times, nz, y, var, ell, r, q=1.0, bc=(0,) * 6,
                      ndim=None, Q=None, workers=1):
    """One step of Algorithm 2 from s = ln kappa; returns a dict with s_next, hs, J, xi, beta."""
    nd = ndim if ndim is not None else (3 if n[2] > 1 else 2)
    hs, J = measure(n, h, s, S, sources, receivers, times, nz, q=q, bc=bc, ndim=nd, workers=workers)
    if Q is None:
        Q = exp_covariance(n, h, var, ell, nd)
    QJt = Q @ J.T
    s_next, xi, beta = saddle_update(J, hs, np.asarray(y, dtype=np.float64), np.asarray(s, dtype=np.float64),
                                     QJt, r)
    return {"s_next": s_next, "hs": hs, "J": J, "xi": xi, "beta": beta}
