"""Heads by Crank-Nicolson time stepping of the semi-discrete system.

Oracle (test infrastructure only).

M dphi/dt + K phi = q b for t > 0 with phi(0) = 0 (a constant pumping rate switched on at
t = 0: the semi-discrete system of Section 2.1) stepped with the trapezoidal rule,
(M + dt/2 K) phi_{n+1} = (M - dt/2 K) phi_n + dt q b.  The paper generates its inversion
data this way (Section 5.3) so that the data carry a model error with respect to the
Laplace-transform solution; it is second-order accurate in dt.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from .fv import assemble, point_weights


def crank_nicolson_heads(n, h, kappa, S, sources, receivers, times, dt_max, q=1.0, bc=(0,) * 6, ndim=None):
    """Heads phi[source, receiver, time] with steps of at most dt_max (each interval
    between consecutive times is cut into equal steps)."""
    K, m = assemble(n, h, kappa, S, bc, ndim=ndim)
    B = point_weights(n, h, sources).toarray().T  # [N, ns]
    Br = point_weights(n, h, receivers)
    qs = np.broadcast_to(np.asarray(q, dtype=np.float64), (B.shape[1],))
    rhs = B * qs
    times = np.asarray(times, dtype=np.float64)
    out = np.zeros((B.shape[1], Br.shape[0], times.size))
    phi = np.zeros_like(rhs)
    t_prev = 0.0
    lus = {}
    for it, t in enumerate(times):
        nsteps = max(1, int(np.ceil((t - t_prev) / dt_max)))
        dt = (t - t_prev) / nsteps
        key = round(dt, 15)
        if key not in lus:
            lus[key] = (splu((sp.diags(m) + 0.5 * dt * K).tocsc()), (sp.diags(m) - 0.5 * dt * K).tocsr())
        lu, Bm = lus[key]
        for _ in range(nsteps):
            phi = lu.solve(Bm @ phi + dt * rhs)
        out[:, :, it] = (Br @ phi).T
        t_prev = t
    return out
