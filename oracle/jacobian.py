"""Sensitivities of receiver heads to ln(kappa) and ln(S) per cell.

Oracle (test infrastructure only).

Section 5.2 derives the sensitivity through the Laplace transform with an
adjoint field driven by a point sink at the receiver, then discretises the
contour integral with the same weights.  Its printed integrand is garbled
in places (a gradient on the storage term, a dropped z_k in the discrete
sum), so this oracle differentiates the discrete heads instead
(discretise-then-differentiate), which is what the continuous derivation
reduces to on the FV operator:

    d_hat(z) = B_m (K + z M)^{-1} b_s,   psi = (K + z M)^{-1} B_m^T
    (K + z M is complex symmetric, so no conjugation),
    d d_hat / d p = - psi^T (dK/dp + z dM/dp) phi_hat,
    J[s, m, t, :] = 2 Re sum_k w_k(t) qhat(z_k) d d_hat_k / d p.

With T_f = 2 A k_i k_j / (h (k_i + k_j)):  dT_f / d ln k_i = T_f k_j / (k_i + k_j);
a Dirichlet wall face T_b = 2 k_i A / h gives dT_b / d ln k_i = T_b;
dm_c / d ln S_c = S_c V_c (a water-table face's S_y A storage does not
depend on S, so it stays out of this derivative).
"""
from __future__ import annotations

import numpy as np

from .fv import assemble, point_weights, storage_mass, _ndim
from .contour import talbot_nodes
from .heads import shifted_fields


def _face_lists(n, h, kappa, bc, ndim):
    nx, ny, nz = n
    kap = np.asarray(kappa).reshape((nz, ny, nx))
    idx = np.arange(nx * ny * nz).reshape((nz, ny, nx))
    V = h[0] * h[1] * h[2]
    faces = []   # (i, j, T, dT/dln k_i, dT/dln k_j)
    walls = []   # (i, T_b)
    for a in range(ndim):
        ax = 2 - a
        area = V / h[a]
        if n[a] > 1:
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax] = slice(0, n[a] - 1)
            hi[ax] = slice(1, n[a])
            ki, kj = kap[tuple(lo)].ravel(), kap[tuple(hi)].ravel()
            T = 2.0 * ki * kj / (ki + kj) * area / h[a]
            faces.append((idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel(), T,
                          T * kj / (ki + kj), T * ki / (ki + kj)))
        for side, face in ((0, 2 * a), (n[a] - 1, 2 * a + 1)):
            if bc[face] != 0:
                continue
            sl = [slice(None)] * 3
            sl[ax] = slice(side, side + 1)
            walls.append((idx[tuple(sl)].ravel(), 2.0 * kap[tuple(sl)].ravel() * area / h[a]))
    return faces, walls


def jacobian(n, h, kappa, S, sources, receivers, times, nz, q=1.0, bc=(0,) * 6,
             workers=1, ndim=None, sy=0.0):
    """Return (J_lnK, J_lnS), each [ns, nr, nt, N] float64; ``q`` is one rate for every
    source or one per source."""
    n = tuple(int(a) for a in n)
    if ndim is None:
        ndim = _ndim(n)
    K, m = assemble(n, h, kappa, S, bc, ndim=ndim, sy=sy)
    mS = storage_mass(n, h, S)
    Bs = point_weights(n, h, sources)
    Br = point_weights(n, h, receivers)
    N = K.shape[0]
    ns, nr, nt = Bs.shape[0], Br.shape[0], len(times)
    qs = np.broadcast_to(np.asarray(q, dtype=np.float64), (ns,))
    faces, walls = _face_lists(n, h, kappa, bc, ndim)
    rhs = np.hstack([Bs.T.toarray(), Br.T.toarray()])
    nodes = [talbot_nodes(nz, t) for t in times]
    shifts = np.concatenate([z for z, _ in nodes])
    X = shifted_fields(K, m, rhs, shifts, workers=workers)
    JK = np.zeros((ns, nr, nt, N))
    JS = np.zeros((ns, nr, nt, N))
    kk = 0
    for it, (z, w) in enumerate(nodes):
        accK = np.zeros((ns, nr, N), dtype=np.complex128)
        accS = np.zeros((ns, nr, N), dtype=np.complex128)
        for k in range(len(z)):
            phi = X[kk][:, :ns]          # [N, ns]
            psi = X[kk][:, ns:]          # [N, nr]
            kk += 1
            c = (w[k] / z[k]) * qs[:, None, None]
            # psi^T (dK/dln k_c) phi, accumulated per cell c
            gK = np.zeros((ns, nr, N), dtype=np.complex128)
            for (i, j, T, dTi, dTj) in faces:
                prod = np.einsum("fs,fr->srf", phi[i] - phi[j], psi[i] - psi[j])
                np.add.at(gK, (slice(None), slice(None), i), dTi * prod)
                np.add.at(gK, (slice(None), slice(None), j), dTj * prod)
            for (i, Tb) in walls:
                prod = np.einsum("fs,fr->srf", phi[i], psi[i])
                np.add.at(gK, (slice(None), slice(None), i), Tb * prod)
            gS = z[k] * mS[None, None, :] * np.einsum("cs,cr->src", phi, psi)
            accK -= c * gK
            accS -= c * gS
        JK[:, :, it, :] = 2.0 * accK.real
        JS[:, :, it, :] = 2.0 * accS.real
    return JK, JS
