"""Cell-centred finite-volume discretisation of the groundwater equation.

Oracle (test infrastructure only; see the package docstring).

The paper discretises S_s d(phi)/dt - div(kappa grad phi) = q(t) delta(x - x_s)
(eqn:timedomain) with P1 finite elements into M phi' + K phi = q(t) b
(Section 2.1).  Here the same semi-discrete form comes from a cell-centred
finite-volume scheme on a regular grid:

* interior face between cells i, j along axis a:
  T = 2 k_i k_j / (k_i + k_j) * A_a / h_a   (harmonic mean of kappa),
* zero-Dirichlet boundary face: the boundary value sits h_a/2 from the cell
  centre, T_b = 2 k_i A_a / h_a; a zero-Neumann face carries no flux,
* (K phi)_i = sum_faces T (phi_i - phi_j) + sum_boundary T_b phi_i,
* lumped storage M = diag(S_i V_i),
* a linearised water-table face (eqn:timedomain, third condition; the
  boundary term of M_ij in Section 2.1) carries no conductive flux; its
  storage S_y d(phi)/dt over the face area A_a is lumped on the cell behind
  it, with the face head taken as that cell's head: M_ii += S_y A_a,
* a point source or receiver at x has bilinear (trilinear) weights on the
  cell centres around it, clamped to the nearest cell within h/2 of a wall.

Cells are numbered with x fastest: (ix, iy, iz) -> ix + nx (iy + ny iz).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

DIRICHLET0 = 0
NEUMANN0 = 1
WATER_TABLE = 2


def _index(n):
    nx, ny, nz = n
    return np.arange(nx * ny * nz).reshape((nz, ny, nx))


def _ndim(n):
    return 3 if n[2] > 1 else (2 if n[1] > 1 else 1)


def assemble(n, h, kappa, S, bc=(0, 0, 0, 0, 0, 0), ndim=None, sy=0.0):
    """Return (K as CSR, m) with K the stiffness and m the lumped mass diagonal.

    Axes at or beyond ``ndim`` are flat (one cell, no walls); by default a
    grid with nz == 1 is 2D.  ``sy`` is the specific yield of every face
    marked WATER_TABLE; such a face must lie on one of the ``ndim`` axes.
    """
    n = tuple(int(a) for a in n)
    if ndim is None:
        ndim = _ndim(n)
    h = tuple(float(a) for a in h)
    sy = float(sy)
    if not (sy >= 0.0 and np.isfinite(sy)):
        raise ValueError("specific yield must be finite and >= 0")
    for face in range(6):
        if bc[face] not in (DIRICHLET0, NEUMANN0, WATER_TABLE):
            raise ValueError("unknown boundary condition")
        if bc[face] == WATER_TABLE and face // 2 >= ndim:
            raise ValueError("a water-table face must lie on a grid axis")
    N = n[0] * n[1] * n[2]
    kap = np.asarray(kappa, dtype=np.float64).reshape((n[2], n[1], n[0]))
    idx = _index(n)
    V = h[0] * h[1] * h[2]
    rows, cols, vals = [], [], []
    diag = np.zeros((n[2], n[1], n[0]))
    wt = np.zeros((n[2], n[1], n[0]))   # water-table storage S_y A per cell
    # storage axis of each grid axis in the (z, y, x) array
    for a in range(ndim):
        ax = 2 - a
        area = V / h[a]
        if n[a] > 1:
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax] = slice(0, n[a] - 1)
            hi[ax] = slice(1, n[a])
            ki, kj = kap[tuple(lo)], kap[tuple(hi)]
            T = 2.0 * ki * kj / (ki + kj) * area / h[a]
            ii, jj = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
            rows += [ii, jj]
            cols += [jj, ii]
            vals += [-T.ravel(), -T.ravel()]
            diag[tuple(lo)] += T
            diag[tuple(hi)] += T
        # boundary faces on the low and high side of this axis
        for side, face in ((0, 2 * a), (n[a] - 1, 2 * a + 1)):
            sl = [slice(None)] * 3
            sl[ax] = slice(side, side + 1)
            if bc[face] == WATER_TABLE:
                wt[tuple(sl)] += sy * area
            if bc[face] != DIRICHLET0:
                continue
            diag[tuple(sl)] += 2.0 * kap[tuple(sl)] * area / h[a]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    K.sum_duplicates()
    m = storage_mass(n, h, S) + wt.ravel()
    return K, m


def storage_mass(n, h, S):
    """The part S_i V_i of the lumped mass that the storage coefficient owns."""
    V = float(h[0]) * float(h[1]) * float(h[2])
    return np.asarray(S, dtype=np.float64).reshape(-1) * V


def _axis_weights(x, h, n):
    u = x / h - 0.5
    i0 = int(np.floor(u))
    f = u - i0
    if i0 < 0:
        return [(0, 1.0)]
    if i0 >= n - 1:
        return [(n - 1, 1.0)]
    out = [(i0, 1.0 - f)]
    if f > 0.0:
        out.append((i0 + 1, f))
    return out


def point_weights(n, h, coords):
    """Sparse [npts, N] matrix of cell-centre interpolation weights."""
    n = tuple(int(a) for a in n)
    N = n[0] * n[1] * n[2]
    coords = np.atleast_2d(np.asarray(coords, dtype=np.float64))
    r, c, v = [], [], []
    for p, x in enumerate(coords):
        wx = _axis_weights(x[0], h[0], n[0])
        wy = _axis_weights(x[1], h[1], n[1]) if n[1] > 1 else [(0, 1.0)]
        wz = _axis_weights(x[2], h[2], n[2]) if n[2] > 1 else [(0, 1.0)]
        for iz, fz in wz:
            for iy, fy in wy:
                for ix, fx in wx:
                    w = fx * fy * fz
                    if w != 0.0:
                        r.append(p)
                        c.append(ix + n[0] * (iy + n[1] * iz))
                        v.append(w)
    return sp.csr_matrix((v, (r, c)), shape=(len(coords), N))
