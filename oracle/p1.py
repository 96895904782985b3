"""Piecewise-linear (P1) finite elements on a triangulated rectangle (Section 2.1's weak form).

Oracle (test infrastructure only).

The weak form of Section 2.1 with continuous piecewise-linear basis functions phi_i gives
M dphi/dt + K phi = q b with K_ij = sum_e kappa_e int_e grad phi_i . grad phi_j and
b_i = phi_i(x_well).  The mesh here: an nx x ny grid of cells of size hx x hy, each cell
split by its anti-diagonal into two right triangles,

    T1 = (v00, v10, v01)  (right angle at v00),    T2 = (v11, v01, v10)  (right angle at v11),

both with the cell's kappa and S.  Every wall holds zero head, so the unknowns are the
interior vertices (nx - 1) x (ny - 1), x fastest.  The mass matrix is lumped: M_ii =
sum_e S_e |e| / 3 over the triangles that touch vertex i (the paper's consistent mass is
replaced by its row sums, so that M stays diagonal).

Everything below is the element-by-element definition: local gradients of the barycentric
coordinates, local stiffness kappa |e| grad lambda_a . grad lambda_b, local lumped mass,
assembled by index; point values by the barycentric coordinates of the containing triangle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .contour import talbot_nodes
from .heads import _map_shifts


def _triangles(nx, ny, hx, hy):
    """Vertex coordinates [3, 2] and vertex indices (i, j) of every triangle, with its cell."""
    out = []
    for j in range(ny):
        for i in range(nx):
            c = i + nx * j
            v00, v10, v01, v11 = (i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1)
            for tri in ((v00, v10, v01), (v11, v01, v10)):
                xy = np.array([[a * hx, b * hy] for a, b in tri], dtype=np.float64)
                out.append((xy, tri, c))
    return out


def _local(xy):
    """Area and gradients [3, 2] of the barycentric coordinates of a triangle."""
    x, y = xy[:, 0], xy[:, 1]
    det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0])
    area = 0.5 * abs(det)
    # grad lambda_a = (y_b - y_c, x_c - x_b) / det for (a, b, c) cyclic
    g = np.zeros((3, 2))
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        g[a] = [(y[b] - y[c]) / det, (x[c] - x[b]) / det]
    return area, g


def vertex_index(nx, ny):
    """Map (i, j) of a vertex to its unknown's index, or -1 on a wall (zero head)."""
    def idx(v):
        i, j = v
        if i <= 0 or j <= 0 or i >= nx or j >= ny:
            return -1
        return (i - 1) + (nx - 1) * (j - 1)
    return idx


def assemble_p1(n, h, kappa, S):
    """K (sparse) and the lumped mass m over the interior vertices of an n[0] x n[1] cell grid."""
    nx, ny = int(n[0]), int(n[1])
    hx, hy = float(h[0]), float(h[1])
    kappa = np.asarray(kappa, dtype=np.float64).ravel()
    S = np.asarray(S, dtype=np.float64).ravel()
    idx = vertex_index(nx, ny)
    N = (nx - 1) * (ny - 1)
    rows, cols, vals = [], [], []
    m = np.zeros(N)
    for xy, tri, c in _triangles(nx, ny, hx, hy):
        area, g = _local(xy)
        ke = kappa[c] * area * (g @ g.T)
        ids = [idx(v) for v in tri]
        for a in range(3):
            if ids[a] < 0:
                continue
            m[ids[a]] += S[c] * area / 3.0
            for b in range(3):
                if ids[b] < 0:
                    continue
                rows.append(ids[a])
                cols.append(ids[b])
                vals.append(ke[a, b])
    K = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    K.sum_duplicates()
    return K, m


def point_weights_p1(n, h, coords):
    """Sparse [npoints, N]: the P1 basis functions at each point (barycentric coordinates in
    the triangle that contains it; vertices on a wall carry zero head and are dropped)."""
    nx, ny = int(n[0]), int(n[1])
    hx, hy = float(h[0]), float(h[1])
    idx = vertex_index(nx, ny)
    pts = np.asarray(coords, dtype=np.float64).reshape(-1, 3)
    rows, cols, vals = [], [], []
    for p, (x, y, _) in enumerate(pts):
        i = min(max(int(np.floor(x / hx)), 0), nx - 1)
        j = min(max(int(np.floor(y / hy)), 0), ny - 1)
        xi, eta = x / hx - i, y / hy - j
        if xi + eta <= 1.0:
            tri = ((i, j), (i + 1, j), (i, j + 1))
            lam = (1.0 - xi - eta, xi, eta)
        else:
            tri = ((i + 1, j + 1), (i, j + 1), (i + 1, j))
            lam = (xi + eta - 1.0, 1.0 - xi, 1.0 - eta)
        for v, l in zip(tri, lam):
            k = idx(v)
            if k >= 0 and l != 0.0:
                rows.append(p)
                cols.append(k)
                vals.append(l)
    return sp.csr_matrix((vals, (rows, cols)), shape=(pts.shape[0], (nx - 1) * (ny - 1)))


def heads_p1(n, h, kappa, S, sources, receivers, times, nz, q=1.0, workers=1):
    """Heads phi[source, receiver, time] of the P1 discretisation: the contour sum of
    eqn:half over direct solves of (K + z_k M) x = qhat(z_k) b_s, qhat = q / z."""
    K, m = assemble_p1(n, h, kappa, S)
    B = point_weights_p1(n, h, sources)
    Br = point_weights_p1(n, h, receivers)
    ns, nr, nt = B.shape[0], Br.shape[0], len(times)
    qs = np.broadcast_to(np.asarray(q, dtype=np.float64), (ns,))
    rhs = B.T.toarray()
    nodes = [talbot_nodes(nz, t) for t in times]
    shifts = np.concatenate([z for z, _ in nodes])
    gathered = _map_shifts(K, m, rhs, shifts, "gather", Br=Br, workers=workers)
    phi = np.zeros((ns, nr, nt))
    kk = 0
    for it, (z, w) in enumerate(nodes):
        acc = np.zeros((nr, ns), dtype=np.complex128)
        for k in range(len(z)):
            acc += w[k] * (qs / z[k]) * gathered[kk]
            kk += 1
        phi[:, :, it] = 2.0 * acc.real.T
    return phi
