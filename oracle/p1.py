"""Piecewise-linear (P1) finite elements on a subdivided box (Section 2.1's weak form).

Oracle (test infrastructure only).

The weak form of Section 2.1 with continuous piecewise-linear basis functions phi_i gives
M dphi/dt + K phi = q b with K_ij = sum_e kappa_e int_e grad phi_i . grad phi_j and
b_i = phi_i(x_well).  The meshes here subdivide a grid of cells (hx x hy, or hx x hy x hz):

* 2D: each cell split by its anti-diagonal into two right triangles,
  T1 = (v00, v10, v01) (right angle at v00) and T2 = (v11, v01, v10) (right angle at v11);
* 3D: each cell split into the six path tetrahedra of the Kuhn subdivision, one per order
  (a1, a2, a3) of the axes: v000, v000 + e_a1, v000 + e_a1 + e_a2, v111.

Every element takes its cell's kappa and S.  Every wall holds zero head, so the unknowns are
the interior vertices, x fastest.  The mass matrix is lumped: M_ii = sum_e S_e |e| / (d + 1)
over the elements that touch vertex i (the paper's consistent mass replaced by its row sums,
so that M stays diagonal).

Everything below is the element-by-element definition: gradients of the barycentric
coordinates from the inverse of the element's affine map, local stiffness
kappa |e| grad lambda_a . grad lambda_b, local lumped mass, assembled by index; point values
by the barycentric coordinates in an element that contains the point (found by trying the
elements of its cell).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .contour import talbot_nodes
from .heads import _map_shifts


def _dims(n, h):
    n = [int(v) for v in n]
    h = [float(v) for v in h]
    d = 3 if len(n) > 2 and n[2] > 1 else 2
    return d, n[:d], h[:d]


def _cell_elements(idx, d):
    """Vertex index tuples of the elements of the cell with lowest corner idx."""
    import itertools
    if d == 2:
        i, j = idx
        v00, v10, v01, v11 = (i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1)
        return [(v00, v10, v01), (v11, v01, v10)]
    out = []
    for order in itertools.permutations(range(3)):
        v = list(idx)
        path = [tuple(v)]
        for a in order:
            v[a] += 1
            path.append(tuple(v))
        out.append(tuple(path))
    return out


def _elements(n, h):
    """(vertex coordinates [d + 1, d], vertex index tuples, cell) of every element."""
    import itertools
    d, n, h = _dims(n, h)
    out = []
    for idx in itertools.product(*[range(n[a]) for a in reversed(range(d))]):
        idx = tuple(reversed(idx))  # x fastest
        c = 0
        for a in reversed(range(d)):
            c = c * n[a] + idx[a]
        for el in _cell_elements(idx, d):
            xy = np.array([[v[a] * h[a] for a in range(d)] for v in el], dtype=np.float64)
            out.append((xy, el, c))
    return out


def _local(xy):
    """Measure and gradients [d + 1, d] of the barycentric coordinates of a simplex."""
    d = xy.shape[1]
    A = np.hstack([np.ones((d + 1, 1)), xy])  # lambda_i(x) = [1, x] . Ainv[:, i]
    Ainv = np.linalg.inv(A)
    vol = abs(np.linalg.det(xy[1:] - xy[0])) / np.prod(np.arange(1, d + 1))
    return vol, Ainv[1:, :].T


def vertex_index(n, h=None):
    """Map the index tuple of a vertex to its unknown's index, or -1 on a wall (zero head)."""
    n = [int(v) for v in n]
    d = 3 if len(n) > 2 and n[2] > 1 else 2
    n = n[:d]

    def idx(v):
        if any(v[a] <= 0 or v[a] >= n[a] for a in range(d)):
            return -1
        k = 0
        for a in reversed(range(d)):
            k = k * (n[a] - 1) + (v[a] - 1)
        return k
    return idx


def assemble_p1(n, h, kappa, S):
    """K (sparse) and the lumped mass m over the interior vertices of a cell grid n (2D or 3D)."""
    d, nn, hh = _dims(n, h)
    kappa = np.asarray(kappa, dtype=np.float64).ravel()
    S = np.asarray(S, dtype=np.float64).ravel()
    idx = vertex_index(n)
    N = int(np.prod([v - 1 for v in nn]))
    rows, cols, vals = [], [], []
    m = np.zeros(N)
    for xy, el, c in _elements(n, h):
        vol, g = _local(xy)
        ke = kappa[c] * vol * (g @ g.T)
        ids = [idx(v) for v in el]
        for a in range(d + 1):
            if ids[a] < 0:
                continue
            m[ids[a]] += S[c] * vol / (d + 1)
            for b in range(d + 1):
                if ids[b] < 0:
                    continue
                rows.append(ids[a])
                cols.append(ids[b])
                vals.append(ke[a, b])
    K = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    K.sum_duplicates()
    return K, m


def point_weights_p1(n, h, coords):
    """Sparse [npoints, N]: the P1 basis functions at each point (barycentric coordinates in an
    element of its cell that contains it; vertices on a wall carry zero head and are dropped)."""
    d, nn, hh = _dims(n, h)
    idx = vertex_index(n)
    pts = np.asarray(coords, dtype=np.float64).reshape(-1, 3)
    rows, cols, vals = [], [], []
    for p, x in enumerate(pts):
        cell = tuple(min(max(int(np.floor(x[a] / hh[a])), 0), nn[a] - 1) for a in range(d))
        for el in _cell_elements(cell, d):
            xy = np.array([[v[a] * hh[a] for a in range(d)] for v in el], dtype=np.float64)
            A = np.hstack([np.ones((d + 1, 1)), xy])
            lam = np.linalg.solve(A.T, np.concatenate([[1.0], x[:d]]))
            if lam.min() >= -1e-12:
                break
        for v, l in zip(el, lam):
            k = idx(v)
            if k >= 0 and abs(l) > 1e-14:
                rows.append(p)
                cols.append(k)
                vals.append(l)
    N = int(np.prod([v - 1 for v in nn]))
    return sp.csr_matrix((vals, (rows, cols)), shape=(pts.shape[0], N))


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


def jacobian_p1(n, h, kappa, S, sources, receivers, times, nz, q=1.0, workers=1):
    """Sensitivities d phi[s, r, t] / d ln kappa_c and / d ln S_c of the P1 heads, for every cell c,
    by the discrete adjoint (Section 5.2): with phi_sk = (K + z_k M)^{-1} qhat_k b_s and
    psi_rk = (K + z_k M)^{-T} B_r^T,

        d phi / d p_c = -2 Re sum_k w_k psi_rk^T (dK/dp_c + z_k dM/dp_c) phi_sk,

    where dK/d ln kappa_c = kappa_c sum_{e in c} K_e(kappa = 1) and dM/d ln S_c =
    S_c sum_{e in c} (|e| / (d + 1)) at the element's vertices (element by element, as in
    assemble_p1).  Returns (JK, JS), each [ns, nr, nt, ncells]."""
    d, nn, hh = _dims(n, h)
    kappa = np.asarray(kappa, dtype=np.float64).ravel()
    S = np.asarray(S, dtype=np.float64).ravel()
    K, m = assemble_p1(n, h, kappa, S)
    B = point_weights_p1(n, h, sources)
    Br = point_weights_p1(n, h, receivers)
    idx = vertex_index(n)
    ns, nr, nt = B.shape[0], Br.shape[0], len(times)
    ncells = int(np.prod(nn))
    qs = np.broadcast_to(np.asarray(q, dtype=np.float64), (ns,))
    nodes = [talbot_nodes(nz, t) for t in times]
    shifts = np.concatenate([z for z, _ in nodes])
    # forward fields (columns: sources) and adjoint fields (columns: receivers); K and M are
    # symmetric, so the adjoint solve uses the same matrix
    rhs = np.hstack([B.T.toarray(), Br.T.toarray()])
    X = _map_shifts(K, m, rhs, shifts, "full", workers=workers)
    elems = _elements(n, h)
    JK = np.zeros((ns, nr, nt, ncells))
    JS = np.zeros((ns, nr, nt, ncells))
    kk = 0
    for it, (z, w) in enumerate(nodes):
        for k in range(len(z)):
            Xk = X[kk]
            kk += 1
            phi = Xk[:, :ns] * (qs / z[k])[None, :]
            psi = Xk[:, ns:]
            for xy, el, c in elems:
                vol, g = _local(xy)
                ids = [idx(v) for v in el]
                # element vectors, zero at wall vertices
                pe = np.array([phi[i] if i >= 0 else np.zeros(ns) for i in ids])  # [d+1, ns]
                qe = np.array([psi[i] if i >= 0 else np.zeros(nr) for i in ids])  # [d+1, nr]
                ke = kappa[c] * vol * (g @ g.T)
                dK = qe.T @ ke @ pe  # [nr, ns]
                dM = S[c] * vol / (d + 1) * (qe.T @ pe)
                JK[:, :, it, c] += -2.0 * (w[k] * dK).real.T
                JS[:, :, it, c] += -2.0 * (w[k] * z[k] * dM).real.T
    return JK, JS
