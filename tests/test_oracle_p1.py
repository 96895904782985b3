"""Pins of the oracle's P1 finite elements (Section 2.1's weak form on a triangulated
rectangle, lumped mass), each against something other than the oracle:

* constant kappa: the stiffness matrix against the five-point difference Laplacian built
  from Kronecker products (hx hy times it; the right triangles' hypotenuse couplings vanish);
* variable kappa: no coupling between the two ends of a cell's diagonal, each axis coupling
  the mean of the two cells beside the edge times hy/hx (or hx/hy), rows of the wall-free
  matrix summing to zero;
* the lumped mass against S times the area each interior vertex owns (hx hy);
* the point weights reproduce linear functions exactly;
* the heads of a sine eigenmode initial-value problem against exp(-lambda t), lambda from
  the closed-form eigenvalue of the five-point Laplacian with lumped mass;
* 3D (the Kuhn subdivision into six path tetrahedra per cell): the seven-point Laplacian for
  constant kappa, no coupling off the axes for variable kappa with each edge's weight and each
  vertex's mass against their closed forms (the GPU assembles those), linear interpolation,
  and the closed-form eigenvalue of a sine mode.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.contour import talbot_nodes
from oracle.heads import _map_shifts
from oracle.p1 import assemble_p1, heads_p1, point_weights_p1, vertex_index


def _lap1d(n, h):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]) / h ** 2


def test_constant_kappa_is_the_five_point_laplacian():
    nx, ny, hx, hy, kap = 7, 5, 0.3, 0.2, 2.5
    K, m = assemble_p1((nx, ny), (hx, hy), np.full(nx * ny, kap), np.full(nx * ny, 1e-3))
    Ix, Iy = sp.identity(nx - 1), sp.identity(ny - 1)
    L = sp.kron(Iy, _lap1d(nx - 1, hx)) + sp.kron(_lap1d(ny - 1, hy), Ix)
    assert abs(K - kap * hx * hy * L).max() <= 1e-12 * kap * (hy / hx + hx / hy)
    assert np.allclose(m, 1e-3 * hx * hy, rtol=1e-14)


def test_variable_kappa_couplings():
    nx, ny, hx, hy = 6, 5, 0.25, 0.4
    rng = np.random.default_rng(4)
    kap = np.exp(rng.standard_normal(nx * ny))
    S = np.exp(rng.standard_normal(nx * ny))
    K, m = assemble_p1((nx, ny), (hx, hy), kap, S)
    idx = vertex_index((nx, ny))
    kc = kap.reshape(ny, nx)  # [j][i]
    Sc = S.reshape(ny, nx)
    for J in range(1, ny):
        for I in range(1, nx):
            a = idx((I, J))
            if I + 1 < nx:  # +x edge: cells (I, J-1) and (I, J)
                assert K[a, idx((I + 1, J))] == pytest.approx(-(hy / hx) * 0.5 * (kc[J - 1, I] + kc[J, I]), rel=1e-13)
            if J + 1 < ny:  # +y edge: cells (I-1, J) and (I, J)
                assert K[a, idx((I, J + 1))] == pytest.approx(-(hx / hy) * 0.5 * (kc[J, I - 1] + kc[J, I]), rel=1e-13)
            if I + 1 < nx and J > 1:  # the ends of cell (I, J-1)'s anti-diagonal: (I+1, J-1) and (I, J)
                assert abs(K[a, idx((I + 1, J - 1))]) <= 1e-14 * abs(K).max()
            # six triangles: one of cell (I, J), two of (I-1, J), two of (I, J-1), one of (I-1, J-1)
            want = hx * hy / 6 * (Sc[J, I] + 2 * Sc[J, I - 1] + 2 * Sc[J - 1, I] + Sc[J - 1, I - 1])
            assert m[a] == pytest.approx(want, rel=1e-13)
    # interior rows away from the walls sum to zero (constants lie in the kernel)
    r = np.asarray(K.sum(axis=1)).ravel()
    inner = [idx((I, J)) for J in range(2, ny - 1) for I in range(2, nx - 1)]
    assert np.abs(r[inner]).max() <= 1e-13 * abs(K).max()


def test_point_weights_reproduce_linear_functions():
    nx, ny, hx, hy = 8, 6, 0.125, 1 / 6
    rng = np.random.default_rng(2)
    idx = vertex_index((nx, ny))
    xv = np.zeros((nx - 1) * (ny - 1))
    yv = np.zeros_like(xv)
    for J in range(1, ny):
        for I in range(1, nx):
            xv[idx((I, J))] = I * hx
            yv[idx((I, J))] = J * hy
    # points whose triangles have only interior vertices (cells 1..nx-2 x 1..ny-2)
    pts = np.column_stack([rng.uniform(hx, (nx - 1) * hx, 50), rng.uniform(hy, (ny - 1) * hy, 50), np.zeros(50)])
    W = point_weights_p1((nx, ny), (hx, hy), pts)
    f = 0.7 + 2.0 * xv - 1.3 * yv
    assert np.abs(W @ f - (0.7 + 2.0 * pts[:, 0] - 1.3 * pts[:, 1])).max() <= 1e-13
    assert np.allclose(np.asarray(W.sum(axis=1)).ravel(), 1.0, rtol=1e-14)


def test_eigenmode_decays_at_its_closed_form_rate():
    nx, ny = 16, 12
    hx, hy = 1 / nx, 1 / ny
    kap, Sv = 1.0, 1e-3
    K, m = assemble_p1((nx, ny), (hx, hy), np.full(nx * ny, kap), np.full(nx * ny, Sv))
    idx = vertex_index((nx, ny))
    v = np.zeros((nx - 1) * (ny - 1))
    for J in range(1, ny):
        for I in range(1, nx):
            v[idx((I, J))] = np.sin(np.pi * I * hx) * np.sin(np.pi * J * hy)
    lam = kap / Sv * (4 / hx ** 2 * np.sin(np.pi * hx / 2) ** 2 + 4 / hy ** 2 * np.sin(np.pi * hy / 2) ** 2)
    assert np.linalg.norm(K @ v - lam * m * v) <= 1e-10 * np.linalg.norm(K @ v)
    # phi(t) = exp(-lam t) v: the contour sum of (K + z M)^{-1} M v over the Talbot nodes
    t = 3.0 / lam
    z, w = talbot_nodes(40, t)
    X = _map_shifts(K, m, (m * v).reshape(-1, 1), z, "full")
    phi = 2.0 * sum(wk * x[:, 0] for wk, x in zip(w, X)).real
    assert np.abs(phi - np.exp(-lam * t) * v).max() <= 1e-12


def test_heads_are_the_contour_sum_of_direct_solves():
    # one well, constant rate: phi(t) against the eigen-expansion of the P1 system (dense)
    nx, ny = 10, 8
    hx, hy = 1 / nx, 1 / ny
    rng = np.random.default_rng(9)
    kap = np.exp(0.5 * rng.standard_normal(nx * ny))
    Sv = np.full(nx * ny, 1e-3)
    src = np.array([[0.43, 0.37, 0.0]])
    rec = np.array([[0.61, 0.52, 0.0], [0.2, 0.7, 0.0]])
    times = [0.05, 0.4]
    ph = heads_p1((nx, ny), (hx, hy), kap, Sv, src, rec, times, 40)
    K, m = assemble_p1((nx, ny), (hx, hy), kap, Sv)
    b = point_weights_p1((nx, ny), (hx, hy), src).toarray().ravel()
    Br = point_weights_p1((nx, ny), (hx, hy), rec).toarray()
    # M^{-1/2} K M^{-1/2} = Q diag(l) Q^T; phi(t) = M^{-1/2} Q diag((1 - e^{-l t}) / l) Q^T M^{-1/2} b
    s = 1 / np.sqrt(m)
    l, Q = np.linalg.eigh((s[:, None] * K.toarray()) * s[None, :])
    for it, t in enumerate(times):
        x = s * (Q @ (((1 - np.exp(-l * t)) / l) * (Q.T @ (s * b))))
        assert np.abs(ph[0, :, it] - Br @ x).max() <= 1e-9 * np.abs(Br @ x).max()


def test_3d_constant_kappa_is_the_seven_point_laplacian():
    n, h, kap = (6, 5, 4), (0.3, 0.2, 0.25), 1.7
    N3 = n[0] * n[1] * n[2]
    K, m = assemble_p1(n, h, np.full(N3, kap), np.full(N3, 2e-3))
    I = [sp.identity(v - 1) for v in n]
    L = (sp.kron(I[2], sp.kron(I[1], _lap1d(n[0] - 1, h[0]))) + sp.kron(I[2], sp.kron(_lap1d(n[1] - 1, h[1]), I[0]))
         + sp.kron(_lap1d(n[2] - 1, h[2]), sp.kron(I[1], I[0])))
    V = h[0] * h[1] * h[2]
    assert abs(K - kap * V * L).max() <= 1e-12 * abs(K).max()
    assert np.allclose(m, 2e-3 * V, rtol=1e-13)


def test_3d_variable_kappa_couples_axis_neighbours_only():
    """The Kuhn subdivision's path tetrahedra couple no vertex pair off the axes, for any kappa
    per cell.  An x edge lies in six tetrahedra of the four cells around it: two of the cell
    below-behind it in y and z, two of the cell beyond it in both, one of each other cell; each
    adds kappa hy hz / (6 hx).  A vertex lies in all six tetrahedra of the cells it is the
    lowest or highest corner of, and in two of each of its other six cells."""
    n, h = (5, 4, 4), (0.25, 0.3, 0.2)
    rng = np.random.default_rng(11)
    N3 = n[0] * n[1] * n[2]
    kap = np.exp(rng.standard_normal(N3))
    S = np.exp(rng.standard_normal(N3))
    K, m = assemble_p1(n, h, kap, S)
    idx = vertex_index(n)
    kc = kap.reshape(n[2], n[1], n[0])  # [k][j][i]
    Sc = S.reshape(n[2], n[1], n[0])
    Kd = K.toarray()
    hx, hy, hz = h
    for Kk in range(1, n[2]):
        for J in range(1, n[1]):
            for I in range(1, n[0]):
                a = idx((I, J, Kk))
                nbrs = {idx((I + di, J + dj, Kk + dk)) for di, dj, dk in
                        ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))}
                # zero up to the rounding of the element inverses
                off = [b for b in np.nonzero(np.abs(Kd[a]) > 1e-13 * np.abs(Kd).max())[0] if b != a]
                assert set(off) <= nbrs
                if I + 1 < n[0]:
                    want = hy * hz / hx * (2 * kc[Kk - 1, J - 1, I] + 2 * kc[Kk, J, I] + kc[Kk, J - 1, I]
                                           + kc[Kk - 1, J, I]) / 6
                    assert Kd[a, idx((I + 1, J, Kk))] == pytest.approx(-want, rel=1e-12)
                if J + 1 < n[1]:
                    want = hx * hz / hy * (2 * kc[Kk - 1, J, I - 1] + 2 * kc[Kk, J, I] + kc[Kk, J, I - 1]
                                           + kc[Kk - 1, J, I]) / 6
                    assert Kd[a, idx((I, J + 1, Kk))] == pytest.approx(-want, rel=1e-12)
                if Kk + 1 < n[2]:
                    want = hx * hy / hz * (2 * kc[Kk, J - 1, I - 1] + 2 * kc[Kk, J, I] + kc[Kk, J, I - 1]
                                           + kc[Kk, J - 1, I]) / 6
                    assert Kd[a, idx((I, J, Kk + 1))] == pytest.approx(-want, rel=1e-12)
                six = Sc[Kk, J, I] + Sc[Kk - 1, J - 1, I - 1]
                two = (Sc[Kk, J, I - 1] + Sc[Kk, J - 1, I] + Sc[Kk - 1, J, I] + Sc[Kk, J - 1, I - 1]
                       + Sc[Kk - 1, J, I - 1] + Sc[Kk - 1, J - 1, I])
                assert m[a] == pytest.approx(hx * hy * hz / 24 * (6 * six + 2 * two), rel=1e-12)


def test_3d_point_weights_reproduce_linear_functions():
    n, h = (6, 5, 4), (1 / 6, 0.2, 0.25)
    rng = np.random.default_rng(3)
    idx = vertex_index(n)
    N = (n[0] - 1) * (n[1] - 1) * (n[2] - 1)
    X = np.zeros((N, 3))
    for Kk in range(1, n[2]):
        for J in range(1, n[1]):
            for I in range(1, n[0]):
                X[idx((I, J, Kk))] = [I * h[0], J * h[1], Kk * h[2]]
    pts = np.column_stack([rng.uniform(h[a], (n[a] - 1) * h[a], 40) for a in range(3)])
    W = point_weights_p1(n, h, pts)
    f = 0.3 + X @ np.array([1.5, -0.7, 2.2])
    assert np.abs(W @ f - (0.3 + pts @ np.array([1.5, -0.7, 2.2]))).max() <= 1e-12


def test_3d_eigenmode_decays_at_its_closed_form_rate():
    n = (10, 8, 6)
    h = tuple(1.0 / v for v in n)
    kap, Sv = 1.0, 1e-3
    N3 = n[0] * n[1] * n[2]
    K, m = assemble_p1(n, h, np.full(N3, kap), np.full(N3, Sv))
    idx = vertex_index(n)
    v = np.zeros(K.shape[0])
    for Kk in range(1, n[2]):
        for J in range(1, n[1]):
            for I in range(1, n[0]):
                v[idx((I, J, Kk))] = np.sin(np.pi * I * h[0]) * np.sin(np.pi * J * h[1]) * np.sin(np.pi * Kk * h[2])
    lam = kap / Sv * sum(4 / ha ** 2 * np.sin(np.pi * ha / 2) ** 2 for ha in h)
    assert np.linalg.norm(K @ v - lam * m * v) <= 1e-10 * np.linalg.norm(K @ v)


@pytest.mark.parametrize("n", [(7, 6), (5, 4, 4)])
def test_jacobian_matches_central_differences(n):
    """The adjoint sensitivities of the P1 heads against central differences of heads_p1 in
    ln kappa_c and ln S_c (a few cells, step 1e-4), relative to each map's largest entry."""
    from oracle.p1 import jacobian_p1
    d = len(n)
    h = tuple(1.0 / v for v in n)
    rng = np.random.default_rng(6)
    nc = int(np.prod(n))
    kap = np.exp(0.6 * rng.standard_normal(nc))
    S = np.exp(0.3 * rng.standard_normal(nc)) * 1e-3
    pad = (0.0,) if d == 2 else ()
    src = np.array([[0.41, 0.47] + ([0.5] if d == 3 else [0.0])])
    rec = np.array([[0.62, 0.33] + ([0.45] if d == 3 else [0.0]), [0.3, 0.7] + ([0.6] if d == 3 else [0.0])])
    times = [2e-4, 1e-3]  # 0.2 and 1 diffusion time S L^2 / kappa: storage still matters
    JK, JS = jacobian_p1(n, h, kap, S, src, rec, times, 24)
    eps = 1e-4
    for c in rng.choice(nc, 4, replace=False):
        for which, J in (("k", JK), ("s", JS)):
            up_k, dn_k, up_s, dn_s = kap.copy(), kap.copy(), S.copy(), S.copy()
            if which == "k":
                up_k[c] *= np.exp(eps)
                dn_k[c] *= np.exp(-eps)
            else:
                up_s[c] *= np.exp(eps)
                dn_s[c] *= np.exp(-eps)
            fd = (heads_p1(n, h, up_k, up_s, src, rec, times, 24) - heads_p1(n, h, dn_k, dn_s, src, rec, times, 24)) / (2 * eps)
            scale = np.abs(J).max()
            assert np.abs(J[..., c] - fd).max() <= 1e-6 * scale, (which, c)
