"""Pins for the oracle's finite-volume assembly (Section 2.1 discretisation,
read as the cell-centred scheme stated in oracle/fv.py)."""
import numpy as np
import pytest

from oracle.fv import assemble, point_weights


def test_hand_computed_2x2():
    # 2x2 cells on the unit square, kappa by cell (x fastest): 1, 3 / 2, 4.
    # Interior faces: harmonic means 2*1*3/4, 2*2*4/6, 2*1*2/3, 2*3*4/7 (A/h = 1).
    # Every cell touches two zero-Dirichlet walls, each worth 2*kappa*A/h = 2 kappa.
    K, m = assemble((2, 2, 1), (0.5, 0.5, 1.0), [1.0, 3.0, 2.0, 4.0], [2.0] * 4)
    t01, t23, t02, t13 = 1.5, 8.0 / 3.0, 4.0 / 3.0, 24.0 / 7.0
    want = np.array([
        [t01 + t02 + 4.0, -t01, -t02, 0.0],
        [-t01, t01 + t13 + 12.0, 0.0, -t13],
        [-t02, 0.0, t23 + t02 + 8.0, -t23],
        [0.0, -t13, -t23, t23 + t13 + 16.0],
    ])
    np.testing.assert_allclose(K.toarray(), want, rtol=1e-15, atol=0)
    np.testing.assert_allclose(m, [0.5] * 4, rtol=1e-15)


def test_hand_computed_3d_column():
    # 1x1x2 column with h = (0.5, 0.25, 0.2): area of a z face 0.125, dz = 0.2.
    # kappa 1 and 4: face T = 2*1*4/5 * 0.125/0.2 = 1.0.  Walls of cell 0:
    # -x,+x: 2*1*(0.25*0.2)/0.5 each = 0.2; -y,+y: 2*1*(0.5*0.2)/0.25 = 0.8 each;
    # -z: 2*1*0.125/0.2 = 1.25.  Cell 1 has kappa 4: 0.8, 0.8, 3.2, 3.2, 5.0.
    K, m = assemble((1, 1, 2), (0.5, 0.25, 0.2), [1.0, 4.0], [3.0, 3.0], ndim=3)
    d0 = 1.0 + 0.4 + 1.6 + 1.25
    d1 = 1.0 + 1.6 + 6.4 + 5.0
    np.testing.assert_allclose(K.toarray(), [[d0, -1.0], [-1.0, d1]], rtol=1e-14)
    np.testing.assert_allclose(m, [3.0 * 0.025] * 2, rtol=1e-15)


def test_neumann_rows_sum_to_zero():
    rng = np.random.default_rng(0)
    n = (5, 4, 3)
    kap = np.exp(rng.standard_normal(60))
    K, _ = assemble(n, (0.2, 0.25, 1 / 3), kap, np.ones(60), bc=(1,) * 6)
    np.testing.assert_allclose(K.sum(axis=1).A.ravel(), 0.0, atol=1e-12)
    assert abs(K - K.T).max() == 0.0


@pytest.mark.parametrize("n", [(6, 5, 1), (4, 3, 5)])
def test_homogeneous_sine_modes_are_exact_eigenvectors(n):
    # With the wall value at h/2, sampled sin(k pi x) modes are exact discrete
    # eigenvectors: lambda = sum_a (4 kappa / h_a^2) sin^2(k_a pi h_a / 2) / S.
    nd = 3 if n[2] > 1 else 2
    h = tuple(1.0 / a for a in n[:nd]) + (1.0,) * (3 - nd)
    N = int(np.prod(n))
    kap, S = 2.5, 0.7
    K, m = assemble(n, h, np.full(N, kap), np.full(N, S))
    xs = [(np.arange(n[a]) + 0.5) * h[a] for a in range(3)]
    for modes in [(1, 1, 1), (2, 3, 1), (5, 1, 2)]:
        modes = modes[:nd] + (0,) * (3 - nd)
        f = np.ones((n[2], n[1], n[0]))
        lam = 0.0
        for a in range(nd):
            shape = [1, 1, 1]
            shape[2 - a] = n[a]
            f = f * np.sin(modes[a] * np.pi * xs[a]).reshape(shape)
            lam += 4 * kap / h[a] ** 2 * np.sin(modes[a] * np.pi * h[a] / 2) ** 2 / S
        v = f.ravel()
        np.testing.assert_allclose(K @ v, lam * m * v, rtol=1e-12, atol=1e-12 * lam * np.abs(m * v).max())


def test_point_weights():
    n, h = (32, 32, 1), (1 / 32, 1 / 32, 1.0)
    B = point_weights(n, h, [(0.5, 0.5, 0.0)]).toarray()[0]
    nz = np.nonzero(B)[0]
    assert sorted(nz.tolist()) == [15 + 32 * 15, 16 + 32 * 15, 15 + 32 * 16, 16 + 32 * 16]
    np.testing.assert_allclose(B[nz], 0.25)
    # bilinear interpolation reproduces linear functions at interior points
    xc = (np.arange(32) + 0.5) / 32
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    lin = (1.0 + 2.0 * X - 3.0 * Y).ravel()
    pts = [(0.3, 0.7, 0.0), (0.123, 0.9, 0.0), (0.61, 0.2, 0.0)]
    W = point_weights(n, h, pts)
    np.testing.assert_allclose(W @ lin, [1 + 2 * x - 3 * y for x, y, _ in pts], rtol=1e-13)
    np.testing.assert_allclose(W.sum(axis=1).A.ravel(), 1.0)
    # within h/2 of a wall the nearest cell takes the whole weight
    Wc = point_weights(n, h, [(0.001, 0.999, 0.0)]).toarray()[0]
    assert Wc[0 + 32 * 31] == 1.0
