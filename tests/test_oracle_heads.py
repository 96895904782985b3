"""Pins for the oracle's heads (eqn:half over direct shifted solves).

Each check compares against something the oracle does not compute itself:
the exact solution of M phi' + K phi = q b by dense eigendecomposition,
an independent Crank-Nicolson integration, a closed-form eigenmode decay,
the steady state from a library sparse solve, reciprocity and linearity.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as wl
from oracle.fv import assemble, point_weights
from oracle.heads import heads, shifted_fields
from oracle.contour import talbot_nodes


def _tiny(n, seed=3, var=1.0):
    nd = 3 if n[2] > 1 else 2
    h = tuple(1.0 / a for a in n[:nd]) + (1.0,) * (3 - nd)
    N = int(np.prod(n))
    kap = np.exp(wl.gaussian_random_field(n[:nd], h[:nd], (0.3,) * nd, var, seed)).flatten(order="F")
    S = np.full(N, 1e-5)
    return n, h, kap, S


def _exact(K, m, b, t, q=1.0):
    """phi(t) for M phi' + K phi = q b, phi(0) = 0, by A = M^-1/2 K M^-1/2 = Q L Q^T."""
    Mi = 1.0 / np.sqrt(m)
    A = Mi[:, None] * K.toarray() * Mi[None, :]
    lam, Q = np.linalg.eigh(A)
    c = Q.T @ (Mi * b)
    return Mi * (Q @ ((1.0 - np.exp(-lam * t)) / lam * c)) * q


@pytest.mark.parametrize("n,nz", [((6, 5, 1), 16), ((6, 5, 1), 24), ((4, 3, 3), 20)])
def test_heads_match_dense_exponential(n, nz):
    n, h, kap, S = _tiny(n)
    src = [(0.5, 0.45, 0.5)]
    rec = [(0.2, 0.3, 0.4), (0.75, 0.6, 0.6), (0.5, 0.45, 0.5)]
    times = wl.T_D * np.array([0.01, 0.1, 1.0, 5.0])
    phi = heads(n, h, kap, S, src, rec, times, nz)
    K, m = assemble(n, h, kap, S)
    b = point_weights(n, h, src).toarray()[0]
    Br = point_weights(n, h, rec).toarray()
    scale = np.abs(Br @ _exact(K, m, b, 1e3)).max()
    tol = 20.0 * 3.89 ** (-nz) * np.exp(0.171 * nz) + 1e-12
    for it, t in enumerate(times):
        ex = Br @ _exact(K, m, b, t)
        assert np.abs(phi[0, :, it] - ex).max() <= tol * scale


def _crank_nicolson(K, m, b, t, nsteps, q=1.0):
    """Two backward-Euler half steps (Rannacher start), then CN steps."""
    Kd = K.toarray()
    M = np.diag(m)
    phi = np.zeros_like(b)
    dt = t / nsteps
    # two implicit Euler half-steps cover the first dt
    A_be = M + 0.5 * dt * Kd
    for _ in range(2):
        phi = np.linalg.solve(A_be, M @ phi + 0.5 * dt * q * b)
    A_l = M + 0.5 * dt * Kd
    A_r = M - 0.5 * dt * Kd
    lu = np.linalg.inv(A_l)
    for _ in range(nsteps - 1):
        phi = lu @ (A_r @ phi + dt * q * b)
    return phi


def test_heads_match_crank_nicolson():
    n, h, kap, S = _tiny((5, 4, 1), seed=7)
    src = [(0.5, 0.5, 0.0)]
    rec = [(0.3, 0.3, 0.0), (0.7, 0.6, 0.0)]
    t = 0.3 * wl.T_D
    phi = heads(n, h, kap, S, src, rec, [t], 24)[0, :, 0]
    K, m = assemble(n, h, kap, S)
    b = point_weights(n, h, src).toarray()[0]
    Br = point_weights(n, h, rec).toarray()
    p1 = Br @ _crank_nicolson(K, m, b, t, 2000)
    p2 = Br @ _crank_nicolson(K, m, b, t, 4000)
    rich = (4.0 * p2 - p1) / 3.0
    np.testing.assert_allclose(phi, rich, rtol=1e-8, atol=1e-10 * np.abs(rich).max())


@pytest.mark.parametrize("n", [(8, 6, 1), (4, 4, 3)])
def test_single_eigenmode_decays_exactly(n):
    nd = 3 if n[2] > 1 else 2
    h = tuple(1.0 / a for a in n[:nd]) + (1.0,) * (3 - nd)
    N = int(np.prod(n))
    kap, s = 1.3, 2e-5
    f = np.ones((n[2], n[1], n[0]))
    lam = 0.0
    for a in range(nd):
        shape = [1, 1, 1]
        shape[2 - a] = n[a]
        f = f * np.sin(np.pi * (np.arange(n[a]) + 0.5) * h[a]).reshape(shape)
        lam += 4 * kap / h[a] ** 2 * np.sin(np.pi * h[a] / 2) ** 2 / s
    phi0 = f.ravel()
    rec = [(0.3, 0.4, 0.5), (0.55, 0.5, 0.5)]
    times = np.array([0.05, 0.5, 2.0]) / lam
    phi = heads(n, h, np.full(N, kap), np.full(N, s), [(0.5, 0.5, 0.5)], rec, times, 24,
                q=0.0, phi0=phi0)
    Br = point_weights(n, h, rec)
    for it, t in enumerate(times):
        np.testing.assert_allclose(phi[0, :, it], np.exp(-lam * t) * (Br @ phi0), rtol=1e-9, atol=1e-12)


def test_steady_state_limit_matches_library_solve():
    n, h, kap, S = _tiny((7, 6, 1), seed=11)
    src = [(0.4, 0.55, 0.0)]
    rec = [(0.2, 0.2, 0.0), (0.8, 0.7, 0.0)]
    K, m = assemble(n, h, kap, S)
    b = point_weights(n, h, src).toarray()[0]
    ss = point_weights(n, h, rec) @ spla.spsolve(K.tocsc(), 2.5 * b)
    phi = heads(n, h, kap, S, src, rec, [1e3 * wl.T_D], 20, q=2.5)[0, :, 0]
    np.testing.assert_allclose(phi, ss, rtol=1e-10)


def test_reciprocity_and_linearity():
    n, h, kap, S = _tiny((8, 7, 1), seed=5)
    a, b = (0.3, 0.35, 0.0), (0.65, 0.7, 0.0)
    times = wl.T_D * np.array([0.05, 0.5])
    ab = heads(n, h, kap, S, [a], [b], times, 16)
    ba = heads(n, h, kap, S, [b], [a], times, 16)
    np.testing.assert_allclose(ab, ba, rtol=1e-12)
    np.testing.assert_allclose(heads(n, h, kap, S, [a], [b], times, 16, q=3.0), 3.0 * ab, rtol=1e-12)


def test_direct_solves_are_exact():
    n, h, kap, S = _tiny((5, 5, 1))
    K, m = assemble(n, h, kap, S)
    rhs = np.random.default_rng(0).standard_normal((25, 3))
    z, _ = talbot_nodes(16, 0.2 * wl.T_D)
    X = shifted_fields(K, m, rhs, z[:3])
    for zk, x in zip(z[:3], X):
        A = K.toarray() + zk * np.diag(m)
        np.testing.assert_allclose(x, np.linalg.solve(A, rhs), rtol=1e-12)
        assert np.abs(A @ x - rhs).max() <= 1e-13 * np.abs(A).max() * np.abs(x).max()


def _exact_ivp(K, m, phi0, t):
    """phi(t) for M phi' + K phi = 0, phi(0) = phi0, by the same eigendecomposition."""
    Ms, Mi = np.sqrt(m), 1.0 / np.sqrt(m)
    A = Mi[:, None] * K.toarray() * Mi[None, :]
    lam, Q = np.linalg.eigh(A)
    return Mi * (Q @ (np.exp(-lam * t) * (Q.T @ (Ms * phi0))))


@pytest.mark.parametrize("n", [(6, 5, 1), (4, 3, 3)])
def test_initial_head_and_rates_match_dense_exponential(n):
    """Two wells at different rates plus a random initial head: each row is the exact
    semi-discrete solution q_s (pumping response of well s) + (decay of phi0), within the
    contour's error (Section 2.1 transformed system with the M phi0 term)."""
    n, h, kap, S = _tiny(n, seed=8)
    N = int(np.prod(n))
    src = [(0.5, 0.45, 0.5), (0.3, 0.7, 0.3)]
    rates = np.array([1.7, -0.6])
    rec = [(0.2, 0.3, 0.4), (0.75, 0.6, 0.6)]
    phi0 = np.random.default_rng(4).standard_normal(N)
    nz = 24
    times = wl.T_D * np.array([0.01, 0.1, 1.0])
    phi = heads(n, h, kap, S, src, rec, times, nz, q=rates, phi0=phi0)
    K, m = assemble(n, h, kap, S)
    B = point_weights(n, h, src).toarray()
    Br = point_weights(n, h, rec).toarray()
    scale = max(np.abs(Br @ _exact(K, m, B[0], 1e3)).max(), np.abs(phi0).max())
    tol = 20.0 * 3.89 ** (-nz) * np.exp(0.171 * nz) + 1e-12
    for it, t in enumerate(times):
        ivp = Br @ _exact_ivp(K, m, phi0, t)
        for s in range(2):
            ex = Br @ _exact(K, m, B[s], t, q=rates[s]) + ivp
            assert np.abs(phi[s, :, it] - ex).max() <= tol * scale


def test_initial_head_alone_gives_one_row():
    """With no wells the result is one row of initial-value heads, equal to the phi0 part of
    any run with wells (superposition)."""
    n, h, kap, S = _tiny((7, 6, 1), seed=2)
    N = int(np.prod(n))
    phi0 = np.random.default_rng(1).standard_normal(N)
    rec = [(0.2, 0.3, 0.0), (0.6, 0.5, 0.0)]
    times = wl.T_D * np.array([0.02, 0.3])
    alone = heads(n, h, kap, S, np.zeros((0, 3)), rec, times, 20, phi0=phi0)
    assert alone.shape == (1, 2, 2)
    both = heads(n, h, kap, S, [(0.5, 0.5, 0.0)], rec, times, 20, q=2.0, phi0=phi0)
    wells = heads(n, h, kap, S, [(0.5, 0.5, 0.0)], rec, times, 20, q=2.0)
    np.testing.assert_allclose(both - wells, alone, rtol=1e-10, atol=1e-14)
    K, m = assemble(n, h, kap, S)
    Br = point_weights(n, h, rec).toarray()
    for it, t in enumerate(times):
        ex = Br @ _exact_ivp(K, m, phi0, t)
        assert np.abs(alone[0, :, it] - ex).max() <= 1e-6 * np.abs(phi0).max()
