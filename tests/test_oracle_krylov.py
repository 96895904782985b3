"""Pins of the oracle's Algorithm 1 (flexible shifted FOM/GMRES with exact
shift-and-invert preconditioners), each against something other than the oracle:

* the solutions against direct solves of each shifted system (true residuals by a
  sparse product, and the solution itself);
* the flexible Arnoldi relation (eqn:shiftedarnoldimod) at a shift that is not
  solved, and the orthonormality of the basis;
* the shift equal to a single preconditioner's tau, solved at the first step;
* the happy breakdown of an eigenmode right-hand side, against the closed-form
  eigenvalue of the homogeneous grid (x_k = b / (S V (lambda + z_k)));
* FOM against GMRES (same basis; FOM's residual is never below GMRES's);
* the restarted FOM: its residuals against -eta_k v_{m+1} by sparse products (the
  collinearity of Section 3.1), its solutions against direct solves, and a cycle longer than
  the solve against FOM without restarts.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve

from oracle.contour import talbot_nodes
from oracle.fv import assemble, point_weights
from oracle.krylov import flexible_shifted, restarted_fom, shift_invert, tau_schedule
from workloads.configs import T_D, make_problem


def _problem(n=(24, 20), var=1.6, seed=7):
    p = make_problem("W1", n=n, seed=seed, var=var)
    K, m = assemble(p.n, p.h, p.kappa, p.S)
    b = point_weights(p.n, p.h, p.sources[:1]).toarray().ravel()
    z, _ = talbot_nodes(20, 0.3 * T_D)
    return K, m, b, z


def test_solutions_match_direct_solves():
    K, m, b, z = _problem()
    out = flexible_shifted(K, m, b, tau_schedule(z, 2), z, tol=1e-9, maxit=80)
    assert out["conv"].all()
    for k in range(z.size):
        A = (K + sp.diags(z[k] * m)).tocsc()
        r = b - A @ out["x"][k]
        assert np.linalg.norm(r) <= 1.05e-9 * np.linalg.norm(b)  # the true residual meets the test
        xd = spsolve(A.astype(np.complex128), b.astype(np.complex128))
        assert np.linalg.norm(out["x"][k] - xd) <= 1e-6 * np.linalg.norm(xd)


def test_flexible_arnoldi_relation_and_orthonormal_basis():
    K, m, b, z = _problem()
    out = flexible_shifted(K, m, b, tau_schedule(z, 2), z, tol=1e-12, maxit=12)
    V, U, Hb, T = out["V"], out["U"], out["Hbar"], out["T"]
    j = U.shape[1]
    assert j == 12 and not out["breakdown"]
    zt = complex(3.0e5, -7.0e5)  # any shift: the relation holds for every z
    lhs = (K + sp.diags(zt * m)) @ U
    rhs = V @ (np.eye(j + 1, j) + Hb @ np.diag(zt - T))
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(lhs)
    assert np.abs(V.conj().T @ V - np.eye(j + 1)).max() <= 1e-12


def test_shift_equal_to_single_tau_converges_at_first_step():
    K, m, b, z = _problem()
    out = flexible_shifted(K, m, b, [z[3]], z, tol=1e-10, maxit=60)
    assert out["conv_at"][3] == 1
    xd = shift_invert(K, m, z[3], b)
    assert np.linalg.norm(out["x"][3] - xd) <= 1e-13 * np.linalg.norm(xd)


@pytest.mark.parametrize("method", ["gmres", "fom"])
def test_eigenmode_right_hand_side_breaks_down_with_the_exact_solution(method):
    n, kap, S = (16, 12), 1.0, 1e-5
    h = (1.0 / n[0], 1.0 / n[1])
    K, m = assemble(n + (1,), h + (1.0,), np.full(n[0] * n[1], kap), np.full(n[0] * n[1], S))
    xs = [(np.arange(n[a]) + 0.5) * h[a] for a in range(2)]
    modes = (2, 3)
    b = np.outer(np.sin(modes[1] * np.pi * xs[1]), np.sin(modes[0] * np.pi * xs[0])).ravel()  # x fastest
    # closed form: K b = lam (S V) b with lam = sum_a 4 kappa / h_a^2 sin^2(k_a pi h_a / 2) / S
    lam = sum(4 * kap / h[a] ** 2 * np.sin(modes[a] * np.pi * h[a] / 2) ** 2 for a in range(2)) / S
    SV = S * h[0] * h[1]
    z, _ = talbot_nodes(16, 0.3 * T_D)
    out = flexible_shifted(K, m, b, tau_schedule(z, 2), z, tol=1e-14, maxit=5, method=method)
    assert out["iters"] == 1
    assert abs(out["Hbar"][1, 0]) <= 1e-12 * abs(out["Hbar"][0, 0])
    for k in range(z.size):
        exact = b / (SV * (lam + z[k]))
        assert np.linalg.norm(out["x"][k] - exact) <= 1e-9 * np.linalg.norm(exact)


def test_fom_residual_never_below_gmres():
    K, m, b, z = _problem(n=(20, 18))
    taus = tau_schedule(z, 2)
    for j in (3, 6, 9):
        g = flexible_shifted(K, m, b, taus, z, tol=0.0, maxit=j, method="gmres")
        f = flexible_shifted(K, m, b, taus, z, tol=0.0, maxit=j, method="fom")
        assert g["iters"] == f["iters"] == j
        assert np.all(f["res"] >= g["res"] * (1 - 1e-10) - 1e-14)  # rounding floor (shifts equal to a tau)


def test_tau_schedule_follows_the_rule_of_section_3():
    z, _ = talbot_nodes(40, 1.0)
    t = tau_schedule(z, 2)
    lo, hi = z[np.argmin(z.real)], z[np.argmax(z.real)]
    assert t == [lo, lo, lo, hi, hi]
    assert lo.real < 0 < lo.imag  # the paper's first preconditioner shift has a negative real part
    assert tau_schedule(z, 1) == [lo]


def test_adaptive_shift_rule():
    from oracle.krylov import adaptive_shift
    z = np.array([-3 + 4j, 1 + 2j, 5 + 1j])
    w = np.array([1.0, 1.0, 0.5])
    res = np.array([0.1, 0.3, 0.9])
    conv = np.array([False, False, False])
    # weighted residuals 0.1, 0.3, 0.45: the third node
    assert adaptive_shift(z, w, res, conv) == 5 + 1j
    # converged shifts are skipped; a node left of the imaginary axis is projected onto it
    conv2 = np.array([False, True, True])
    assert adaptive_shift(z, w, res, conv2) == 4j
    # candidates: the nearest one
    assert adaptive_shift(z, w, res, conv2, candidates=[-2 + 3j, 6 + 0j]) == -2 + 3j
    assert adaptive_shift(z, w, res, np.array([True, True, True])) is None


def test_adaptive_shifts_still_solve_the_systems():
    K, m, b, z = _problem()
    out = flexible_shifted(K, m, b, tau_schedule(z, 2), z, tol=1e-9, maxit=80, adapt=True)
    assert out["conv"].all() and len(set(np.round(out["T"], 6))) > 2
    for k in range(z.size):
        xd = shift_invert(K, m, z[k], b)
        assert np.linalg.norm(out["x"][k] - xd) <= 1e-6 * np.linalg.norm(xd)


def test_fom_residuals_are_collinear_with_the_next_basis_vector():
    """Section 3.1: with an exact preconditioner the FOM residual of every shift after m steps
    is -eta_k v_{m+1}.  Pinned by explicit sparse products: the true residual of each shift
    still active at the end of a 4-step cycle, against -eta_k times the cycle's last basis
    vector."""
    K, m, b, z = _problem()
    out = restarted_fom(K, m, b, tau_schedule(z, 2), z, tol=0.0, cycle=4, max_cycles=1)
    v5, eta = out["history"][0]
    for k in range(z.size):
        r = b - (K + sp.diags(z[k] * m)) @ out["x"][k]
        assert np.linalg.norm(r + eta[k] * v5) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(v5) == pytest.approx(1.0, abs=1e-12)


def test_restarted_fom_solves_the_systems():
    """Restarts every 3 steps from the collinear residuals: every shift's true residual meets
    the test (a sparse product) and the solution matches a direct solve."""
    K, m, b, z = _problem()
    out = restarted_fom(K, m, b, tau_schedule(z, 2), z, tol=1e-9, cycle=3, max_cycles=60)
    assert out["conv"].all() and out["cycles"] > 2
    for k in range(z.size):
        A = (K + sp.diags(z[k] * m)).tocsc()
        r = b - A @ out["x"][k]
        assert np.linalg.norm(r) <= 1.05e-9 * np.linalg.norm(b)
        xd = spsolve(A.astype(np.complex128), b.astype(np.complex128))
        assert np.linalg.norm(out["x"][k] - xd) <= 1e-6 * np.linalg.norm(xd)


def test_restart_longer_than_the_solve_is_plain_fom():
    """A cycle longer than the steps needed never restarts: the same steps, residuals and
    solutions as FOM without restarts."""
    K, m, b, z = _problem(n=(20, 18))
    taus = tau_schedule(z, 2)
    f = flexible_shifted(K, m, b, taus, z, tol=1e-9, maxit=80, method="fom")
    r = restarted_fom(K, m, b, taus, z, tol=1e-9, cycle=80, max_cycles=1)
    assert r["cycles"] == 1 and r["iters"] == f["iters"]
    assert np.allclose(r["res"], f["res"], rtol=1e-9, atol=1e-15)
    assert np.abs(r["x"] - f["x"]).max() <= 1e-12 * np.abs(f["x"]).max()
