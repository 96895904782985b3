"""Flexible FOM / GMRES for shifted systems with exact shift-and-invert preconditioners.

Oracle (test infrastructure only).

Algorithm 1 of Section 3 (flexible FOM/GMRES for shifted systems) solves
(K + z_k M) x_k = b for every shift z_k with one basis.  Step j applies the
preconditioner of that step exactly, u_j = (K + tau_j M)^{-1} v_j (a sparse direct
factorisation, made once per distinct tau), and orthogonalises s_j = M u_j against
v_1 .. v_j by modified Gram-Schmidt; the coefficients form column j of the
(j + 1) x j Hessenberg matrix Hbar_j and the normalised remainder is v_{j+1}.  With
T_j = diag(tau_1 .. tau_j) the flexible Arnoldi relation (eqn:shiftedarnoldimod)

    (K + z M) U_j = V_{j+1} ( [I; 0] + Hbar_j (z I - T_j) )

reduces each shifted system to a (j + 1) x j one: the GMRES variant (FGMRES-Sh) takes
the y that minimises || beta e_1 - Hbar_j(z; T_j) y ||, the FOM variant (FFOM-Sh)
solves its square upper part, and x = U_j y.  A shift whose residual norm meets the
test keeps its last y; the loop stops once every shift has.  A zero h_{j+1, j} ends
the loop with every shift solved exactly (the basis spans the solutions).

Reading: the printed orthogonalisation subtracts h_ij v_j; Gram-Schmidt removes the
component along each v_i, which is what is done here.

The preconditioner schedule of Section 3 (tau_schedule) takes the shift of smallest
real part (tau_bar_1) and of largest real part (tau_bar_2) among all shifts, and uses
tau_bar_1 for three steps and tau_bar_2 for two, repeated; a single preconditioner is
tau_bar_1 alone (the 'Single' solver of Section 4.1).

restarted_fom restarts the FOM variant from its residuals, which an exact preconditioner makes
collinear with the next basis vector (Section 3.1: r_k = -eta_k v_{m+1}).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu


def shift_invert(K, m, tau, rhs):
    """(K + tau M)^{-1} rhs by one sparse direct factorisation (the plain definition)."""
    A = (K + sp.diags(tau * np.asarray(m, dtype=np.float64))).astype(np.complex128).tocsc()
    return splu(A, permc_spec="MMD_AT_PLUS_A").solve(np.asarray(rhs, dtype=np.complex128))


def tau_schedule(shifts, n_tau):
    """Preconditioner shifts of Section 3 over the given shifts (any real part)."""
    z = np.asarray(shifts, dtype=np.complex128).ravel()
    t1 = z[np.argmin(z.real)]
    t2 = z[np.argmax(z.real)]
    if n_tau == 1:
        return [t1]
    if n_tau == 2:
        return [t1, t1, t1, t2, t2]
    raise ValueError("n_tau must be 1 or 2")


def adaptive_shift(z, w, res, conv, candidates=None):
    """The next preconditioner shift from the residual estimates: the unconverged shift z_k of
    largest weighted residual w_k ||r_k||, or the nearest of ``candidates`` to it; without
    candidates, z_k itself when Re z_k >= 0, else i Im z_k (a multigrid preconditioner needs a
    non-negative real part).  None when every shift has converged."""
    wr = np.where(conv, -np.inf, w * res)
    k = int(np.argmax(wr))
    if not np.isfinite(wr[k]):
        return None
    zk = complex(z[k])
    if candidates is not None:
        c = np.asarray(candidates, dtype=np.complex128)
        return complex(c[np.argmin(np.abs(c - zk))])
    return zk if zk.real >= 0 else complex(0.0, zk.imag)


def flexible_shifted(K, m, b, taus, shifts, tol, maxit, method="gmres", weights=None, precond=None,
                     adapt=False, candidates=None):
    """Algorithm 1 for one right-hand side b (real or complex [N]).

    ``taus``: preconditioner shifts used cyclically (tau_j = taus[(j - 1) % len]);
    ``shifts``: the z_k; a shift is converged when weights_k ||r_k|| <= tol ||b||, with
    r_k the small problem's residual (weights default 1: the relative test of
    Section 4.1).  ``precond(tau, v)``, if given, replaces the exact solve of
    (K + tau M) u = v (a test hook for inexact preconditioners).  ``adapt``: from the
    second step on, tau_j = adaptive_shift(...) of the previous step's residuals (the build's
    own rule for choosing shifts from the a-posteriori estimates; ``candidates`` as there)
    instead of the cyclic schedule.  Returns a dict
    with x [nk, N], iters (steps taken), res [nk] (||r_k|| / ||b||), conv [nk],
    conv_at [nk] (step at which each shift met the
    test, 0 if never), V [N, iters + 1], U [N, iters], Hbar [iters + 1, iters],
    T [iters] and breakdown (True when h_{j+1, j} = 0 ended the loop).
    """
    m = np.asarray(m, dtype=np.float64)
    z = np.asarray(shifts, dtype=np.complex128).ravel()
    nk = z.size
    w = np.ones(nk) if weights is None else np.asarray(weights, dtype=np.float64)
    b = np.asarray(b, dtype=np.complex128)
    N = b.size
    beta = np.linalg.norm(b)
    lus = {}

    def solve(tau, v):
        key = (float(tau.real), float(tau.imag))
        if key not in lus:
            A = (K + sp.diags(tau * m)).astype(np.complex128).tocsc()
            lus[key] = splu(A, permc_spec="MMD_AT_PLUS_A")
        return lus[key].solve(v)

    V = np.zeros((N, maxit + 1), dtype=np.complex128)
    U = np.zeros((N, maxit), dtype=np.complex128)
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    T = np.zeros(maxit, dtype=np.complex128)
    V[:, 0] = b / beta
    Y = [None] * nk
    res = np.full(nk, np.inf)
    conv = np.zeros(nk, dtype=bool)
    conv_at = np.zeros(nk, dtype=int)
    j = 0
    breakdown = False
    for j in range(1, maxit + 1):
        tau = complex(taus[(j - 1) % len(taus)])
        if adapt and j > 1:
            t_ad = adaptive_shift(z, w, res, conv, candidates)
            if t_ad is not None:
                tau = t_ad
        T[j - 1] = tau
        u = solve(tau, V[:, j - 1]) if precond is None else np.asarray(precond(tau, V[:, j - 1]), dtype=np.complex128)
        U[:, j - 1] = u
        s = m * u
        for i in range(j):
            H[i, j - 1] = np.vdot(V[:, i], s)
            s = s - H[i, j - 1] * V[:, i]
        H[j, j - 1] = np.linalg.norm(s)
        breakdown = H[j, j - 1] == 0.0
        if not breakdown:
            V[:, j] = s / H[j, j - 1]
        Hb = H[:j + 1, :j]
        e1 = np.zeros(j + 1, dtype=np.complex128)
        e1[0] = beta
        for k in range(nk):
            if conv[k]:
                continue
            Hz = np.eye(j + 1, j, dtype=np.complex128) + Hb @ np.diag(z[k] - T[:j])
            if method == "gmres":
                y = np.linalg.lstsq(Hz, e1, rcond=None)[0]
            else:
                y = np.linalg.solve(Hz[:j, :j], e1[:j])
            Y[k] = y
            res[k] = np.linalg.norm(e1 - Hz @ y) / beta
            if w[k] * res[k] <= tol or breakdown:
                conv[k] = True
                conv_at[k] = j
        if conv.all():
            break
    x = np.stack([U[:, :len(Y[k])] @ Y[k] for k in range(nk)])
    return {"x": x, "iters": j, "res": res, "conv": conv, "conv_at": conv_at,
            "V": V[:, :j + 1], "U": U[:, :j], "Hbar": H[:j + 1, :j], "T": T[:j], "breakdown": breakdown}


def restarted_fom(K, m, b, taus, shifts, tol, cycle, max_cycles, weights=None, precond=None):
    """FFOM-Sh restarted every ``cycle`` steps from its collinear residuals (exact preconditioners).

    With FOM and an exact preconditioner, the residual of every shift after m steps of
    Algorithm 1 is b - (K + z_k M) x_k = -eta_k v_{m+1}, with the a-posteriori quantity
    eta_k = h_{m+1,m} (z_k - tau_m) e_m^T H_m(z_k; T_m)^{-1} beta e_1 of Section 3.1: one
    vector for all shifts.  A restart therefore continues with one basis started at
    v_1 = v_{m+1}, in which shift k solves (K + z_k M) d_k = -eta_k v_1: its small problem
    H_m(z_k; T_m) y = beta_k e_1 takes beta_k = -eta_k (complex) instead of ||b||.  The
    preconditioner shifts run through ``taus`` cyclically across restarts (step j of the whole
    solve uses taus[(j - 1) % len]).  A shift is converged when w_k |eta_k| <= tol ||b||.

    Returns a dict with x [nk, N], cycles, iters (steps over all cycles), res [nk]
    (|eta_k| / ||b|| after the last step that updated shift k), conv [nk], and per cycle the
    pairs (v_{m+1}, eta) in ``history`` for tests of the collinearity.
    """
    m = np.asarray(m, dtype=np.float64)
    z = np.asarray(shifts, dtype=np.complex128).ravel()
    nk = z.size
    w = np.ones(nk) if weights is None else np.asarray(weights, dtype=np.float64)
    b = np.asarray(b, dtype=np.complex128)
    N = b.size
    bnorm = np.linalg.norm(b)
    lus = {}

    def solve(tau, v):
        key = (float(tau.real), float(tau.imag))
        if key not in lus:
            A = (K + sp.diags(tau * m)).astype(np.complex128).tocsc()
            lus[key] = splu(A, permc_spec="MMD_AT_PLUS_A")
        return lus[key].solve(v)

    x = np.zeros((nk, N), dtype=np.complex128)
    conv = np.zeros(nk, dtype=bool)
    res = np.full(nk, np.inf)
    beta_k = np.full(nk, bnorm, dtype=np.complex128)  # the first cycle starts from b itself
    v1 = b / bnorm
    step = 0
    history = []
    cycles = 0
    for cycles in range(1, max_cycles + 1):
        V = np.zeros((N, cycle + 1), dtype=np.complex128)
        U = np.zeros((N, cycle), dtype=np.complex128)
        H = np.zeros((cycle + 1, cycle), dtype=np.complex128)
        T = np.zeros(cycle, dtype=np.complex128)
        V[:, 0] = v1
        eta = np.zeros(nk, dtype=np.complex128)
        Y = [None] * nk
        done = conv.copy()  # shifts already converged take no part in this cycle
        j = 0
        for j in range(1, cycle + 1):
            step += 1
            tau = complex(taus[(step - 1) % len(taus)])
            T[j - 1] = tau
            u = solve(tau, V[:, j - 1]) if precond is None else np.asarray(precond(tau, V[:, j - 1]),
                                                                            dtype=np.complex128)
            U[:, j - 1] = u
            s = m * u
            for i in range(j):
                H[i, j - 1] = np.vdot(V[:, i], s)
                s = s - H[i, j - 1] * V[:, i]
            H[j, j - 1] = np.linalg.norm(s)
            if H[j, j - 1] != 0.0:
                V[:, j] = s / H[j, j - 1]
            for k in range(nk):
                if done[k]:
                    continue
                # the square FOM system of this cycle, right-hand side beta_k e_1
                Hz = np.eye(j, dtype=np.complex128) + H[:j, :j] @ np.diag(z[k] - T[:j])
                rhs = np.zeros(j, dtype=np.complex128)
                rhs[0] = beta_k[k]
                y = np.linalg.solve(Hz, rhs)
                Y[k] = y
                eta[k] = H[j, j - 1] * (z[k] - T[j - 1]) * y[j - 1]
                res[k] = abs(eta[k]) / bnorm
                if w[k] * res[k] <= tol or H[j, j - 1] == 0.0:
                    done[k] = True
            if done.all():
                break
        for k in range(nk):
            if Y[k] is not None:
                x[k] += U[:, :len(Y[k])] @ Y[k]
        history.append((V[:, j].copy(), eta.copy()))
        conv = done
        if conv.all():
            break
        # restart: every unconverged shift's residual is -eta_k v_{j+1}
        v1 = V[:, j].copy()
        beta_k = -eta
    return {"x": x, "cycles": cycles, "iters": step, "res": res, "conv": conv, "history": history}
