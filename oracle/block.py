"""Block flexible GMRES for shifted systems with several right-hand sides.

Oracle (test infrastructure only).

Section 6 names block Krylov methods as the way to share work between the right-hand sides of
the shifted systems (one per well and per receiver).  This is the block form of Algorithm 1
(section 3): the p right-hand sides B = [b_1 .. b_p] start one block basis, B = V_1 R_0 (thin
QR), and step j applies the preconditioner of that step to every column of the block V_j,
U_j = (K + tau_j M)^{-1} V_j, orthogonalises S_j = M U_j against V_1 .. V_j by block
modified Gram-Schmidt (the p x p blocks H_ij = V_i^* S_j), and takes the thin QR of the
remainder, V_{j+1} H_{j+1, j}.  With T_j = blockdiag(tau_1 I_p .. tau_j I_p) the flexible
Arnoldi relation keeps its form,

    (K + z M) U_j = V_{j+1} ( [I; 0] + Hbar_j (z I - T_j) ),

now with (j + 1) p x j p matrices, so every shift z_k again reduces to one small problem:
Y_k minimises || [R_0; 0] - Hbar_j(z_k; T_j) Y ||_F column by column, and X_k = U_j Y_k.
Each column's solution minimises its residual over the whole block space, which contains the
space its own single-RHS run builds.

Readings (the paper gives no block algorithm): a shift is converged when every column meets the
test of Section 4.1, weights_k ||r_kc|| <= tol ||b_c||, and keeps its last Y from then on; the
loop stops once every shift has.  A remainder block of numerically lower rank (a diagonal
entry of its R factor at most 1e-14 of the remainder's largest column norm) ends the loop, as a
zero h_{j+1, j} ends Algorithm 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu


def block_flexible_shifted(K, m, B, taus, shifts, tol, maxit, weights=None, precond=None):
    """Block FGMRES-Sh for the columns of B [N, p] (real or complex).

    ``taus`` are used cyclically (tau_j = taus[(j - 1) % len]); ``precond(tau, V)``, if given,
    replaces the exact solve of (K + tau M) U = V.  Returns a dict with X [nk, N, p],
    iters, res [nk, p] (||r_kc|| / ||b_c||), res_hist [iters, nk, p] (the same after every
    step, for every shift whether converged or not), conv [nk], V [N, (iters + 1) p],
    U [N, iters p], Hbar [(iters + 1) p, iters p], T [iters] and breakdown.
    """
    m = np.asarray(m, dtype=np.float64)
    z = np.asarray(shifts, dtype=np.complex128).ravel()
    nk = z.size
    w = np.ones(nk) if weights is None else np.asarray(weights, dtype=np.float64)
    B = np.asarray(B, dtype=np.complex128)
    if B.ndim == 1:
        B = B[:, None]
    N, p = B.shape
    bnorm = np.linalg.norm(B, axis=0)
    lus = {}

    def solve(tau, Vj):
        key = (float(tau.real), float(tau.imag))
        if key not in lus:
            A = (K + sp.diags(tau * m)).astype(np.complex128).tocsc()
            lus[key] = splu(A, permc_spec="MMD_AT_PLUS_A")
        return lus[key].solve(Vj)

    V = np.zeros((N, (maxit + 1) * p), dtype=np.complex128)
    U = np.zeros((N, maxit * p), dtype=np.complex128)
    H = np.zeros(((maxit + 1) * p, maxit * p), dtype=np.complex128)
    T = np.zeros(maxit, dtype=np.complex128)
    Q0, R0 = np.linalg.qr(B)
    V[:, :p] = Q0
    Y = [None] * nk
    res = np.full((nk, p), np.inf)
    hist = []
    conv = np.zeros(nk, dtype=bool)
    breakdown = False
    j = 0
    for j in range(1, maxit + 1):
        tau = complex(taus[(j - 1) % len(taus)])
        T[j - 1] = tau
        cols = slice((j - 1) * p, j * p)
        Vj = V[:, cols]
        Uj = solve(tau, Vj) if precond is None else np.asarray(precond(tau, Vj), dtype=np.complex128)
        U[:, cols] = Uj
        S = m[:, None] * Uj
        for i in range(j):
            blk = slice(i * p, (i + 1) * p)
            H[blk, cols] = V[:, blk].conj().T @ S
            S = S - V[:, blk] @ H[blk, cols]
        Qn, Rn = np.linalg.qr(S)
        scale = max(np.linalg.norm(S, axis=0).max(), np.finfo(float).tiny)
        breakdown = np.abs(np.diag(Rn)).min() <= 1e-14 * scale
        V[:, j * p:(j + 1) * p] = Qn
        H[j * p:(j + 1) * p, cols] = Rn
        Hb = H[:(j + 1) * p, :j * p]
        G = np.zeros(((j + 1) * p, p), dtype=np.complex128)
        G[:p] = R0
        step_res = np.zeros((nk, p))
        for k in range(nk):
            Tz = np.repeat(z[k] - T[:j], p)
            Hz = np.eye((j + 1) * p, j * p, dtype=np.complex128) + Hb * Tz[None, :]
            Yk = np.linalg.lstsq(Hz, G, rcond=None)[0]
            rk = np.linalg.norm(G - Hz @ Yk, axis=0) / bnorm
            step_res[k] = rk
            if conv[k]:
                continue
            Y[k] = Yk
            res[k] = rk
            if (w[k] * rk).max() <= tol or breakdown:
                conv[k] = True
        hist.append(step_res)
        if conv.all() or breakdown:
            break
    X = np.stack([U[:, :Y[k].shape[0]] @ Y[k] for k in range(nk)])
    return {"x": X, "iters": j, "res": res, "res_hist": np.array(hist), "conv": conv,
            "V": V[:, :(j + 1) * p], "U": U[:, :j * p], "Hbar": H[:(j + 1) * p, :j * p], "T": T[:j],
            "breakdown": breakdown}
