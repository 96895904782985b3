"""Pins of the oracle's block flexible shifted GMRES, each against something other than itself:

* the solutions against direct solves of each shifted system, column by column;
* the block flexible Arnoldi relation at a shift that is not solved, and the orthonormality of
  the block basis (sparse products);
* a block of one column against the pinned single right-hand-side Algorithm 1 (same steps, same
  solutions);
* every column's residual after every step at most its own single right-hand-side run's (the
  block space contains that run's space, and GMRES minimises over it);
* B = I (a block as wide as the grid): the first block of the preconditioned basis spans every
  solution, so one step solves every shift.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve

from oracle.block import block_flexible_shifted
from oracle.contour import talbot_nodes
from oracle.fv import assemble, point_weights
from oracle.krylov import flexible_shifted, tau_schedule
from workloads.configs import T_D, make_problem


def _problem(n=(20, 18), nsrc=4, seed=7):
    p = make_problem("W1", n=n, seed=seed, var=1.6)
    K, m = assemble(p.n, p.h, p.kappa, p.S)
    rng = np.random.default_rng(seed)
    pts = np.column_stack([rng.uniform(0.1, 0.9, nsrc), rng.uniform(0.1, 0.9, nsrc), np.zeros(nsrc)])
    B = point_weights(p.n, p.h, pts).toarray().T  # wells as the oracle discretises them
    z, _ = talbot_nodes(16, 0.3 * T_D)
    return K, m, B, z


def test_block_solutions_match_direct_solves():
    K, m, B, z = _problem()
    out = block_flexible_shifted(K, m, B, tau_schedule(z, 2), z, tol=1e-10, maxit=60)
    assert out["conv"].all()
    for k in range(z.size):
        A = (K + sp.diags(z[k] * m)).tocsc()
        ref = spsolve(A, B.astype(np.complex128))
        for c in range(B.shape[1]):
            assert np.linalg.norm(out["x"][k][:, c] - ref[:, c]) <= 1e-8 * np.linalg.norm(ref[:, c])
            r = B[:, c] - A @ out["x"][k][:, c]
            assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(B[:, c])


def test_block_arnoldi_relation_and_orthonormality():
    K, m, B, z = _problem()
    out = block_flexible_shifted(K, m, B, tau_schedule(z, 2), z, tol=1e-30, maxit=8)
    V, U, Hb, T = out["V"], out["U"], out["Hbar"], out["T"]
    p = B.shape[1]
    j = out["iters"]
    assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() <= 1e-12
    sigma = 3.7e4 - 2.2e4j  # not a shift of the solve
    lhs = (K + sp.diags(sigma * m)) @ U
    Hz = np.eye((j + 1) * p, j * p) + Hb * np.repeat(sigma - T, p)[None, :]
    rhs = V @ Hz
    assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(lhs).max()
    # the first block spans B
    assert np.linalg.norm(V[:, :p] @ (V[:, :p].conj().T @ B) - B) <= 1e-12 * np.linalg.norm(B)


def test_block_of_one_is_algorithm_1():
    K, m, B, z = _problem(nsrc=1)
    taus = tau_schedule(z, 2)
    blk = block_flexible_shifted(K, m, B, taus, z, tol=1e-9, maxit=60)
    one = flexible_shifted(K, m, B[:, 0], taus, z, tol=1e-9, maxit=60)
    assert blk["iters"] == one["iters"]
    for k in range(z.size):
        assert np.linalg.norm(blk["x"][k][:, 0] - one["x"][k]) <= 1e-10 * np.linalg.norm(one["x"][k])
    assert np.abs(blk["res"][:, 0] - one["res"]).max() <= 1e-8 * max(one["res"].max(), 1e-12) + 1e-15


def test_every_column_at_most_its_single_residual():
    K, m, B, z = _problem(nsrc=3)
    taus = tau_schedule(z, 2)
    blk = block_flexible_shifted(K, m, B, taus, z, tol=1e-30, maxit=10)
    for c in range(B.shape[1]):
        one = block_flexible_shifted(K, m, B[:, c:c + 1], taus, z, tol=1e-30, maxit=10)
        steps = min(blk["iters"], one["iters"])
        h1, hb = one["res_hist"][:steps, :, 0], blk["res_hist"][:steps, :, c]
        assert np.all(hb <= h1 * (1 + 1e-8) + 1e-14)
        # and strictly smaller somewhere: the block space is larger
        assert (hb < 0.9 * h1).any()


def test_identity_block_solves_in_one_step():
    p = make_problem("W1", n=(4, 3), seed=3, var=1.0)
    K, m = assemble(p.n, p.h, p.kappa, p.S)
    N = K.shape[0]
    z, _ = talbot_nodes(8, 0.3 * T_D)
    out = block_flexible_shifted(K, m, np.eye(N), [z[0]], z, tol=1e-10, maxit=5)
    assert out["iters"] == 1 and out["conv"].all()
    for k in range(z.size):
        ref = np.linalg.inv((K + sp.diags(z[k] * m)).toarray())
        assert np.abs(out["x"][k] - ref).max() <= 1e-9 * np.abs(ref).max()
