"""Block flexible GMRES for shifted systems on the GPU (lt_shifted_solve_block) against the
oracle's block algorithm and direct solves.

* Exact shift-and-invert preconditioners: the solutions of every shift and column against the
  oracle's block FGMRES-Sh (same blocks, same preconditioner shifts) element by element (1e-8 of
  each column's largest entry) and against direct solves; the steps agree with the oracle's
  within one (the tolerance test sits on rounding); blocks of 1, 4 and 8 columns; and a 3D grid.
* Blocks need fewer steps than single right-hand sides (the block space contains each single
  space), on the same problem.
* Multigrid preconditioners (V-cycles to tol / 100, FP64 or FP32 under FP64 refinement), 2D and
  3D: solutions against direct solves (1e-6) and FP64 true residuals within tol.
* Weighted shifts; refusals (a block that does not divide nvec, a block of 17, a zero column,
  multigrid with a negative real preconditioner shift, x overlapping b).
* The widest block (16 columns) at its step cap (7): LT_WNOTCONV, and the solutions are the
  oracle's after the same 7 steps.
* A P1 handle (lumped mass): multigrid block solves against direct solves of the oracle's
  element assembly.
* A block with a repeated column stops after one step (LT_WNOTCONV, finite output); the other
  block converges as before.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch
from scipy.sparse.linalg import splu

import workloads as wl
from gpu_util import announce, device_problem
from oracle.block import block_flexible_shifted
from oracle.contour import talbot_nodes
from oracle.fv import assemble
from oracle.krylov import tau_schedule
from workloads.configs import T_D

pytestmark = pytest.mark.gpu


def _setup(lt, name="W1", n=(40, 36), nsrc=8, seed=11):
    # right-hand sides: unit vectors at seeded random cells away from the walls, and one smooth
    # column (both sides take the same columns; none comes from either side's arithmetic)
    p = wl.make_problem(name, n=n)
    K, m = assemble(p.n, p.h, p.kappa, p.S, bc=p.bc, sy=p.sy)
    rng = np.random.default_rng(seed)
    N = K.shape[0]
    B = np.zeros((N, nsrc))
    B[rng.choice(N, size=nsrc - 1, replace=False), np.arange(nsrc - 1)] = 1.0
    B[:, nsrc - 1] = np.sin(np.linspace(0.0, 7.0, N)) + 0.5
    hd = device_problem(lt, p)
    assert hd.N == K.shape[0]
    b = torch.zeros((nsrc, 2, hd.N), dtype=torch.float64, device="cuda")
    b[:, 0, :] = torch.tensor(B.T, dtype=torch.float64, device="cuda")
    return p, K, m, B, hd, b


def _direct(K, m, z, B):
    return [splu((K + sp.diags(zk * m)).astype(np.complex128).tocsc()).solve(B.astype(np.complex128)) for zk in z]


def _cplx(x):
    x = x.cpu().numpy()
    return x[:, :, 0, :] + 1j * x[:, :, 1, :]  # [nk, nvec, N]


@pytest.mark.parametrize("block", [1, 4, 8])
def test_block_exact_matches_oracle(lt, block):
    p, K, m, B, hd, b = _setup(lt)
    z, _ = talbot_nodes(16, 0.3 * T_D)
    taus = tau_schedule(z, 2)
    announce("block exact", block, p.n)
    o = lt.make_opts(tol=1e-10, maxit=60, precond=lt.LT_PRECOND_EXACT)
    x, st = lt.lt_shifted_solve_block(hd, z, b, block, taus, o)
    assert st["rc"] == 0
    got = _cplx(x)
    ref_d = _direct(K, m, z, B)
    steps = []
    for c0 in range(0, B.shape[1], block):
        orc = block_flexible_shifted(K, m, B[:, c0:c0 + block], taus, z, tol=1e-10, maxit=60)
        steps.append(orc["iters"])
        for k in range(z.size):
            for c in range(block):
                g, r = got[k, c0 + c], orc["x"][k][:, c]
                assert np.abs(g - r).max() <= 1e-8 * np.abs(r).max()
                d = ref_d[k][:, c0 + c]
                assert np.abs(g - d).max() <= 1e-8 * np.abs(d).max()
    gsteps = st["iters_per_rhs"][::block]
    print(f"[block exact] p {block}: gpu steps {list(gsteps)} oracle {steps}; true residual "
          f"{st['true_relres_max']:.2e}; factorisations {st['factorizations']}", flush=True)
    assert all(abs(int(a) - b_) <= 1 for a, b_ in zip(gsteps, steps))
    assert st["true_relres_max"] <= 1e-9
    hd.close()


def test_blocks_take_fewer_steps(lt):
    p, K, m, B, hd, b = _setup(lt, n=(48, 40))
    z, _ = talbot_nodes(16, 0.3 * T_D)
    taus = tau_schedule(z, 2)
    announce("block steps", p.n)
    o = lt.make_opts(tol=1e-8, maxit=60, precond=lt.LT_PRECOND_EXACT)
    _, s1 = lt.lt_shifted_solve_block(hd, z, b, 1, taus, o)
    _, s4 = lt.lt_shifted_solve_block(hd, z, b, 4, taus, o)
    print(f"[block steps] single {list(s1['iters_per_rhs'])} blocks of 4 {list(s4['iters_per_rhs'])}", flush=True)
    assert s1["rc"] == 0 and s4["rc"] == 0
    assert s4["iters_max"] < s1["iters_max"]
    hd.close()


@pytest.mark.parametrize("case", ["2d", "3d"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_block_multigrid_matches_direct_solves(lt, case, prec):
    if case == "2d":
        p, K, m, B, hd, b = _setup(lt, "C2", n=(64, 48), nsrc=8)
    else:
        p, K, m, B, hd, b = _setup(lt, "C3", n=(24, 20, 16), nsrc=4)
    z, _ = talbot_nodes(16, p.times[0])
    # multigrid needs Re(tau) >= 0: the shift of largest real part, and its imaginary part
    # alone for the far end of the contour
    zr = z[np.argmax(z.real)]
    zi = z[np.argmax(np.abs(z.imag))]
    taus = [zr, complex(0.0, zi.imag)]
    announce("block gmg", case, prec, p.n)
    tol = 1e-8
    o = lt.make_opts(tol=tol, maxit=100, precond=lt.LT_PRECOND_GMG,
                     precision=lt.LT_PREC_MIXED if prec == "mixed" else lt.LT_PREC_FP64)
    x, st = lt.lt_shifted_solve_block(hd, z, b, 4, taus, o)
    got = _cplx(x)
    ref = _direct(K, m, z, B)
    err = max(np.abs(got[k, c] - ref[k][:, c]).max() / np.abs(ref[k][:, c]).max()
              for k in range(z.size) for c in range(B.shape[1]))
    print(f"[block gmg] {case} {prec}: rc {st['rc']} steps {st['iters_max']} vcycles {st['vcycles']} "
          f"true residual {st['true_relres_max']:.2e} err {err:.2e}", flush=True)
    assert st["rc"] == 0
    assert st["true_relres_max"] <= tol
    assert err <= 1e-6
    hd.close()


def test_block_weights_and_refusals(lt):
    p, K, m, B, hd, b = _setup(lt, nsrc=4)
    z, w = talbot_nodes(12, 0.3 * T_D)
    taus = tau_schedule(z, 2)
    wt = np.abs(w)
    wt = wt / wt.max()
    o = lt.make_opts(tol=1e-8, maxit=60, precond=lt.LT_PRECOND_EXACT)
    x, st = lt.lt_shifted_solve_block(hd, z, b, 2, taus, o, weights=wt)
    assert st["rc"] == 0
    tr = st["true_relres"]  # [nvec][nshift]
    assert (tr * wt[None, :]).max() <= 1e-8
    orc = block_flexible_shifted(K, m, B[:, :2], taus, z, tol=1e-8, maxit=60, weights=wt)
    got = _cplx(x)
    for k in range(z.size):
        assert np.abs(got[k, 0] - orc["x"][k][:, 0]).max() <= 1e-7 * np.abs(orc["x"][k][:, 0]).max() + 1e-300
    for blk in (3, 17):
        with pytest.raises(lt.LTError) as e:
            lt.lt_shifted_solve_block(hd, z, b, blk, taus, o)
        assert e.value.code == lt.LT_EINVAL
    with pytest.raises(lt.LTError) as e:  # multigrid with a negative real preconditioner shift
        lt.lt_shifted_solve_block(hd, z, b, 2, [complex(-1e4, 1e4)],
                                  lt.make_opts(tol=1e-8, maxit=10, precond=lt.LT_PRECOND_GMG))
    assert e.value.code == lt.LT_EINVAL
    xo = torch.empty((z.size + 1, b.shape[0], 2, hd.N), dtype=torch.float64, device="cuda")
    with pytest.raises(lt.LTError) as e:  # x overlapping b
        lt.lt_shifted_solve_block(hd, z, xo[1], 2, taus, o, x=xo[1:])  # refused before b is read
    assert e.value.code == lt.LT_EINVAL
    b0 = b.clone()
    b0[1].zero_()
    with pytest.raises(lt.LTError) as e:
        lt.lt_shifted_solve_block(hd, z, b0, 2, taus, o)
    assert e.value.code == lt.LT_EINVAL
    hd.close()


def test_widest_block_stops_at_its_step_cap(lt):
    # 16 columns: one (block, shift)'s least-squares columns fill 32 KB of LDS after 7 steps; the
    # call stops there, reports LT_WNOTCONV, and its solutions are the oracle's after 7 steps
    p, K, m, B, hd, b = _setup(lt, nsrc=16)
    z, _ = talbot_nodes(16, 0.3 * T_D)
    taus = tau_schedule(z, 2)
    announce("block 16 cap", p.n)
    o = lt.make_opts(tol=1e-14, maxit=60, precond=lt.LT_PRECOND_EXACT)
    x, st = lt.lt_shifted_solve_block(hd, z, b, 16, taus, o)
    assert st["rc"] == lt.LT_WNOTCONV
    assert st["iters_max"] == 7 and (st["iters_per_rhs"] == 7).all()
    orc = block_flexible_shifted(K, m, B, taus, z, tol=1e-14, maxit=7)
    got = _cplx(x)
    err = max(np.abs(got[k, c] - orc["x"][k][:, c]).max() / np.abs(orc["x"][k][:, c]).max()
              for k in range(z.size) for c in range(16))
    print(f"[block 16] steps {st['iters_max']} true residual {st['true_relres_max']:.2e} err {err:.2e}", flush=True)
    assert err <= 1e-8
    hd.close()


def test_block_on_p1_elements(lt):
    # a P1 handle (lumped mass, interior vertices): FP64 multigrid, against direct solves of the
    # oracle's element assembly
    from oracle.p1 import assemble_p1
    p = wl.make_problem("C2", n=(33, 25))
    n, h = p.n[:2], p.h[:2]
    K, m = assemble_p1(n, h, p.kappa, p.S)
    hd = lt.lt_setup_p1(n, h, torch.tensor(p.kappa, dtype=torch.float64, device="cuda"),
                        torch.tensor(p.S, dtype=torch.float64, device="cuda"))
    assert hd.N == K.shape[0]
    rng = np.random.default_rng(4)
    B = np.zeros((hd.N, 4))
    B[rng.choice(hd.N, size=4, replace=False), np.arange(4)] = 1.0
    b = torch.zeros((4, 2, hd.N), dtype=torch.float64, device="cuda")
    b[:, 0, :] = torch.tensor(B.T, dtype=torch.float64, device="cuda")
    z, _ = talbot_nodes(16, p.times[3])
    zr, zi = z[np.argmax(z.real)], z[np.argmax(np.abs(z.imag))]
    announce("block p1", n)
    x, st = lt.lt_shifted_solve_block(hd, z, b, 2, [zr, complex(0.0, zi.imag)],
                                      lt.make_opts(tol=1e-8, maxit=100, precond=lt.LT_PRECOND_GMG))
    got = _cplx(x)
    ref = _direct(K, m, z, B)
    err = max(np.abs(got[k, c] - ref[k][:, c]).max() / np.abs(ref[k][:, c]).max()
              for k in range(z.size) for c in range(4))
    print(f"[block p1] rc {st['rc']} steps {st['iters_max']} true residual {st['true_relres_max']:.2e} "
          f"err {err:.2e}", flush=True)
    assert st["rc"] == 0 and err <= 1e-6
    hd.close()


def test_block_with_a_repeated_column_stops_alone(lt):
    # a block whose columns are linearly dependent (one column twice) loses rank at its first QR:
    # that block stops after one step (LT_WNOTCONV from its true residuals, finite output); the
    # other block is unaffected
    p, K, m, B, hd, b = _setup(lt, nsrc=8)
    b[5] = b[4]
    B[:, 5] = B[:, 4]
    z, _ = talbot_nodes(16, 0.3 * T_D)
    taus = tau_schedule(z, 2)
    announce("block repeated column", p.n)
    x, st = lt.lt_shifted_solve_block(hd, z, b, 4, taus, lt.make_opts(tol=1e-10, maxit=60,
                                                                      precond=lt.LT_PRECOND_EXACT))
    got = _cplx(x)
    print(f"[block repeated] rc {st['rc']} steps {list(st['iters_per_rhs'])}", flush=True)
    assert st["rc"] == lt.LT_WNOTCONV
    assert np.isfinite(got).all()
    assert (st["iters_per_rhs"][4:] == 1).all() and (st["iters_per_rhs"][:4] > 1).all()
    ref = _direct(K, m, z, B)
    for k in range(z.size):
        for c in range(4):
            assert np.abs(got[k, c] - ref[k][:, c]).max() <= 1e-8 * np.abs(ref[k][:, c]).max()
    hd.close()


def test_block_exact_3d_matches_oracle(lt):
    # a 3D grid (the exact preconditioner's block-tridiagonal factorisation over planes)
    p, K, m, B, hd, b = _setup(lt, "C3", n=(12, 10, 8), nsrc=4)
    z, _ = talbot_nodes(16, p.times[0])
    taus = tau_schedule(z, 2)
    announce("block exact 3d", p.n)
    x, st = lt.lt_shifted_solve_block(hd, z, b, 4, taus, lt.make_opts(tol=1e-10, maxit=60,
                                                                      precond=lt.LT_PRECOND_EXACT))
    assert st["rc"] == 0
    orc = block_flexible_shifted(K, m, B, taus, z, tol=1e-10, maxit=60)
    got = _cplx(x)
    err = max(np.abs(got[k, c] - orc["x"][k][:, c]).max() / np.abs(orc["x"][k][:, c]).max()
              for k in range(z.size) for c in range(4))
    print(f"[block exact 3d] steps {st['iters_max']} oracle {orc['iters']} err {err:.2e}", flush=True)
    assert abs(st["iters_max"] - orc["iters"]) <= 1 and err <= 1e-8
    hd.close()
