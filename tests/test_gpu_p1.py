"""P1 finite elements on the GPU (Section 2.1's weak form; lt_setup_p1: right triangles,
lumped mass, zero-head walls, the interior vertices as unknowns) against the oracle's
element-by-element assembly.

* The operator K + tau M applied on the GPU against the oracle's assembled matrices, element
  by element (1e-13 of the largest entry), on a GRF field with unequal spacings.
* Heads of the 2D workload's field (65 x 49 cells: 64 x 48 vertices) against the oracle's
  P1 heads (direct solves per shift), FP64 (1e-6) and mixed (1e-5), and with the exact
  shift-and-invert preconditioner (1e-7).
* Refusals: grids of fewer than 3 x 3 cells.
* Sensitivities (lt_adjoint on a P1 handle) to ln kappa and ln S of every cell against the
  oracle's element-by-element discrete adjoint, 2D and 3D, FP64 (1e-6) and mixed (1e-5) of the
  largest entry per (source, receiver, time).  With zero head on every wall the 3D problem
  nears steady state within the workload's second time, where the storage sensitivity is a
  sum of contour terms 1e7 times its size (so its error is set by the solver tolerance
  relative to those terms); the 3D case takes the first time, where they differ by 6e2.
* The V-cycle's contraction on the vertex grid (about 0.25 per cycle, as on cells).
* 3D (the Kuhn subdivision): the operator element by element and heads in both precisions
  against the oracle, and the V-cycle's contraction.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.p1 import assemble_p1, heads_p1, jacobian_p1
from gpu_util import announce, check_heads

pytestmark = pytest.mark.gpu


def _handle(lt, n, h, kappa, S):
    return lt.lt_setup_p1(n, h, torch.tensor(kappa, dtype=torch.float64, device="cuda"),
                          torch.tensor(S, dtype=torch.float64, device="cuda"))


def test_p1_operator_matches_oracle(lt):
    n, h = (21, 14), (0.05, 0.08)
    rng = np.random.default_rng(5)
    kappa = np.exp(1.2 * rng.standard_normal(n[0] * n[1]))
    S = np.exp(rng.standard_normal(n[0] * n[1])) * 1e-4
    announce("P1 operator", n)
    hd = _handle(lt, n, h, kappa, S)
    K, m = assemble_p1(n, h, kappa, S)
    N = (n[0] - 1) * (n[1] - 1)
    assert hd.N == N
    xc = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    x = torch.tensor(np.stack([xc.real, xc.imag], axis=1), dtype=torch.float64, device="cuda").contiguous()
    y = torch.empty_like(x)
    for tau in (0.0, 3e5 + 2e6j, -1e4 + 5e3j):
        lt.lt_apply_operator(hd, 0, tau, x, y, 3)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        got = got[:, 0] + 1j * got[:, 1]
        ref = np.stack([K @ v + tau * m * v for v in xc])
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    hd.close()


@pytest.mark.parametrize("variant", ["fp64", "mixed", "exact"])
def test_p1_heads_match_oracle(lt, variant):
    p = wl.make_problem("C2", n=(65, 49), nsrc=3, nrec=6, ntimes=4)
    n, h = p.n[:2], p.h[:2]
    announce("P1 heads", variant)
    ref = heads_p1(n, h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q)
    hd = _handle(lt, n, h, p.kappa, p.S)
    if variant == "fp64":
        o, bar = lt.make_opts(tol=1e-10), 1e-6
    elif variant == "mixed":
        o, bar = lt.make_opts(tol=1e-8, precision=lt.LT_PREC_MIXED), 1e-5
    else:
        o, bar = lt.make_opts(tol=1e-10, maxit=400, n_tau=2, precond=lt.LT_PRECOND_EXACT), 1e-7
    phi, st = lt.lt_solve(hd, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
    assert st["rc"] == 0
    print(f"[P1] {variant}: iters {st['iters_max']} vcycles {st['vcycles']} levels {st['levels']}", flush=True)
    check_heads(phi.cpu().numpy(), ref, bar, f"P1 65x49 {variant}")
    hd.close()


def test_p1_refusals(lt):
    k = torch.ones(4 * 2, dtype=torch.float64, device="cuda")
    with pytest.raises(lt.LTError) as e:
        lt.lt_setup_p1((4, 2), (0.25, 0.5), k, k)
    assert e.value.code == lt.LT_EINVAL


@pytest.mark.parametrize("case", ["2d", "3d"])
@pytest.mark.parametrize("prec", [0, 1])
def test_p1_sensitivities_match_oracle(lt, case, prec):
    if case == "2d":
        p = wl.make_problem("C2", n=(21, 17), nsrc=2, nrec=3, ntimes=2)
        n, h = p.n[:2], p.h[:2]
    else:
        p = wl.make_problem("C3", n=(9, 8, 7), nsrc=2, nrec=3, ntimes=1)
        n, h = p.n, p.h
    announce("P1 adjoint", case, prec, n)
    hd = _handle(lt, n, h, p.kappa, p.S)
    opts = lt.make_opts(tol=1e-11 if prec == 0 else 1e-9, precision=prec, n_tau=p.n_tau)
    JK, JS, st = lt.lt_adjoint(hd, p.sources, p.q, p.receivers, p.times, p.nz_contour, opts)
    assert st["rc"] == 0
    ncells = int(np.prod(n))
    assert JK.shape[-1] == ncells == hd.nparam
    rK, rS = jacobian_p1(n, h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q)
    bound = 1e-6 if prec == 0 else 1e-5
    for name, got, ref in (("kappa", JK.cpu().numpy(), rK), ("S", JS.cpu().numpy(), rS)):
        scale = np.abs(ref).max(axis=-1, keepdims=True)
        err = (np.abs(got - ref) / scale).max()
        print(f"[P1 adjoint] {case} prec {prec} {name}: iters {st['iters_max']} err {err:.2e}", flush=True)
        assert err <= bound
    hd.close()


def test_p1_vcycle_contracts_like_the_cell_centred_one(lt):
    # the aggregation's wall terms and the prolongation's wall weights follow the vertex grid's
    # wall distance (one spacing on the fine level): the V-cycle reduces a random residual by
    # about a quarter per cycle, as on cells (0.6-0.8 without the correction)
    p = wl.make_problem("C2", n=(129, 129))
    hd = _handle(lt, p.n[:2], p.h[:2], p.kappa, p.S)
    announce("P1 V-cycle contraction")
    rng = np.random.default_rng(0)
    for tau in (0.0, 3.4e6 + 8.3e5j):
        r = torch.tensor(rng.standard_normal((1, 2, hd.N)), dtype=torch.float64, device="cuda").contiguous()
        e, Ae = torch.empty_like(r), torch.empty_like(r)
        rates = []
        for _ in range(8):
            lt.lt_vcycle(hd, tau, lt.LT_PREC_FP64, 2, 2, r, e, 1)
            lt.lt_apply_operator(hd, 0, tau, e, Ae, 1)
            r2 = (r - Ae).contiguous()
            rates.append(float(torch.linalg.vector_norm(r2) / torch.linalg.vector_norm(r)))
            r = r2
        print(f"[P1] tau {tau}: contraction per cycle {[round(v, 3) for v in rates]}", flush=True)
        assert max(rates[4:]) <= 0.4
    hd.close()


def test_p1_3d_operator_and_heads_match_oracle(lt):
    # the Kuhn subdivision of a 3D cell grid: the operator element by element, then heads
    n, h = (9, 7, 6), (1 / 9, 1 / 7, 0.5 / 6)
    rng = np.random.default_rng(8)
    kappa = np.exp(rng.standard_normal(n[0] * n[1] * n[2]))
    S = np.exp(rng.standard_normal(n[0] * n[1] * n[2])) * 1e-4
    announce("P1 3D operator", n)
    hd = _handle(lt, n, h, kappa, S)
    K, m = assemble_p1(n, h, kappa, S)
    assert hd.N == K.shape[0]
    xc = rng.standard_normal((2, hd.N)) + 1j * rng.standard_normal((2, hd.N))
    x = torch.tensor(np.stack([xc.real, xc.imag], axis=1), dtype=torch.float64, device="cuda").contiguous()
    y = torch.empty_like(x)
    for tau in (0.0, 3e5 + 2e6j):
        lt.lt_apply_operator(hd, 0, tau, x, y, 2)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        got = got[:, 0] + 1j * got[:, 1]
        ref = np.stack([K @ v + tau * m * v for v in xc])
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    hd.close()
    p = wl.make_problem("C3", n=(17, 15, 13), nsrc=2, nrec=4, ntimes=2)
    announce("P1 3D heads", p.n)
    ref = heads_p1(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q)
    hd = _handle(lt, p.n, p.h, p.kappa, p.S)
    for prec, tol, bar in ((lt.LT_PREC_FP64, 1e-10, 1e-6), (lt.LT_PREC_MIXED, 1e-8, 1e-5)):
        phi, st = lt.lt_solve(hd, p.sources, p.q, p.times, p.nz_contour, p.receivers,
                              lt.make_opts(tol=tol, precision=prec, n_tau=p.n_tau))
        assert st["rc"] == 0
        print(f"[P1 3D] precision {prec}: iters {st['iters_max']} vcycles {st['vcycles']} levels {st['levels']}",
              flush=True)
        check_heads(phi.cpu().numpy(), ref, bar, f"P1 3D 17x15x13 precision {prec}")
    hd.close()


def _rates(lt, hd, tau, cycles=10):
    rng = np.random.default_rng(0)
    r = torch.tensor(rng.standard_normal((1, 2, hd.N)), dtype=torch.float64, device="cuda").contiguous()
    e, Ae = torch.empty_like(r), torch.empty_like(r)
    rates = []
    for _ in range(cycles):
        lt.lt_vcycle(hd, tau, lt.LT_PREC_FP64, 2, 2, r, e, 1)
        lt.lt_apply_operator(hd, 0, tau, e, Ae, 1)
        r2 = (r - Ae).contiguous()
        rates.append(float(torch.linalg.vector_norm(r2) / torch.linalg.vector_norm(r)))
        r = r2
    return rates


def test_p1_3d_vcycle_contracts_like_the_cell_centred_one(lt):
    # 32 x 32 x 16 vertex unknowns against 32 x 32 x 16 cells of the same field statistics
    tau = 1e5 + 3e5j
    p = wl.make_problem("C3", n=(33, 33, 17))
    hp = _handle(lt, p.n, p.h, p.kappa, p.S)
    q = wl.make_problem("C3", n=(32, 32, 16))
    hf = lt.lt_setup(q.ndim, q.n, q.h, torch.tensor(q.kappa, device="cuda"), torch.tensor(q.S, device="cuda"))
    announce("P1 3D V-cycle contraction")
    rp, rf = _rates(lt, hp, tau), _rates(lt, hf, tau)
    print(f"[P1 3D] contraction per cycle {[round(v, 3) for v in rp]}; cells {[round(v, 3) for v in rf]}",
          flush=True)
    assert max(rp[5:]) <= max(rf[5:]) + 0.1
    hp.close()
    hf.close()
