"""The linearised water-table boundary (eqn:timedomain, third condition; the
boundary term of M in Section 2.1) on the HIP path against the oracle, which
is pinned to closed forms and central differences on the CPU.

A water-table face adds S_y A to the lumped mass of the cell behind it and
carries no conductive flux.  Specific yields are set so that the face
storage outweighs the volume storage of a whole column (the unconfined
regime, S_y >> S_s b), which is where the boundary changes the heads most.
Bars as for the other boundaries: operator 1e-13 relative, heads 1e-6 (FP64)
and 1e-5 (mixed) relative per source, sensitivities 1e-6 of each map's
largest entry."""
from dataclasses import replace

import numpy as np
import pytest

import workloads as wl
from oracle.fv import assemble
from oracle.heads import heads_problem
from oracle.jacobian import jacobian
from gpu_util import device_problem, rel_err_per_source, check_heads, announce

pytestmark = pytest.mark.gpu

CASES = {
    # unconfined 3D aquifer: fixed-head sides, no-flux base, water table on top
    "3d_16x12x8": dict(name="C3", kw=dict(n=(16, 12, 8), nsrc=2, nrec=4), bc=(0, 0, 0, 0, 1, 2), sy=1e-3),
    "3d_ragged_10x6x5": dict(name="C3", kw=dict(n=(10, 6, 5), nsrc=2, nrec=4), bc=(1, 0, 0, 1, 1, 2), sy=1e-3),
    # 2D section: the +y wall is the water table, the others fixed or closed
    "2d_ragged_30x22": dict(name="C2", kw=dict(n=(30, 22), nsrc=2, ntimes=4), bc=(0, 1, 0, 2, 0, 0), sy=5e-5),
    "2d_64x64_closed": dict(name="C2", kw=dict(n=(64, 64), nsrc=2), bc=(1, 1, 1, 2, 0, 0), sy=2e-5),
}


def _problem(case):
    spec = CASES[case]
    p = wl.make_problem(spec["name"], **spec["kw"])
    return replace(p, bc=spec["bc"], sy=spec["sy"])


@pytest.mark.parametrize("case", ["3d_ragged_10x6x5", "2d_ragged_30x22"])
def test_operator_matches_oracle(lt, case):
    import torch
    p = _problem(case)
    announce("water-table operator", case)
    h = device_problem(lt, p)
    K, m = assemble(p.n, p.h, p.kappa, p.S, p.bc, ndim=p.ndim, sy=p.sy)
    rng = np.random.default_rng(2)
    z = rng.standard_normal((3, 2, p.N))
    x = torch.tensor(z, dtype=torch.float64, device="cuda").contiguous()
    xc = z[:, 0] + 1j * z[:, 1]
    y = torch.empty_like(x)
    for tau in (3e5 + 2e6j, -1e4 + 5e3j):
        lt.lt_apply_operator(h, 0, tau, x, y, 3)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        got = got[:, 0] + 1j * got[:, 1]
        ref = np.stack([K @ v + tau * m * v for v in xc])
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    h.close()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [0, 1])
def test_heads_match_oracle(lt, case, prec):
    p = _problem(case)
    announce("water-table heads", case, prec, p.n)
    ref = heads_problem(p)
    # the boundary matters: the same problem with a closed face gives other heads
    closed = heads_problem(replace(p, bc=tuple(1 if b == 2 else b for b in p.bc)))
    assert rel_err_per_source(closed, ref).min() > 1e-3
    h = device_problem(lt, p)
    tol = 1e-10 if prec == 0 else 1e-8
    opts = lt.make_opts(tol=tol, precision=prec, n_tau=p.n_tau)
    phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, opts)
    print(case, prec, "iters", st["iters_max"], "resolves", st["resolves"], flush=True)
    assert st["rc"] == 0
    check_heads(phi.cpu().numpy(), ref, 1e-6 if prec == 0 else 1e-5, f"water table {case} prec {prec}")
    assert st["true_relres_max"] <= tol
    h.close()


@pytest.mark.parametrize("case", ["3d_ragged_10x6x5", "2d_ragged_30x22"])
def test_sensitivities_match_oracle(lt, case):
    """The storage sensitivity differentiates S V only: on the water-table cells it
    differs from the derivative of the whole mass."""
    p = _problem(case)
    if p.ndim == 2:
        p = replace(p, times=p.times[:2])
    announce("water-table adjoint", case, p.n)
    h = device_problem(lt, p)
    opts = lt.make_opts(tol=1e-11, precision=0, n_tau=p.n_tau)
    JK, JS, st = lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, opts)
    assert st["rc"] == 0
    rK, rS = jacobian(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q,
                      bc=p.bc, ndim=p.ndim, sy=p.sy)
    for got, ref in ((JK.cpu().numpy(), rK), (JS.cpu().numpy(), rS)):
        scale = np.abs(ref).max(axis=-1, keepdims=True)
        err = (np.abs(got - ref) / scale).max()
        print(case, "adjoint err", err, flush=True)
        assert err <= 1e-6
    h.close()


def test_batch_mixes_boundaries_bit_exactly(lt):
    """One lt_solve_batch call over a water-table problem and a zero-head problem on other grids
    gives, bit for bit, the heads of the two single calls (the boundary lives in the handle)."""
    from gpu_util import device_problem_on_stream
    pw = _problem("2d_ragged_30x22")
    pd = wl.make_problem("C3", n=(10, 6, 5), nsrc=2, nrec=4)
    announce("water-table batch", pw.n, pd.n)
    hs = [device_problem_on_stream(lt, q) for q in (pw, pd)]
    o = lt.make_opts(tol=1e-10, precision=lt.LT_PREC_FP64, n_tau=2)
    singles = [lt.lt_solve(h, q.sources, q.q, q.times, q.nz_contour, q.receivers, o)[0].cpu().numpy()
               for h, q in zip(hs, (pw, pd))]
    items = [dict(handle=h, sources=q.sources, q=q.q, times=q.times, nz=q.nz_contour, receivers=q.receivers,
                  opts=o) for h, q in zip(hs, (pw, pd))]
    phis, sts, rc = lt.lt_solve_batch(items)
    assert rc == 0
    for got, want in zip(phis, singles):
        np.testing.assert_array_equal(got.cpu().numpy(), want)
    ref = heads_problem(pw)
    check_heads(singles[0], ref, 1e-6, "water-table batch")
    for h in hs:
        h.close()


def test_fom_variant_with_water_table(lt):
    p = _problem("3d_ragged_10x6x5")
    announce("water-table fom", p.n)
    ref = heads_problem(p)
    h = device_problem(lt, p)
    opts = lt.make_opts(tol=1e-10, precision=0, n_tau=p.n_tau, method=lt.LT_METHOD_FOM)
    phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, opts)
    assert st["rc"] == 0
    check_heads(phi.cpu().numpy(), ref, 1e-6, "water-table fom")
    h.close()
