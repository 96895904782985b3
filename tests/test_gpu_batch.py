"""Batches of problems on uneven grids (lt_solve_batch, lt_adjoint_batch).

Every item of a batch is an independent shifted-system family (Section 3):
the batch must return, bit for bit, what each item returns when solved
alone (the kernels are deterministic), and the heads must match the oracle
to the FP64 bar.  Grids mix 2D and 3D, tile-aligned and ragged shapes."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.heads import heads
from gpu_util import device_problem, device_problem_on_stream, announce, check_heads

pytestmark = pytest.mark.gpu

SMALL = [("C5_128", (64, 64)), ("C5_256", (100, 70)), ("C5_32c", (16, 16, 16)), ("C5_64c", (20, 12, 10))]


def _problems():
    return [wl.make_problem(nm, n=n, nsrc=4, nrec=6) for nm, n in SMALL]


def _item(p, h, o):
    return dict(handle=h, sources=p.sources, q=p.q, times=p.times, nz=p.nz_contour, receivers=p.receivers, opts=o)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_single_solves(lt, prec):
    ps = _problems()
    hs = [device_problem_on_stream(lt, p) for p in ps]
    pr, tol = (lt.LT_PREC_FP64, 1e-9) if prec == "fp64" else (lt.LT_PREC_MIXED, 1e-8)
    opts = [lt.make_opts(tol=tol, precision=pr, n_tau=p.n_tau, maxit=80) for p in ps]
    single = []
    for p, h, o in zip(ps, hs, opts):
        announce("single", p.name, p.n, prec)
        phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
        single.append((phi.clone(), st))
    announce("batch", len(ps), prec)
    outs, stats, rc = lt.lt_solve_batch([_item(p, h, o) for p, h, o in zip(ps, hs, opts)])
    assert rc == 0
    for p, (phi, st), got, bst in zip(ps, single, outs, stats):
        assert bst["rc"] == 0
        assert torch.equal(got, phi), p.name
        assert bst["iters_max"] == st["iters_max"] and bst["vcycles"] == st["vcycles"]
        assert np.array_equal(bst["true_relres"], st["true_relres"])
    for h in hs:
        h.close()


def test_batch_matches_oracle(lt):
    ps = _problems()
    hs = [device_problem_on_stream(lt, p) for p in ps]
    opts = [lt.make_opts(tol=1e-10, precision=lt.LT_PREC_FP64, n_tau=p.n_tau, maxit=80) for p in ps]
    announce("batch vs oracle")
    outs, stats, rc = lt.lt_solve_batch([_item(p, h, o) for p, h, o in zip(ps, hs, opts)])
    for p, st in zip(ps, stats):
        print(p.name, p.n, "rc", st["rc"], "iters", st["iters_max"], "resolves", st["resolves"], "true",
              st["true_relres_max"], flush=True)
    assert rc == 0
    for p, got, st in zip(ps, outs, stats):
        ref = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q, workers=8)
        print(p.name, p.n, "iters", st["iters_max"], "resolves", st["resolves"], "true", st["true_relres_max"],
              flush=True)
        check_heads(got.cpu().numpy(), ref, 1e-6, f"batch {p.name}")
        # rc 0: the FP64 true residual met the weighted tolerance
        assert st["true_relres_max"] <= 1e-10
    for h in hs:
        h.close()


def test_adjoint_batch_equals_single(lt):
    ps = [wl.make_problem("C5_128", n=(24, 20), nsrc=2, nrec=3),
          wl.make_problem("C5_32c", n=(8, 6, 5), nsrc=2, nrec=3)]
    hs = [device_problem_on_stream(lt, p) for p in ps]
    o = lt.make_opts(tol=1e-10, precision=lt.LT_PREC_FP64, n_tau=1)
    single = []
    for p, h in zip(ps, hs):
        announce("adjoint single", p.n)
        dK, dS, st = lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, o)
        single.append((dK.clone(), dS.clone()))
    announce("adjoint batch")
    outs, stats, rc = lt.lt_adjoint_batch([dict(handle=h, sources=p.sources, q=p.q, receivers=p.receivers,
                                                times=p.times, nz=p.nz_contour, opts=o) for p, h in zip(ps, hs)])
    assert rc == 0
    for (dK, dS), (gK, gS) in zip(single, outs):
        assert torch.equal(gK, dK) and torch.equal(gS, dS)
    for h in hs:
        h.close()


def test_batch_rejects_repeated_handle(lt):
    p = wl.make_problem("C5_128", n=(16, 16), nsrc=1, nrec=1)
    h = device_problem_on_stream(lt, p)
    it = _item(p, h, None)
    with pytest.raises(lt.LTError) as e:
        lt.lt_solve_batch([it, it])
    assert e.value.code == lt.LT_EINVAL
    h.close()


def test_source_groups_equal_one_solve(lt):
    """The benchmark's split: the sources of one problem solved as two concurrent groups
    (two handles on the same grid, one lt_solve_batch call) give, bit for bit, the heads
    and iteration counts of one lt_solve over all sources -- every right-hand side has
    its own basis, so grouping changes no arithmetic."""
    p = wl.make_problem("C2", n=(96, 64), nsrc=6, nrec=5)
    hs = [device_problem_on_stream(lt, p) for _ in range(2)]
    o = lt.make_opts(tol=1e-8, precision=lt.LT_PREC_MIXED, n_tau=1, relax=3.0)
    announce("source groups", p.n)
    whole, st = lt.lt_solve(hs[0], p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
    whole = whole.cpu().numpy()
    phi = torch.empty((len(p.sources), len(p.receivers), len(p.times)), dtype=torch.float64, device="cuda")
    cuts = [slice(0, 3), slice(3, 6)]
    items = [dict(handle=h, sources=p.sources[c], q=p.q, times=p.times, nz=p.nz_contour, receivers=p.receivers,
                  opts=o, phi_out=phi[c]) for h, c in zip(hs, cuts)]
    for _ in range(2):  # the second call reuses every workspace
        _, sts, rc = lt.lt_solve_batch(items)
        assert rc == 0
        np.testing.assert_array_equal(phi.cpu().numpy(), whole)
        its = np.concatenate([s["iters_per_rhs"] for s in sts])
        np.testing.assert_array_equal(its, st["iters_per_rhs"])
    for h in hs:
        h.close()


def test_3d_rhs_independent_of_their_groups(lt):
    """The 3D multigrid kernels serve the active right-hand sides in groups (eight in a
    half-sweep, four in the transfers and the refinement update), formed afresh every cycle
    from the list of those still refining.  A right-hand side's arithmetic must not depend
    on which others share its group: each source solved alone gives, bit for bit, its heads
    and iteration count from the solve over all sources, where the sources' inner
    refinements (and outer iterations) end at different steps, so they drop out of the
    groups one by one."""
    p = wl.make_problem("C3", n=(32, 24, 16), nsrc=11, nrec=6)
    h = device_problem(lt, p)
    o = lt.make_opts(tol=1e-9, precision=lt.LT_PREC_MIXED, n_tau=p.n_tau, relax=0.3, nu1=2, nu2=2)
    announce("3D groups", p.n, len(p.sources))
    whole, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
    whole = whole.cpu().numpy()
    its = np.asarray(st["iters_per_rhs"])
    print(f"[3D groups] outer iterations per source {its.tolist()}", flush=True)
    for s in range(len(p.sources)):
        q = p.q[s:s + 1] if np.ndim(p.q) else p.q
        one, st1 = lt.lt_solve(h, p.sources[s:s + 1], q, p.times, p.nz_contour, p.receivers, o)
        np.testing.assert_array_equal(one.cpu().numpy()[0], whole[s])
        assert st1["iters_per_rhs"][0] == its[s]
    h.close()
