"""Captured refinement steps (opts.graph) against kernel-by-kernel launches.

A captured step replays the same kernels on the same buffers, so every
result must be bit-identical to the launched path: heads, iteration and
V-cycle counts, true residuals and sensitivities.  The cases replay each
graph many times with host work and synchronisation between replays, reuse
graphs across calls, and retire them when a larger batch of right-hand
sides reallocates the workspaces."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_util import device_problem_on_stream, announce

pytestmark = pytest.mark.gpu

CASES = [("C2", (64, 48), 1), ("C3", (16, 12, 10), 3), ("C1", (32, 32), 2)]


def _solve(lt, h, p, graph, prec, nsrc=None):
    tol = 1e-9 if prec == lt.LT_PREC_FP64 else 1e-7
    o = lt.make_opts(tol=tol, precision=prec, n_tau=p.n_tau, maxit=80, graph=graph)
    src = p.sources if nsrc is None else p.sources[:nsrc]
    return lt.lt_solve(h, src, p.q, p.times, p.nz_contour, p.receivers, o)


def _same(a, b):
    (pa, sa), (pb, sb) = a, b
    assert torch.equal(pa, pb)
    assert sa["iters_max"] == sb["iters_max"] and sa["vcycles"] == sb["vcycles"]
    assert np.array_equal(sa["true_relres"], sb["true_relres"])


@pytest.mark.parametrize("name,n,ntau", CASES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_equals_launched(lt, name, n, ntau, prec):
    p = wl.make_problem(name, n=n, nsrc=4, ntimes=3)
    p.n_tau = ntau
    pr = lt.LT_PREC_FP64 if prec == "fp64" else lt.LT_PREC_MIXED
    h = device_problem_on_stream(lt, p)
    announce("graph", name, n, prec, ntau)
    ref = _solve(lt, h, p, 0, pr)
    ref = (ref[0].clone(), ref[1])
    g1 = _solve(lt, h, p, 1, pr)
    _same(g1, ref)
    g2 = _solve(lt, h, p, 1, pr)  # graphs reused across calls
    _same(g2, ref)
    # fewer right-hand sides: new graphs at the same workspace generation
    small_ref = _solve(lt, h, p, 0, pr, nsrc=2)
    small_ref = (small_ref[0].clone(), small_ref[1])
    _same(_solve(lt, h, p, 1, pr, nsrc=2), small_ref)
    h.close()


def test_graphs_retired_when_workspaces_grow(lt):
    p = wl.make_problem("C2", n=(64, 48), ntimes=2)
    h = device_problem_on_stream(lt, p)
    announce("graph retire")
    few = _solve(lt, h, p, 1, lt.LT_PREC_MIXED, nsrc=2)
    few = (few[0].clone(), few[1])
    many_g = _solve(lt, h, p, 1, lt.LT_PREC_MIXED)  # 8 sources: workspaces grow
    many_g = (many_g[0].clone(), many_g[1])
    _same(_solve(lt, h, p, 0, lt.LT_PREC_MIXED), many_g)
    _same(_solve(lt, h, p, 1, lt.LT_PREC_MIXED, nsrc=2), few)
    h.close()


def test_graph_adjoint_equals_launched(lt):
    p = wl.make_problem("C3", n=(8, 8, 6), nsrc=2, nrec=3, ntimes=1)
    h = device_problem_on_stream(lt, p)
    announce("graph adjoint")
    out = {}
    for g in (0, 1):
        o = lt.make_opts(tol=1e-10, precision=lt.LT_PREC_FP64, n_tau=3, graph=g)
        dK, dS, st = lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, o)
        out[g] = (dK.clone(), dS.clone())
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    h.close()
