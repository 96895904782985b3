"""Edge cases of the boundary on the GPU: bad arguments are rejected before any
work, a tolerance that maxit cannot reach returns LT_WNOTCONV with the best
estimate and its true residuals, the smallest grids and single sources and
receivers work, wells on walls and corners are accepted, zero pumping gives
zero heads, and heads scale linearly with the pumping rate (Section 2.1:
the semi-discrete system is linear in q)."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.heads import heads
from gpu_util import device_problem, announce, check_heads

pytestmark = pytest.mark.gpu


def test_bad_arguments_raise(lt):
    p = wl.make_problem("C1", n=(16, 16), ntimes=2)
    h = device_problem(lt, p)
    announce("bad arguments")
    cases = [
        dict(times=[-1.0]),                       # non-positive time
        dict(times=[0.0]),
        dict(nz=7),                               # odd contour
        dict(nz=0),
        dict(opts=lt.make_opts(tol=-1.0)),
        dict(opts=lt.make_opts(maxit=0)),
        dict(opts=lt.make_opts(precision=7)),
        dict(opts=lt.make_opts(nu1=0, nu2=0)),
        dict(opts=lt.make_opts(graph=2)),
        dict(opts=lt.make_opts(method=2)),
        dict(q=float("nan")),
    ]
    for c in cases:
        kw = dict(times=p.times, nz=p.nz_contour, opts=None, q=p.q)
        kw.update(c)
        with pytest.raises(lt.LTError) as e:
            lt.lt_solve(h, p.sources, kw["q"], kw["times"], kw["nz"], p.receivers, kw["opts"])
        assert e.value.code == lt.LT_EINVAL, c
    # the learned preconditioner needs a network and a grid it supports
    with pytest.raises(lt.LTError):
        lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers,
                    lt.make_opts(precond=lt.LT_PRECOND_UNET_GMG))
    # at most 1000 right-hand sides per call (sources; sources and receivers for the adjoint)
    many = np.tile(np.asarray(p.sources, dtype=np.float64)[:1], (1001, 1))
    with pytest.raises(lt.LTError) as e:
        lt.lt_solve(h, many, p.q, p.times, p.nz_contour, p.receivers)
    assert e.value.code == lt.LT_EINVAL
    with pytest.raises(lt.LTError) as e:
        lt.lt_adjoint(h, many[:999], p.q, many[:2], p.times, p.nz_contour)
    assert e.value.code == lt.LT_EINVAL
    h.close()


def test_maxit_too_small_warns_with_best_estimate(lt):
    p = wl.make_problem("C1", ntimes=2)
    h = device_problem(lt, p)
    announce("maxit warning")
    phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, lt.make_opts(tol=1e-12, maxit=3))
    assert st["rc"] == lt.LT_WNOTCONV
    assert st["iters_max"] == 3
    assert np.all(np.isfinite(phi.cpu().numpy()))
    assert st["true_relres_max"] > 1e-12          # the reported residual is the real one
    h.close()


@pytest.mark.parametrize("n", [(2, 2), (3, 5), (8, 1), (2, 2, 2), (3, 2, 5)])
def test_tiny_grids_match_oracle(lt, n):
    name = "C1" if len(n) == 2 else "C3"
    p = wl.make_problem(name, n=n, nsrc=1, nrec=2, ntimes=2)
    announce("tiny", n)
    h = device_problem(lt, p)
    phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, lt.make_opts(tol=1e-12))
    ref = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q, ndim=p.ndim)
    assert st["rc"] == 0
    check_heads(phi.cpu().numpy(), ref, 1e-8, f"tiny {n}")
    h.close()


def test_wells_on_walls_and_corners(lt):
    p = wl.make_problem("C1", n=(24, 20), ntimes=2)
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.5, 0.0], [0.999, 0.001, 0.0]])
    announce("wall wells")
    h = device_problem(lt, p)
    phi, st = lt.lt_solve(h, pts, 1.0, p.times, p.nz_contour, pts, lt.make_opts(tol=1e-12))
    ref = heads(p.n, p.h, p.kappa, p.S, pts, pts, p.times, p.nz_contour, q=1.0, ndim=p.ndim)
    assert st["rc"] == 0
    check_heads(phi.cpu().numpy(), ref, 1e-8, "wall wells")
    h.close()


def test_zero_rate_and_linearity_in_q(lt):
    p = wl.make_problem("C2", n=(40, 32), nsrc=3, ntimes=3)
    announce("linearity")
    h = device_problem(lt, p)
    o = lt.make_opts(tol=1e-11)
    phi1, _ = lt.lt_solve(h, p.sources, 1.0, p.times, p.nz_contour, p.receivers, o)
    phi3, _ = lt.lt_solve(h, p.sources, -2.5, p.times, p.nz_contour, p.receivers, o)
    phi0, _ = lt.lt_solve(h, p.sources, 0.0, p.times, p.nz_contour, p.receivers, o)
    a, b = phi1.cpu().numpy(), phi3.cpu().numpy()
    assert np.abs(b + 2.5 * a).max() <= 1e-9 * np.abs(a).max()
    assert np.abs(phi0.cpu().numpy()).max() == 0.0
    h.close()
