"""The restarted FOM variant with the exact preconditioner on the GPU (Section 3.1: the FOM
residual of every shift is -eta_k v_{m+1}, so the basis restarts from v_{m+1} with a
coefficient -eta_k per shift; opts.restart) against the oracle.

* The single-well test at 64x64 (40-node contour, relative test 1e-10, the paper's two-shift
  schedule): heads against the oracle's direct solves, and the steps over all cycles against
  the oracle's restarted FOM (same basis, same test), for cycles of 5 and 12 steps; a cycle
  longer than the solve gives the heads and steps of FOM without restarts.
* Several wells that converge in different cycles, and several times in one basis.
* Per-well rates and the initial head's term (its own contour weights) under restarts.
* Refusals: restarts need FOM and the exact preconditioner, and only lt_solve restarts.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.contour import talbot_nodes
from oracle.fv import assemble, point_weights
from oracle.heads import heads_problem
from oracle.krylov import restarted_fom, tau_schedule
from gpu_util import announce, check_heads, device_problem

pytestmark = pytest.mark.gpu


def _opts(lt, restart, tol=1e-10):
    return lt.make_opts(tol=tol, maxit=400, n_tau=2, precond=lt.LT_PRECOND_EXACT, conv=lt.LT_CONV_RELATIVE,
                        method=lt.LT_METHOD_FOM, restart=restart)


def _oracle_steps(p, cycle, tol=1e-10):
    K, m = assemble(p.n, p.h, p.kappa, p.S, p.bc, ndim=p.ndim)
    z = np.concatenate([talbot_nodes(p.nz_contour, t)[0] for t in p.times])
    taus = tau_schedule(z, 2)
    B = point_weights(p.n, p.h, p.sources).toarray()
    return [restarted_fom(K, m, B[s], taus, z, tol, cycle, 400)["iters"] for s in range(B.shape[0])]


def test_restarted_fom_matches_oracle(lt):
    p = wl.make_problem("W1", n=(64, 64))
    h = device_problem(lt, p)
    ref = heads_problem(p)
    plain, st0 = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, _opts(lt, 0))
    plain = plain.cpu().numpy()
    n0 = int(st0["iters_per_rhs"][0])
    for cycle in (5, 12):
        announce("restarted FOM", cycle)
        phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, _opts(lt, cycle))
        assert st["rc"] == 0
        got = phi.cpu().numpy()
        check_heads(got, ref, 1e-7, f"W1 64x64 restart {cycle}")
        want = _oracle_steps(p, cycle)
        steps = [int(v) for v in st["iters_per_rhs"]]
        print(f"[restart] cycle {cycle}: gpu steps {steps} oracle {want} (no restart {n0}); true residual "
              f"{st['true_relres_max']:.2e}", flush=True)
        # same basis and test; classical against modified Gram-Schmidt may flip a shift
        # within rounding of the bar
        assert all(abs(g - w) <= 1 for g, w in zip(steps, want)), (steps, want)
        assert st["true_relres_max"] <= 1e-10
    # a cycle longer than the solve never restarts
    phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, _opts(lt, n0 + 5))
    assert int(st["iters_per_rhs"][0]) == n0
    np.testing.assert_allclose(phi.cpu().numpy(), plain, rtol=0, atol=1e-13 * np.abs(plain).max())
    h.close()


def test_restarted_wells_finish_in_different_cycles(lt):
    # several wells and two times in one basis: right-hand sides leave at different cycles,
    # keep their last cycle, and their heads equal each well solved alone
    p = wl.make_problem("C2", n=(48, 40), nsrc=5, nrec=6, ntimes=2)
    h = device_problem(lt, p)
    ref = heads_problem(p)
    announce("restarted FOM, 5 wells")
    o = _opts(lt, 4, tol=1e-9)
    phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
    assert st["rc"] == 0
    got = phi.cpu().numpy()
    steps = [int(v) for v in st["iters_per_rhs"]]
    print(f"[restart] 5 wells: steps {steps}, true residual {st['true_relres_max']:.2e}", flush=True)
    check_heads(got, ref, 1e-6, "C2 48x40 restart 4")
    for s in range(len(p.sources)):
        one, st1 = lt.lt_solve(h, p.sources[s:s + 1], p.q, p.times, p.nz_contour, p.receivers, o)
        np.testing.assert_allclose(one.cpu().numpy()[0], got[s], rtol=0, atol=1e-12 * np.abs(got[s]).max())
        assert int(st1["iters_per_rhs"][0]) == steps[s]
    h.close()


def test_restart_refusals(lt):
    p = wl.make_problem("W1", n=(32, 32))
    h = device_problem(lt, p)
    for kw in (dict(precond=lt.LT_PRECOND_GMG), dict(method=lt.LT_METHOD_GMRES), dict(restart=-1),
               dict(restart=2001)):
        o = _opts(lt, 4)
        for k, v in kw.items():
            setattr(o, k, v)
        with pytest.raises(lt.LTError) as e:
            lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
        assert e.value.code == lt.LT_EINVAL
    with pytest.raises(lt.LTError) as e:
        lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, _opts(lt, 4))
    assert e.value.code == lt.LT_EUNSUPPORTED
    h.close()


def test_restart_with_rates_and_initial_head(lt):
    # per-well rates and the initial head's term M phi0 (its shifts weigh by w_k alone, its
    # heads enter every row): restarted against the oracle's heads
    from oracle.heads import heads
    p = wl.make_problem("C2", n=(48, 40), nsrc=3, ntimes=3)
    rates = np.array([1.0, -0.5, 2.5])
    phi0 = np.exp(wl.gaussian_random_field((48, 40), (1 / 48, 1 / 40), (0.2, 0.2), 1.0, 77)).flatten(order="F") - 1.0
    announce("restarted FOM, rates + phi0")
    ref = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=rates, phi0=phi0,
                ndim=p.ndim)
    h = device_problem(lt, p)
    ph0 = torch.tensor(phi0, dtype=torch.float64, device="cuda")
    o = lt.make_opts(tol=1e-10, maxit=400, n_tau=2, precond=lt.LT_PRECOND_EXACT, method=lt.LT_METHOD_FOM, restart=6)
    phi, st = lt.lt_solve(h, p.sources, rates, p.times, p.nz_contour, p.receivers, o, phi0=ph0)
    print(f"[restart] rates + phi0: steps {[int(v) for v in st['iters_per_rhs']]}, true residual "
          f"{st['true_relres_max']:.2e}", flush=True)
    assert st["rc"] == 0 and st["n_rhs"] == 4
    check_heads(phi.cpu().numpy(), ref, 1e-6, "restart 6, rates + phi0")
    h.close()
