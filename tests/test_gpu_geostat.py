"""The geostatistical inversion on the GPU (Section 5.1, Algorithm 2; the transient hydraulic
tomography case of Section 5.3) against the oracle.

* lt_cov_apply against the dense exponential covariance on 2D and 3D grids (ragged against the
  64-cell tiles, anisotropic lengths, more vectors than one workgroup's 32).
* One Gauss-Newton step from two linearisation points, and three steps of the whole inversion
  (with the multigrid and with the exact shift-and-invert preconditioner), against the oracle's: the data are Crank-Nicolson heads of the true field (model error, as in
  the paper) with 2 % noise.  Bars: h(s) 1e-9 of its largest entry; beta and s_{k+1} 1e-8
  (relative to |beta| and the largest |s_{k+1}|); the inversion's iterate 1e-8 and misfits 1e-7
  after three steps.  The heads' and Jacobian's errors, ~1e-12 of their scale at the solver
  tolerance 1e-12, reach s_{k+1} through the saddle-point system, whose condition (r = (2 % of
  the data's rms)^2 against J Q J^T) amplifies them by up to ~1e3; measured: 4e-11.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.geostat import exp_covariance, gauss_newton_step
from oracle.timestep import crank_nicolson_heads
from gpu_util import announce

pytestmark = pytest.mark.gpu

VAR, ELL = 1.0, (0.2, 0.2, 0.2)


def _handle(lt, p, s):
    kap = torch.tensor(np.exp(s), dtype=torch.float64, device="cuda")
    S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
    return lt.lt_setup(p.ndim, p.n, p.h, kap, S, bc=p.bc)


@pytest.mark.parametrize("name,n,ell", [("THT", (20, 16), (0.2, 0.2, 0.2)), ("THT", (37, 23), (0.15, 0.3, 1.0)),
                                        ("C3", (8, 6, 5), (0.2, 0.3, 0.1))])
def test_cov_apply_matches_dense(lt, name, n, ell):
    p = wl.make_problem(name, n=n)
    announce("cov_apply", name, n)
    h = _handle(lt, p, np.log(p.kappa))
    Q = exp_covariance(p.n, p.h, 1.7, ell, p.ndim)
    rng = np.random.default_rng(3)
    M = 45
    v = rng.standard_normal((M, p.N))
    out = torch.zeros((M, p.N), dtype=torch.float64, device="cuda")
    lt.lt_cov_apply(h, 1.7, ell, torch.tensor(v, device="cuda"), out, M)
    ref = v @ Q  # Q symmetric: (Q v^T)^T
    err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"[cov] {name}{n} err {err:.2e}", flush=True)
    assert err <= 1e-12
    with pytest.raises(lt.LTError):
        lt.lt_cov_apply(h, -1.0, ell, torch.tensor(v, device="cuda"), out, M)
    h.close()


def _data(p, seed=7):
    cn = crank_nicolson_heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, 0.0025 * wl.T_D,
                              ndim=p.ndim)
    y0 = cn.ravel()
    rng = np.random.default_rng(seed)
    y = y0 * (1 + 0.02 * rng.standard_normal(y0.size))
    return y, (0.02 * np.sqrt(np.mean(y0 ** 2))) ** 2


def _opts(lt, precond="gmg"):
    if precond == "exact":
        return lt.make_opts(tol=1e-12, maxit=200, n_tau=2, precond=lt.LT_PRECOND_EXACT)
    return lt.make_opts(tol=1e-12, maxit=200)


@pytest.mark.parametrize("start", ["zero", "half_true"])
def test_step_matches_oracle(lt, start):
    p = wl.make_problem("THT", n=(32, 32))
    announce("geostat step", start)
    y, r = _data(p)
    s = np.zeros(p.N) if start == "zero" else 0.5 * np.log(p.kappa)
    h = _handle(lt, p, s)
    sd = torch.tensor(s, device="cuda")
    sn = torch.zeros_like(sd)
    hs, beta, rc = lt.lt_geostat_step(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, VAR, ELL, r,
                                      torch.tensor(y, device="cuda"), sd, sn, _opts(lt))
    assert rc == 0
    ref = gauss_newton_step(p.n, p.h, s, p.S, p.sources, p.receivers, p.times, p.nz_contour, y, VAR, ELL, r,
                            ndim=p.ndim)
    eh = np.abs(hs.cpu().numpy() - ref["hs"]).max() / np.abs(ref["hs"]).max()
    es = np.abs(sn.cpu().numpy() - ref["s_next"]).max() / np.abs(ref["s_next"]).max()
    eb = abs(beta - ref["beta"]) / max(abs(ref["beta"]), 1e-30)
    print(f"[geostat] step from {start}: h {eh:.2e} s_next {es:.2e} beta {eb:.2e} "
          f"(beta {beta:.4f})", flush=True)
    assert eh <= 1e-9 and eb <= 1e-8 and es <= 1e-8
    h.close()


@pytest.mark.parametrize("precond", ["gmg", "exact"])
def test_inversion_matches_oracle(lt, precond):
    p = wl.make_problem("THT", n=(32, 32))
    announce("geostat inversion", precond)
    y, r = _data(p)
    iters = 3
    S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
    s0 = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    s, mis, stp, rc = lt.lt_geostat_invert(p.ndim, p.n, p.h, S, p.sources, p.q, p.receivers, p.times, p.nz_contour,
                                           VAR, ELL, r, torch.tensor(y, device="cuda"), s0, iters,
                                           opts=_opts(lt, precond))
    assert rc == 0
    Q = exp_covariance(p.n, p.h, VAR, ELL, p.ndim)
    sr = np.zeros(p.N)
    mref = []
    for _ in range(iters):
        out = gauss_newton_step(p.n, p.h, sr, p.S, p.sources, p.receivers, p.times, p.nz_contour, y, VAR, ELL, r,
                                ndim=p.ndim, Q=Q)
        mref.append(np.sum((y - out["hs"]) ** 2) / r)
        sr = out["s_next"]
    es = np.abs(s.cpu().numpy() - sr).max() / np.abs(sr).max()
    em = np.abs(mis - np.array(mref)) / np.array(mref)
    print(f"[geostat] inversion ({precond}): s err {es:.2e}; misfit gpu {mis} oracle {mref}; steps {stp}",
          flush=True)
    assert es <= 1e-8 and em.max() <= 1e-7
    assert mis[-1] < mis[0]
