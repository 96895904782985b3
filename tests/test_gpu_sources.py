"""Sources of a solve on the GPU path: a pumping rate per well and an initial head
(the transformed semi-discrete system of Section 2.1, (K + zM) phi_hat = sum_s
qhat_s(z) b_s + M phi0, whose M phi0 term enters the contour sum with factor 1).

Pins: the exact decay of a single discrete eigenmode on a homogeneous grid
(closed form, no oracle), and element-wise agreement with the oracle's
direct solves for wells at different rates plus a random initial head."""
import numpy as np
import pytest

import workloads as wl
from oracle.fv import point_weights
from oracle.heads import heads
from gpu_util import device_problem, check_heads, announce

pytestmark = pytest.mark.gpu


def _eigenmode(n, h):
    """Sampled sin(pi x) sin(pi y) on the cell centres and its eigenvalue
    lambda = sum_a (4 kappa / h_a^2) sin^2(pi h_a / 2) / S of K phi = lambda M phi
    (zero-Dirichlet walls at h/2 make the sampled mode exact)."""
    nd = 3 if n[2] > 1 else 2
    f = np.ones((n[2], n[1], n[0]))
    lam = 0.0
    for a in range(nd):
        shape = [1, 1, 1]
        shape[2 - a] = n[a]
        f = f * np.sin(np.pi * (np.arange(n[a]) + 0.5) * h[a]).reshape(shape)
        lam += 4.0 / h[a] ** 2 * np.sin(np.pi * h[a] / 2) ** 2
    return f.ravel(), lam


@pytest.mark.parametrize("n", [(64, 64, 1), (16, 16, 8)])
@pytest.mark.parametrize("prec", [0, 1])
def test_initial_eigenmode_decays_exactly(lt, n, prec):
    """No wells, phi0 a discrete eigenmode: every head is exp(-lambda t) B_r phi0."""
    import torch
    nd = 3 if n[2] > 1 else 2
    h = tuple(1.0 / a for a in n[:nd]) + (1.0,) * (3 - nd)
    N = int(np.prod(n))
    kap, s = 1.0, 1e-5
    phi0, lam = _eigenmode(n, h)
    lam /= s
    announce("eigenmode decay", n, prec)
    p = wl.Problem(name="mode", ndim=nd, n=n, h=h, kappa=np.full(N, kap), S=np.full(N, s),
                   sources=np.zeros((0, 3)), receivers=np.array([(0.3, 0.4, 0.5), (0.55, 0.5, 0.5), (0.8, 0.2, 0.3)]),
                   times=np.array([0.05, 0.5, 2.0]) / lam, nz_contour=24)
    hd = device_problem(lt, p)
    tol = 1e-10 if prec == 0 else 1e-8
    o = lt.make_opts(tol=tol, precision=prec)
    ph0 = torch.tensor(phi0, dtype=torch.float64, device="cuda")
    phi, st = lt.lt_solve(hd, p.sources, 1.0, p.times, p.nz_contour, p.receivers, o, phi0=ph0)
    assert st["rc"] == 0 and phi.shape == (1, 3, 3)
    Br = point_weights(n, h, p.receivers) @ phi0
    exact = (Br[:, None] * np.exp(-lam * p.times)[None, :])[None]
    # the contour's own error at 24 nodes (3.89^-24 amplified by exp(0.171 * 24)) is ~1e-12
    check_heads(phi.cpu().numpy(), exact, 1e-6 if prec == 0 else 1e-5, f"eigenmode {n} prec {prec}")
    print("iterations", st["iters_max"], "resolves", st["resolves"], flush=True)
    hd.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_rates_and_initial_head_match_oracle(lt, prec):
    import torch
    p = wl.make_problem("C2", n=(48, 40), nsrc=3, ntimes=4)
    rates = np.array([1.0, -0.5, 2.5])
    phi0 = np.exp(wl.gaussian_random_field((48, 40), (1 / 48, 1 / 40), (0.2, 0.2), 1.0, 77)).flatten(order="F") - 1.0
    announce("rates + phi0", p.n, prec)
    ref = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=rates, phi0=phi0,
                ndim=p.ndim)
    hd = device_problem(lt, p)
    tol = 1e-10 if prec == 0 else 1e-8
    o = lt.make_opts(tol=tol, precision=prec)
    ph0 = torch.tensor(phi0, dtype=torch.float64, device="cuda")
    phi, st = lt.lt_solve(hd, p.sources, rates, p.times, p.nz_contour, p.receivers, o, phi0=ph0)
    assert st["rc"] == 0 and st["n_rhs"] == 4
    check_heads(phi.cpu().numpy(), ref, 1e-6 if prec == 0 else 1e-5, f"rates+phi0 prec {prec}")
    # the initial head alone: one row, equal to the phi0 part of every well's row
    alone, st0 = lt.lt_solve(hd, np.zeros((0, 3)), 1.0, p.times, p.nz_contour, p.receivers, o, phi0=ph0)
    assert st0["rc"] == 0 and alone.shape == (1, len(p.receivers), len(p.times))
    wells, _ = lt.lt_solve(hd, p.sources, rates, p.times, p.nz_contour, p.receivers, o)
    ref0 = heads(p.n, p.h, p.kappa, p.S, np.zeros((0, 3)), p.receivers, p.times, p.nz_contour, phi0=phi0,
                 ndim=p.ndim)
    check_heads(alone.cpu().numpy(), ref0, 1e-6 if prec == 0 else 1e-5, f"phi0 alone prec {prec}")
    diff = phi.cpu().numpy() - wells.cpu().numpy()
    assert np.abs(diff - alone.cpu().numpy()).max() <= 1e-6 * np.abs(ref).max()
    hd.close()


def test_adjoint_takes_rates_and_refuses_initial_head(lt):
    import torch
    from oracle.jacobian import jacobian
    p = wl.make_problem("C2", n=(20, 16), nsrc=2, nrec=3, ntimes=2)
    rates = np.array([2.0, -0.75])
    announce("adjoint rates", p.n)
    hd = device_problem(lt, p)
    o = lt.make_opts(tol=1e-11, precision=0)
    dK, dS, st = lt.lt_adjoint(hd, p.sources, rates, p.receivers, p.times, p.nz_contour, o)
    assert st["rc"] == 0
    rK, rS = jacobian(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=rates, ndim=p.ndim)
    for got, ref in ((dK.cpu().numpy(), rK), (dS.cpu().numpy(), rS)):
        scale = np.abs(ref).max(axis=-1, keepdims=True)
        assert (np.abs(got - ref) / scale).max() <= 1e-6
    # an initial head is not a parameter of the sensitivity path
    src, keep = lt._sources(p.sources, 1.0, torch.zeros(p.N, dtype=torch.float64, device="cuda"))
    rp, _ = lt._points(p.receivers)
    t = np.ascontiguousarray(p.times)
    st2, _, _ = lt._stats(5, 2 * (p.nz_contour // 2))
    rc = lt._lib.lt_adjoint(hd.ptr, lt.C.byref(src), lt.C.byref(rp), t.ctypes.data_as(lt._dp), 2,
                            lt.C.byref(lt.lt_contour(p.nz_contour)), lt.C.byref(o), lt._dev_f64(dK, "dK"),
                            lt._dev_f64(dS, "dS"), lt.C.byref(st2))
    assert rc == lt.LT_EUNSUPPORTED
    hd.close()
