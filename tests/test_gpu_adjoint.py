"""GPU sensitivities (lt_adjoint) against the oracle's discrete-adjoint
Jacobian, which is itself pinned to central finite differences.  Bar: the
FP64 path within 1e-6 of the largest sensitivity of each (source, receiver,
time) map; the mixed path within 1e-5."""
import numpy as np
import pytest

import workloads as wl
from oracle.jacobian import jacobian
from gpu_util import device_problem, announce

pytestmark = pytest.mark.gpu

CASES = {
    "2d_20x16": dict(name="C2", kw=dict(n=(20, 16), nsrc=2, nrec=3, ntimes=2)),
    "3d_8x6x5": dict(name="C3", kw=dict(n=(8, 6, 5), nsrc=2, nrec=3)),
    "2d_40x40_c1": dict(name="C1", kw=dict(n=(40, 40), ntimes=2, nrec=2)),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [0, 1])
def test_sensitivities_match_oracle(lt, case, prec):
    spec = CASES[case]
    p = wl.make_problem(spec["name"], **spec["kw"])
    announce("adjoint", case, prec, p.n)
    h = device_problem(lt, p)
    tol = 1e-11 if prec == 0 else 1e-9
    opts = lt.make_opts(tol=tol, precision=prec, n_tau=p.n_tau)
    JK, JS, st = lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, opts)
    gK, gS = JK.cpu().numpy(), JS.cpu().numpy()
    rK, rS = jacobian(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q, ndim=p.ndim)
    bound = 1e-6 if prec == 0 else 1e-5
    for got, ref in ((gK, rK), (gS, rS)):
        scale = np.abs(ref).max(axis=-1, keepdims=True)
        err = (np.abs(got - ref) / scale).max()
        print(case, prec, "iters", st["iters_max"], "err", err, flush=True)
        assert err <= bound
    assert st["n_rhs"] == len(p.sources) + len(p.receivers)
    h.close()


def test_sensitivity_reciprocity(lt):
    p = wl.make_problem("C2", n=(24, 24), ntimes=2)
    a, b = np.array([[0.3, 0.4, 0.0]]), np.array([[0.7, 0.55, 0.0]])
    announce("adjoint reciprocity")
    h = device_problem(lt, p)
    o = lt.make_opts(tol=1e-11)
    K1, S1, _ = lt.lt_adjoint(h, a, 1.0, b, p.times, p.nz_contour, o)
    K2, S2, _ = lt.lt_adjoint(h, b, 1.0, a, p.times, p.nz_contour, o)
    k1, k2 = K1.cpu().numpy(), K2.cpu().numpy()
    assert np.abs(k1 - k2).max() <= 1e-6 * np.abs(k1).max()
    s1, s2 = S1.cpu().numpy(), S2.cpu().numpy()
    assert np.abs(s1 - s2).max() <= 1e-6 * np.abs(s1).max()
    h.close()


def test_contraction_paths_agree(lt):
    """With 130 fields the staged contraction would need more than 64 KB of LDS and the
    per-pair kernel runs; split into two calls of 35 sources (95 fields) the staged kernel
    runs.  The solves of each right-hand side do not depend on the others, so the two
    contractions of the same fields agree to rounding."""
    p = wl.make_problem("C3", n=(10, 8, 6))
    rng = np.random.default_rng(7)
    src = rng.uniform(0.15, 0.85, size=(70, 3))
    rec = rng.uniform(0.15, 0.85, size=(60, 3))
    announce("adjoint contraction paths", p.n, len(src), len(rec))
    h = device_problem(lt, p)
    o = lt.make_opts(tol=1e-10, precision=0, n_tau=p.n_tau)
    K, S, st = lt.lt_adjoint(h, src, 1.0, rec, p.times, p.nz_contour, o)
    assert st["rc"] == 0
    K, S = K.cpu().numpy(), S.cpu().numpy()
    for sl in (slice(0, 35), slice(35, 70)):
        Kp, Sp, stp = lt.lt_adjoint(h, src[sl], 1.0, rec, p.times, p.nz_contour, o)
        assert stp["rc"] == 0
        for got, ref in ((Kp.cpu().numpy(), K[sl]), (Sp.cpu().numpy(), S[sl])):
            scale = np.abs(ref).max(axis=-1, keepdims=True)
            err = (np.abs(got - ref) / scale).max()
            print("contraction paths", sl, err, flush=True)
            assert err <= 1e-10
    h.close()


def test_fom_sensitivities_match_oracle(lt):
    """lt_adjoint with the FOM variant of the flexible shifted method, same bar as GMRES."""
    spec = CASES["2d_20x16"]
    p = wl.make_problem(spec["name"], **spec["kw"])
    announce("adjoint fom", p.n)
    h = device_problem(lt, p)
    opts = lt.make_opts(tol=1e-11, precision=0, n_tau=p.n_tau, method=lt.LT_METHOD_FOM)
    JK, JS, st = lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, opts)
    assert st["rc"] == 0
    rK, rS = jacobian(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q, ndim=p.ndim)
    for got, ref in ((JK.cpu().numpy(), rK), (JS.cpu().numpy(), rS)):
        scale = np.abs(ref).max(axis=-1, keepdims=True)
        err = (np.abs(got - ref) / scale).max()
        print("adjoint fom err", err, flush=True)
        assert err <= 1e-6
    h.close()
