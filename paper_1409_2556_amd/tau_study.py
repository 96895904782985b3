"""One preconditioner shift against several: the comparison of Section 4.1.

The paper compares a Krylov solver preconditioned by one shift-and-invert
operator (K + tau M)^{-1}, tau the contour node of smallest real part
("Single"), with the flexible solver that cycles several preconditioner
shifts (Section 3, "Flexible"), over the variance of ln kappa, the
measurement time and the grid size, and solves 40 late times at once with
two shifts.  This module runs the same sweeps through the library on
synthetic Gaussian random fields (the single-well workload W1) and reports
outer iterations, V-cycles and seconds per solve.

The paper applies its preconditioners with a sparse direct factorisation.
Here each application is the multigrid refinement driven to the inner
tolerance that the relaxation rule allows (the ``relax`` option).  With a small
relax factor the first applications are solved to near FP64 round-off,
which stands in for the exact factorisation; inexact-Krylov theory lets
the later ones loosen without changing the outer iteration count.  The
default relax factor of the library gives the inexact counts beside them.  The
paper stops every shift at a relative residual of 1e-10 (``conv =
LT_CONV_RELATIVE``); the library's default weighted test is shown too.

    python -m paper_1409_2556_amd.tau_study [--quick]

prints one JSON object (every row) and a Markdown summary on stderr.
Needs a GPU; every solve is a library call.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import replace

import numpy as np


def _solve(lt, p, n_tau, relax, inner_max, tol, conv, tau=None):
    import torch
    kap = torch.tensor(p.kappa, dtype=torch.float64, device="cuda")
    S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
    h = lt.lt_setup(p.ndim, p.n, p.h, kap, S, bc=p.bc, sy=p.sy)
    kw = dict(tol=tol, precision=lt.LT_PREC_FP64, relax=relax, inner_max=inner_max, maxit=400, conv=conv)
    if tau is not None:
        kw["tau"] = tau
    else:
        kw["n_tau"] = n_tau
    opts = lt.make_opts(**kw)
    lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, opts)  # warm-up (workspaces)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h.close()
    return {"rc": st["rc"], "iters": st["iters_max"], "vcycles": st["vcycles"], "seconds": dt,
            "true_relres": st["true_relres_max"]}


def _projected_shifts(lt, p):
    """The paper's two preconditioner shifts with the first moved onto the imaginary axis.

    The paper's first shift is the contour node of smallest real part, which is
    negative; a V-cycle on K + tau M diverges there, so the library's own rules
    only take nodes with Re z >= 0.  i |Im tau_1| keeps the paper's imaginary
    part, where the V-cycle converges."""
    z = np.concatenate([lt.lt_talbot(p.nz_contour, t)[0] for t in p.times])
    t1 = z[np.argmin(z.real)]
    t2 = z[np.argmax(z.real)]
    return 1j * abs(t1.imag), t2


def _pair(lt, p, relax, inner_max, tol, conv):
    t1, t2 = _projected_shifts(lt, p)
    return {"single": _solve(lt, p, 1, relax, inner_max, tol, conv),
            "flexible": _solve(lt, p, 2, relax, inner_max, tol, conv),
            "single_projected": _solve(lt, p, 1, relax, inner_max, tol, conv, tau=[t1]),
            "flexible_projected": _solve(lt, p, 2, relax, inner_max, tol, conv, tau=[t1, t1, t1, t2, t2])}


def run(quick=False, tol=1e-10, relax_exact=1e-4, inner_exact=60, relax_inexact=3.0):
    import workloads as wl
    from paper_1409_2556_amd import binding as lt

    # (relax, inner_max, convergence test): the paper's plain relative test with near-exact and
    # with relaxed preconditioner solves, and the library's default weighted test
    settings = {"exact": (relax_exact, inner_exact, lt.LT_CONV_RELATIVE),
                "inexact": (relax_inexact, 30, lt.LT_CONV_RELATIVE),
                "inexact_weighted": (relax_inexact, 30, lt.LT_CONV_WEIGHTED)}
    rows = []

    def add(table, label, p):
        for name, (rx, im, cv) in settings.items():
            r = _pair(lt, p, rx, im, tol, cv)
            rows.append({"table": table, "case": label, "preconditioner": name, **r})
            print(f"[study] {table} {label} {name}: " + ", ".join(f"{k} {v['iters']}" for k, v in r.items())
                  + " its", file=sys.stderr, flush=True)

    variances = (0.8, 1.6) if quick else (0.8, 1.6, 3.5)
    for v in variances:
        add("variance", v, wl.make_problem("W1", var=v))
    t_d = (0.06, 0.3) if quick else (0.06, 0.3, 1.2)   # the paper's 1, 5 and 20 minutes
    for t in t_d:
        p = wl.make_problem("W1")
        add("time", t, replace(p, times=np.array([t * wl.T_D])))
    grids = (64, 128) if quick else (64, 128, 256, 512)
    for g in grids:
        add("grid", g, wl.make_problem("W1", n=(g, g)))
    # 40 late times (the paper's 40 to 60 minutes: 2.4 to 3.6 diffusion times) in one solve
    # with two preconditioner shifts, against the single time in the middle of the window
    p = wl.make_problem("W1")
    late = replace(p, times=np.linspace(2.4, 3.6, 10 if quick else 40) * wl.T_D)
    mid = replace(p, times=np.array([3.0 * wl.T_D]))
    for name, (rx, im, cv) in settings.items():
        rows.append({"table": "many_times", "case": len(late.times), "preconditioner": name,
                     "flexible": _solve(lt, late, 2, rx, im, tol, cv),
                     "one_time_flexible": _solve(lt, mid, 2, rx, im, tol, cv)})
    return {"workload": "W1: 128x128 GRF, ln kappa exponential covariance (corr 0.2), one well at the "
                        "centre, 4 receivers, 40-node Talbot, FP64 V(2,2) GMG preconditioner",
            "tol": tol, "settings": {k: {"relax": v[0], "inner_max": v[1],
                                         "test": "relative" if v[2] == lt.LT_CONV_RELATIVE else "weighted"}
                                     for k, v in settings.items()},
            "rows": rows}


def _markdown(res):
    out = ["| table | case | setting | Single its | Flexible its | Single proj. its | Flexible proj. its "
           "| Single ms | Flexible ms |",
           "|---|---|---|---:|---:|---:|---:|---:|---:|"]
    for r in res["rows"]:
        if r["table"] == "many_times":
            f, o = r["flexible"], r["one_time_flexible"]
            out.append(f"| many_times | {r['case']} times | {r['preconditioner']} | | {f['iters']} (one time: "
                       f"{o['iters']}) | | | | {1e3 * f['seconds']:.1f} |")
            continue
        s, f = r["single"], r["flexible"]
        out.append(f"| {r['table']} | {r['case']} | {r['preconditioner']} | {s['iters']} | {f['iters']} | "
                   f"{r['single_projected']['iters']} | {r['flexible_projected']['iters']} | "
                   f"{1e3 * s['seconds']:.1f} | {1e3 * f['seconds']:.1f} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--quick", action="store_true", help="fewer cases (a short check)")
    ap.add_argument("--tol", type=float, default=1e-10)
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    res = run(quick=a.quick, tol=a.tol)
    print(_markdown(res), file=sys.stderr, flush=True)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
