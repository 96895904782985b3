"""Throughput of the Laplace-transform shifted-system solver on one MI355X.

Default workload (--workload C5J): six Jacobian-assembly problems on uneven
grids (128^2, 256^2, 512^2 in 2D; 32^3, 64^3, 128x128x64 in 3D; ln kappa
Gaussian random fields, 2D as the 256x256 workload, 3D anisotropic with
log-uniform storage), each with 16 pumping wells and 32 observation wells,
times {0.3, 1.2} diffusion times and a 24-node Talbot contour.  One step is
one lt_adjoint_batch call: for every problem the forward fields of the 16
wells and the adjoint fields of the 32 receivers (48 right-hand sides x 24
shifts = 1,152 shifted solves, 6,912 over the batch), contracted cell by
cell into d phi / d ln kappa and d phi / d ln S for every (well, receiver,
time) triple.  Inputs are resident on the GPU before the timed region.
Metric: shifted solves per second, counted only when the sensitivities of
the 128x128 problem agree with the CPU oracle's Jacobian to 1e-5 of each
map's largest entry.

Variants: FP64 throughout ("fp64", the plain method), the FP32 V-cycle
inside the FP64 outer solve ("mixed"), and "learned": mixed precision with
the U-Net preconditioner giving each preconditioner solve of the 2D problems
its first guess (trained on the GPU just before, on 128x128 fields; training
time reported separately), switched off by the solver once its guesses stop
paying for themselves, the V-cycle the fallback (3D problems: V-cycle only).
The headline value is the learned variant.

--workload C2 times the 256x256 heads workload (lt_solve), C3 the 64x64x32
sensitivities (lt_adjoint), C5 the six grids' heads (lt_solve_batch), EXACT the
single-well test of Section 4.1 with the exact shift-and-invert preconditioner
('Single' and 'Flexible' over the variances, times and grid sizes of Tables 1-3), THT
the geostatistical inversion of the transient hydraulic tomography case (Section 5.3).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "C2"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_post2d_refine_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1409_2556_amd", "csrc", "mg_fused.hip")


def _measured_traffic(traffic_file=TRAFFIC_FILE, kernel_src=KERNEL_SRC):
    """HBM bytes per launch of the profiled kernel from the committed counter
    summary, or None once the kernel source (one file, or several hashed in order)
    differs from the profiled one."""
    import hashlib
    import re
    srcs = [kernel_src] if isinstance(kernel_src, str) else list(kernel_src)
    try:
        txt = open(traffic_file).read()
        want = re.search(r"sha256\[:16\] = ([0-9a-f]{16})", txt).group(1)
        val = float(re.search(r"traffic_bytes_per_launch: ([0-9.]+)", txt).group(1))
        hsh = hashlib.sha256()
        for f in srcs:
            hsh.update(open(f, "rb").read())
        have = hsh.hexdigest()[:16]
    except (OSError, AttributeError):
        return None
    return val if have == want else None


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    # C2: every variant stops at the same weighted tolerance: at equal settings the FP64 and mixed
    # paths take the same outer iterations and give the same head error (the refinement of every
    # preconditioner solve is FP64 in both), so the comparison is at equal accuracy.  1e-7 with
    # relax 0.3 and shifts from the residual estimates leaves 2.5e-6 against the oracle over all
    # ten times, a 4x margin to the 1e-5 bar.
    ap.add_argument("--tol-fp64", type=float, default=1e-7)
    ap.add_argument("--tol-mixed", type=float, default=1e-7)
    ap.add_argument("--relax", type=float, default=0.3)
    ap.add_argument("--variant", choices=["all", "mixed", "fp64", "learned"], default="all")
    ap.add_argument("--train-steps", type=int, default=400)
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="after the solves, copy a 512 MiB buffer once (a plain copy kernel of known "
                         "size, to scale hardware byte counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--exact-cases", choices=["all", "headline", "one"], default="all",
                    help="EXACT: every case of Tables 1-3, only the headline (one well and 16 wells), or only "
                         "the one-well headline")
    ap.add_argument("--cpu-sample-times", type=int, default=10)
    ap.add_argument("--no-tune", action="store_true", help="keep the default smoother tile shapes")
    ap.add_argument("--groups", type=int, default=2,
                    help="solve the sources as this many concurrent groups, one handle and stream each")
    ap.add_argument("--workload", choices=["C5J", "C2", "C3", "C5", "EXACT", "THT", "BLOCK"], default="C5J",
                    help="C5J (default): the six Jacobian-assembly problems in one lt_adjoint_batch call; "
                         "C2: the 256x256 heads workload; C3: sensitivities (lt_adjoint) of the "
                         "64x64x32 workload; C5: the six grids' heads in one lt_solve_batch call; "
                         "EXACT: the single-well test with the exact shift-and-invert preconditioner; "
                         "THT: the geostatistical inversion of the tomography case; BLOCK: block flexible "
                         "GMRES (lt_shifted_solve_block) on the 256x256 workload's Jacobian right-hand sides "
                         "and contour shifts, blocks of 1, 4 and 8")
    ap.add_argument("--tht-iters", type=int, default=6, help="THT: Gauss-Newton iterations per inversion")
    ap.add_argument("--tht-precond", choices=["exact", "gmg"], default="exact",
                    help="THT: preconditioner of the forward and adjoint solves (exact: the paper's "
                         "shift-and-invert with its two-shift schedule, factorised anew each iteration)")
    ap.add_argument("--tol-jacobian", type=float, default=3e-10,
                    help="C5J: weighted tolerance of every variant (equal accuracy)")
    ap.add_argument("--relax-jacobian", type=float, default=0.3,
                    help="C5J, C3, C5: inner tolerance factor of every variant")
    ap.add_argument("--tau-adapt", type=int, choices=[0, 1], default=None,
                    help="C5J/C2: 1: preconditioner shifts from the residual estimates (opts.tau_adapt; every "
                         "variant alike); 0: the fixed schedule (default: 1 for C2, 0 for C5J, whose storage "
                         "sensitivities need the fixed schedule's margin)")
    ap.add_argument("--nu3d", type=int, default=2,
                    help="C5J: red-black sweeps before and after the coarse correction on the 3D problems")
    ap.add_argument("--maxit", type=int, default=48,
                    help="C5J: outer iterations the basis workspace is sized for")
    ap.add_argument("--p1", action="store_true",
                    help="C2: the same workload on P1 finite elements (lt_setup_p1: 257x257 cells, the 256x256 "
                         "interior vertices as unknowns; the oracle sample from the P1 oracle)")
    ap.add_argument("--water-table", type=float, default=None, metavar="SY",
                    help="C2/C3: make the top wall (+y in 2D, +z in 3D) a linearised water table with this "
                         "specific yield (the other walls keep zero head)")
    ap.add_argument("--n-tau", type=int, default=None,
                    help="C2/C3: preconditioner shifts cycled over the outer iterations (default: the workload's)")
    return ap.parse_args()


def _with_boundary(p, args):
    """The workload, with its top wall turned into a water table when asked (--water-table),
    and another preconditioner-shift count (--n-tau)."""
    from dataclasses import replace
    if args.n_tau is not None:
        p = replace(p, n_tau=int(args.n_tau))
    if args.water_table is None:
        return p
    bc = list(p.bc)
    bc[2 * p.ndim - 1] = 2
    return replace(p, bc=tuple(bc), sy=float(args.water_table))


def _boundary_config(p):
    if p.sy > 0 or 2 in p.bc:
        return {"boundary": "zero head, water table on the top wall", "sy": p.sy}
    return {}


def _handle(lt, p, tune, nvec, p1=False):
    """Handle on a stream of its own, with smoother tiles tuned for both precisions (setup, untimed).
    p1: P1 elements on the problem's cells (the interior vertices as unknowns)."""
    import torch
    kap = torch.tensor(p.kappa, dtype=torch.float64, device="cuda")
    S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    if p1:
        h = lt.lt_setup_p1(p.n[:2], p.h[:2], kap, S, stream=stream)
    else:
        h = lt.lt_setup(p.ndim, p.n, p.h, kap, S, bc=p.bc, stream=stream, sy=p.sy)
    h._torch_stream = stream
    tiles = {}
    if tune:
        for name, prec in (("fp64", lt.LT_PREC_FP64), ("mixed", lt.LT_PREC_MIXED)):
            t0 = time.perf_counter()
            ids, us = lt.lt_autotune(h, prec, 2, 2, nvec)
            tiles[name] = {"tiles": [list(lt.lt_tile_shape(t)) for t in ids], "us_per_step": us,
                           "tune_ms": (time.perf_counter() - t0) * 1e3}
    return h, tiles


def _merge_stats(sts):
    """Stats of one solve split over source groups (each group is an independent lt_solve)."""
    if len(sts) == 1:
        return sts[0]
    return {"rc": max(s["rc"] for s in sts), "iters_max": max(s["iters_max"] for s in sts),
            "vcycles": sum(s["vcycles"] for s in sts), "true_relres_max": max(s["true_relres_max"] for s in sts),
            "net_applied": sum(s["net_applied"] for s in sts),
            "net_disabled_at": max(s["net_disabled_at"] for s in sts)}


def _solve_groups(lt, hs, p, opts, phi):
    """All sources in one step: one lt_solve, or with several handles one lt_solve_batch call
    whose items (contiguous source groups, each on its handle's stream) run concurrently."""
    if len(hs) == 1:
        _, st = lt.lt_solve(hs[0], p.sources, p.q, p.times, p.nz_contour, p.receivers, opts, phi_out=phi)
        return st
    cuts = np.array_split(np.arange(len(p.sources)), len(hs))
    items = [dict(handle=h, sources=p.sources[c], q=p.q, times=p.times, nz=p.nz_contour, receivers=p.receivers,
                  opts=opts, phi_out=phi[c[0]:c[-1] + 1]) for h, c in zip(hs, cuts)]
    _, sts, rc = lt.lt_solve_batch(items)
    st = _merge_stats(sts)
    st["rc"] = max(st["rc"], rc)
    return st


def _run_variant(lt, hs, p, opts, steps, warmup, profile=0):
    """Warm up, then time `steps` solves.  With `profile`, the same `steps` solves
    are run once more, on the first handle alone, with the library timing every
    launch of the profiled kernel with HIP events on its own stream and counting
    its algorithmic bytes (kept out of the headline timing so the events do not slow it)."""
    import torch
    phi = torch.empty((len(p.sources), len(p.receivers), len(p.times)), dtype=torch.float64, device="cuda")
    h = hs[0]
    st = None
    opts.profile = 0
    for _ in range(warmup):
        st = _solve_groups(lt, hs, p, opts, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = _solve_groups(lt, hs, p, opts, phi)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = {"launches": 0, "ms": 0.0, "bytes": 0.0}
    if profile:
        opts.profile = profile
        for _ in range(steps):
            _, stp = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, opts, phi_out=phi)
            prof["launches"] += stp["prof_launches"]
            prof["ms"] += stp["prof_ms"]
            prof["bytes"] += stp["prof_bytes"]
        torch.cuda.synchronize()
        opts.profile = 0
    return dt, st, phi.cpu().numpy(), prof


def _cpu_baseline(p, ntimes, p1=False):
    """The oracle as it stands, on a bounded sample: every source, the first
    `ntimes` measurement times (ntimes * N_z/2 factorisations)."""
    workers = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    if p1:
        from oracle.p1 import heads_p1
        ref = heads_p1(p.n[:2], p.h[:2], p.kappa, p.S, p.sources, p.receivers, p.times[:ntimes], p.nz_contour,
                       q=p.q, workers=workers)
    else:
        from oracle.heads import heads
        ref = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times[:ntimes], p.nz_contour,
                    q=p.q, bc=p.bc, workers=workers, ndim=p.ndim, sy=p.sy)
    dt = time.perf_counter() - t0
    pairs = len(p.sources) * ntimes * (p.nz_contour // 2)
    return ref, {"value": pairs / dt, "unit": "shifted solves/s", "cores": workers, "kind": "oracle",
                 "sample": f"{len(p.sources)} sources x first {ntimes} times x {p.nz_contour // 2} shifts "
                           f"= {pairs} pairs of the same 256x256 workload, SuperLU per shift "
                           f"({dt:.1f} s)"}


def main():
    args = _parse()
    if args.tau_adapt is None:
        args.tau_adapt = 1 if args.workload == "C2" else 0
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "C5J":
        return main_jacobian(args)
    if args.workload == "EXACT":
        return main_exact(args)
    if args.workload == "THT":
        return main_tht(args)
    if args.workload == "BLOCK":
        return main_block(args)
    if args.workload == "C5":
        return main_batch(args)
    if args.workload == "C3":
        return main_adjoint(args)
    import workloads as wl
    if args.p1:
        if args.water_table is not None:
            print(json.dumps({"error": "--p1 takes zero-head walls only"}))
            sys.exit(2)
        p = wl.make_problem(WORKLOAD, n=(257, 257))  # 256 x 256 interior vertices
    else:
        p = _with_boundary(wl.make_problem(WORKLOAD), args)
    # the CPU oracle runs first, before this process touches the GPU
    cpu, ref = None, None
    nt = args.cpu_sample_times
    if not args.no_cpu_baseline:
        ref, cpu = _cpu_baseline(p, nt, p1=args.p1)
        print(f"[bench] oracle sample: {cpu['value']:.2f} solves/s on {cpu['cores']} cores", file=sys.stderr,
              flush=True)

    import torch
    from paper_1409_2556_amd import binding as lt

    torch.cuda.set_device(0)
    groups = max(1, min(args.groups, len(p.sources)))
    # tiles tuned for the right-hand sides one launch carries (one group's share)
    h, tiles = _handle(lt, p, not args.no_tune, -(-len(p.sources) // groups), p1=args.p1)
    hs = [h]
    for _ in range(groups - 1):
        # the other groups' handles take the first handle's tiles (tuned for the full batch)
        hg, _ = _handle(lt, p, False, len(p.sources), p1=args.p1)
        if tiles:
            for name, prec in (("fp64", lt.LT_PREC_FP64), ("mixed", lt.LT_PREC_MIXED)):
                lt.lt_set_tiles(hg, prec, [_tile_id(lt, t) for t in tiles[name]["tiles"]])
        hs.append(hg)
    pairs = len(p.sources) * len(p.times) * (p.nz_contour // 2)
    res = {}
    variants = [("fp64", lt.LT_PREC_FP64, args.tol_fp64), ("mixed", lt.LT_PREC_MIXED, args.tol_mixed),
                ("learned", lt.LT_PREC_MIXED, args.tol_mixed)]
    if args.variant != "all":
        variants = [v for v in variants if v[0] == args.variant]
    training = None
    net = None
    if any(v[0] == "learned" for v in variants):
        from paper_1409_2556_amd.train_unet import train
        t0 = time.perf_counter()
        net, hist = train(steps=args.train_steps, batch=8, lr=1e-3, verbose=False)
        torch.cuda.synchronize()
        training = {"steps": args.train_steps, "seconds": time.perf_counter() - t0,
                    "final_loss_mean20": float(np.mean(hist[-20:])),
                    "data": "128x128 GRF fields (seeds 10000-10007), point-source and smooth residuals, "
                            "targets from lt_precond_solve"}
        print(f"[bench] trained U-Net: {training['seconds']:.1f} s, loss {training['final_loss_mean20']:.3f}",
              file=sys.stderr, flush=True)
        # each group's handle gets its own copy of the trained network (a network's
        # workspace serves one solve at a time)
        nets = [net]
        for _ in hs[1:]:
            cp = lt.UNet(seed=0)
            cp.set_params(net.get_params())
            nets.append(cp)
        for hg, ng in zip(hs, nets):
            lt.lt_unet_attach(hg, ng)
    prof_name = "mixed" if any(v[0] == "mixed" for v in variants) else variants[0][0]
    for name, prec, tol in variants:
        opts = lt.make_opts(tol=tol, precision=prec, n_tau=p.n_tau, relax=args.relax, tau_adapt=args.tau_adapt,
                            precond=lt.LT_PRECOND_UNET_GMG if name == "learned" else lt.LT_PRECOND_GMG)
        prof_kind = lt.LT_PROF_POST_FINE if name == prof_name else 0
        dt, st, phi, prof = _run_variant(lt, hs, p, opts, args.steps, args.warmup, prof_kind)
        res[name] = dict(dt=dt, st=st, phi=phi, tol=tol, prof=prof)
        print(f"[bench] {name}: {dt * 1e3:.2f} ms/step, {pairs / dt:.0f} solves/s, iters {st['iters_max']}, "
              f"vcycles {st['vcycles']}, true residual {st['true_relres_max']:.2e}, net applied "
              f"{st['net_applied']} disabled after iteration {st['net_disabled_at']}", file=sys.stderr, flush=True)
    errs = {}
    if ref is not None:
        for name in res:
            got = res[name]["phi"][:, :, :nt]
            e = np.linalg.norm((got - ref).reshape(len(p.sources), -1), axis=1) / \
                np.linalg.norm(ref.reshape(len(p.sources), -1), axis=1)
            errs[name] = float(e.max())
        print(f"[bench] rel head err vs oracle sample: {errs}", file=sys.stderr, flush=True)
    if args.pmc_calibrate:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 536870912 bytes read and written", file=sys.stderr, flush=True)
    hname = "learned" if "learned" in res else ("mixed" if "mixed" in res else "fp64")
    head = res[hname]
    pr_src = res[prof_name]
    valid = (errs.get(hname, 0.0) <= 1e-5)
    pr = pr_src["prof"]
    roofline = None
    if pr["launches"] > 0 and pr["ms"] > 0:
        avg_s = pr["ms"] * 1e-3 / pr["launches"]
        bytes_per_launch = pr["bytes"] / pr["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        t0 = (tiles.get(prof_name) or {}).get("tiles") or [[32, 16]]
        tx, ty = t0[0]
        # the committed counter run used the 32x16 fine-level tile (and the FV operator)
        traffic = _measured_traffic() if (tx, ty) == (32, 16) and not args.p1 else None
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "kernel": f"k_post2d_refine<float,2,{tx},{ty}> (fine-grid prolongation, 2 red-black sweeps, "
                              "FP64 refinement update)",
                    "avg_launch_us": avg_s * 1e6, "bytes_per_launch": bytes_per_launch,
                    "launches": pr["launches"]}
    out = {
        "metric": "shifted solves/sec (RHS\u00d7shift, rel head err 1e-5): learned+mixed vs plain FGMRES",
        "value": pairs / head["dt"] if valid else 0.0,
        "unit": "shifted solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": ("2D P1 finite elements, 256x256 interior vertices of a 257x257-cell GRF aquifer "
                                "(right triangles, lumped mass)" if args.p1 else "2D 256x256 GRF aquifer") +
                               " (var 1, corr 0.1), 8 sources x 16 receivers, "
                               "10 times, 20-node Talbot, 1 tau, GMG V(2,2) RB-GS",
                   "rhs": len(p.sources), "shifts_per_rhs": len(p.times) * (p.nz_contour // 2),
                   "pairs": pairs, "tol": head["tol"], "relax": args.relax, "variant": hname, "tau_adapt": args.tau_adapt,
                   "precision": "FP32 V-cycle, FP64 outer",
                   "iters": head["st"]["iters_max"], "vcycles": head["st"]["vcycles"],
                   "source_groups": groups, "smoother_tiles": tiles, "n_tau": p.n_tau, **_boundary_config(p)},
        "variants": {
            name: {"solves_per_s": pairs / r["dt"], "ms_per_step": r["dt"] * 1e3, "tol": r["tol"],
                   "iters": r["st"]["iters_max"], "vcycles": r["st"]["vcycles"],
                   "true_relres_weighted_max": r["st"]["true_relres_max"],
                   "net_applied": r["st"]["net_applied"], "net_disabled_after_iteration": r["st"]["net_disabled_at"],
                   "rel_head_err_vs_oracle": errs.get(name)} for name, r in res.items()},
        "training": training,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "fp64" in res:
        out["vs_plain_fp64"] = (pairs / head["dt"]) / (pairs / res["fp64"]["dt"])
    print(json.dumps(out), flush=True)
    if net is not None:
        for hg in hs:
            lt.lt_unet_attach(hg, None)
        for ng in nets:
            ng.close()
    for hg in hs:
        hg.close()


def _tile_id(lt, shape):
    for i in range(16):
        try:
            if tuple(lt.lt_tile_shape(i)) == tuple(shape):
                return i
        except Exception:
            break
    raise ValueError(f"unknown tile shape {shape}")


def main_adjoint(args):
    """Sensitivities of the 64x64x32 workload: 25 sources and 48 receivers give 73 right-hand
    sides x 24 shifts = 1,752 shifted solves per lt_adjoint call, contracted to d phi / d ln kappa
    and d phi / d ln S of every cell for 25 x 48 x 2 (source, receiver, time) triples."""
    import workloads as wl
    p = _with_boundary(wl.make_problem("C3"), args)
    nrhs = len(p.sources) + len(p.receivers)
    pairs = nrhs * len(p.times) * (p.nz_contour // 2)
    cpu, ref = None, None
    if not args.no_cpu_baseline:
        # the oracle as it stands: the shifts of the first time (one factorisation each, all 73
        # right-hand sides), in parallel; their heads also check the GPU setup at full size
        from oracle.heads import heads
        workers = min(os.cpu_count() or 1, 16)
        t0 = time.perf_counter()
        ref = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times[:1], p.nz_contour, q=p.q, bc=p.bc,
                    workers=workers, ndim=p.ndim, sy=p.sy)
        dt = time.perf_counter() - t0
        nshift = p.nz_contour // 2
        cpu = {"value": nrhs * nshift / dt, "unit": "shifted solves/s", "cores": workers, "kind": "oracle",
               "sample": f"64x64x32 workload, first time: {nshift} shifts x {nrhs} right-hand sides "
                         f"(sources and receivers) = {nrhs * nshift} pairs, SuperLU per shift, "
                         f"{min(workers, nshift)} processes ({dt:.1f} s); no contraction"}
        print(f"[bench] oracle sample: {cpu['value']:.2f} solves/s ({dt:.1f} s)", file=sys.stderr, flush=True)
    import torch
    from paper_1409_2556_amd import binding as lt
    torch.cuda.set_device(0)
    h, tiles = _handle(lt, p, False, nrhs)
    res = {}
    for name, prec, tol in (("fp64", lt.LT_PREC_FP64, 1e-10), ("mixed", lt.LT_PREC_MIXED, 1e-9)):
        o = lt.make_opts(tol=tol, precision=prec, n_tau=p.n_tau, maxit=64, relax=args.relax_jacobian)
        out = None
        for _ in range(args.warmup):
            out = lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, o)
            del out
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        dK, dS, st = out
        res[name] = {"dt": dt, "tol": tol, "st": st, "dK": dK, "dS": dS}
        print(f"[bench] C3 adjoint {name}: {dt * 1e3:.1f} ms/step, {pairs / dt:.0f} solves/s, iters "
              f"{st['iters_max']}, true residual {st['true_relres_max']:.2e}", file=sys.stderr, flush=True)
    # mixed against FP64 sensitivities.  d/d ln kappa: per (source, receiver, time) field.  d/d ln S:
    # relative to the largest storage field of the same (source, receiver) over the times; near
    # steady state (the later time) the storage sensitivity is a vanishing difference of contour
    # terms of the earlier size, resolved to the tolerance of that scale, not of its own norm
    def rel(a, b, over_times=False):
        d = torch.linalg.vector_norm(a - b, dim=-1)
        n = torch.linalg.vector_norm(b, dim=-1)
        if over_times:
            n = n.max(dim=-1, keepdim=True).values
        return float((d / n).max())
    agree = {"dlnK": rel(res["mixed"]["dK"], res["fp64"]["dK"]),
             "dlnS_vs_scale_over_times": rel(res["mixed"]["dS"], res["fp64"]["dS"], True),
             "dlnS_per_field": rel(res["mixed"]["dS"], res["fp64"]["dS"])}
    head_err = None
    if ref is not None:
        o = lt.make_opts(tol=1e-9, precision=lt.LT_PREC_FP64, n_tau=p.n_tau, maxit=64)
        phi, _ = lt.lt_solve(h, p.sources, p.q, p.times[:1], p.nz_contour, p.receivers, o)
        got = phi.cpu().numpy()
        e = np.linalg.norm((got - ref).reshape(len(p.sources), -1), axis=1) / \
            np.linalg.norm(ref.reshape(len(p.sources), -1), axis=1)
        head_err = float(e.max())
    print(f"[bench] C3 mixed vs fp64 sensitivities {agree}, FP64 heads vs oracle {head_err}", file=sys.stderr,
          flush=True)
    head = res["mixed"]
    valid = (head["st"]["rc"] == 0 and agree["dlnK"] <= 1e-4 and agree["dlnS_vs_scale_over_times"] <= 1e-3
             and (head_err is None or head_err <= 1e-6))
    out = {
        "metric": "shifted solves/sec (RHS\u00d7shift, rel head err 1e-5): learned+mixed vs plain FGMRES",
        "value": pairs / head["dt"] if valid else 0.0,
        "unit": "shifted solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["dt"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "3D 64x64x32 GRF (var 2, corr 0.2/0.2/0.05), log-uniform S, 25 sources + 48 "
                               "receivers (adjoint), times {0.3, 1.2}, 24-node Talbot, 3 tau, lt_adjoint "
                               "(d phi / d ln kappa and d ln S of every cell)",
                   "rhs": nrhs, "pairs": pairs, "variant": "mixed", "tol": head["tol"], "relax": args.relax_jacobian,
                   "iters": head["st"]["iters_max"], "vcycles": head["st"]["vcycles"], "n_tau": p.n_tau,
                   **_boundary_config(p)},
        "variants": {n: {"solves_per_s": pairs / r["dt"], "ms_per_step": r["dt"] * 1e3, "tol": r["tol"],
                         "iters": r["st"]["iters_max"], "vcycles": r["st"]["vcycles"],
                         "true_relres_weighted_max": r["st"]["true_relres_max"]} for n, r in res.items()},
        "mixed_vs_fp64_sensitivity_rel_max": agree,
        "fp64_heads_vs_oracle_first_time": head_err,
        "vs_plain_fp64": res["fp64"]["dt"] / head["dt"],
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    h.close()


C5J_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c5j_gs_color_half_traffic.md")
C5J_KERNEL_SRC = (os.path.join(ROOT, "paper_1409_2556_amd", "csrc", "mg.hip"),
                  os.path.join(ROOT, "paper_1409_2556_amd", "csrc", "lt_internal.h"))
EXACT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "exact_k_ex_solve.md")
EXACT_KERNEL_SRC = os.path.join(ROOT, "paper_1409_2556_amd", "csrc", "exact.hip")


def _map_err(got, ref, scale=None):
    """Element-wise error of sensitivity maps [..., N]: max over maps of max_c |got - ref| / scale,
    scale = each map's largest |ref| (or the given one, broadcast over the maps)."""
    import torch
    d = (got - ref).abs().amax(dim=-1)
    n = ref.abs().amax(dim=-1) if scale is None else scale
    return float((d / n).max())


def _cpu_jacobian(p):
    """The oracle as it stands on a bounded sample: the full Jacobian (both maps, every well,
    receiver, time and cell) of the batch's 128x128 problem by SuperLU per shift."""
    from oracle.jacobian import jacobian
    workers = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    JK, JS = jacobian(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q, bc=p.bc,
                      workers=workers, ndim=p.ndim)
    dt = time.perf_counter() - t0
    nrhs = len(p.sources) + len(p.receivers)
    npair = nrhs * len(p.times) * (p.nz_contour // 2)
    return (JK, JS), {"value": npair / dt, "unit": "shifted solves/s", "cores": workers, "kind": "oracle",
                      "sample": f"the 128x128 problem of the batch: {len(p.sources)} wells + {len(p.receivers)} "
                                f"receivers x {len(p.times)} times x {p.nz_contour // 2} shifts = {npair} pairs, "
                                f"SuperLU per shift, contracted to both sensitivity maps of all cells "
                                f"({dt:.1f} s)"}


def main_jacobian(args):
    """The six Jacobian-assembly problems (128^2, 256^2, 512^2, 32^3, 64^3, 128x128x64; 16 wells +
    32 receivers, 2 times, 24-node contour each) in one lt_adjoint_batch call per step."""
    import workloads as wl
    ps = wl.make_batch()
    nrhs = [len(p.sources) + len(p.receivers) for p in ps]
    pairs = sum(n * len(p.times) * (p.nz_contour // 2) for n, p in zip(nrhs, ps))
    small = ps[0]
    cpu, ref = None, None
    if not args.no_cpu_baseline:
        ref, cpu = _cpu_jacobian(small)
        print(f"[bench] oracle sample: {cpu['value']:.2f} solves/s, {cpu['sample']}", file=sys.stderr, flush=True)
    import torch
    from paper_1409_2556_amd import binding as lt
    torch.cuda.set_device(0)
    hs, tiles = [], {}
    for p, n in zip(ps, nrhs):
        h, t = _handle(lt, p, not args.no_tune, n)
        hs.append(h)
        tiles[p.name] = t
    outs = [(torch.empty((len(p.sources), len(p.receivers), len(p.times), p.N), dtype=torch.float64, device="cuda"),
             torch.empty((len(p.sources), len(p.receivers), len(p.times), p.N), dtype=torch.float64, device="cuda"))
            for p in ps]
    # the same cells of every problem are compared between variants (the maps' scales come from
    # all cells of the FP64 run)
    gen = torch.Generator(device="cpu").manual_seed(7)
    samp = [torch.randperm(p.N, generator=gen)[:min(p.N, 8192)].cuda() for p in ps]
    net_2d = [p.ndim == 2 and p.n[0] % 128 == 0 and p.n[1] % 8 == 0 for p in ps]
    training, nets = None, []
    tol = args.tol_jacobian
    variants = [("fp64", lt.LT_PREC_FP64), ("mixed", lt.LT_PREC_MIXED), ("learned", lt.LT_PREC_MIXED)]
    if args.variant != "all":
        variants = [v for v in variants if v[0] in (args.variant, "fp64")]
    if any(v[0] == "learned" for v in variants):
        from paper_1409_2556_amd.train_unet import train
        t0 = time.perf_counter()
        net, hist = train(steps=args.train_steps, batch=8, lr=1e-3, verbose=False)
        torch.cuda.synchronize()
        training = {"steps": args.train_steps, "seconds": time.perf_counter() - t0,
                    "final_loss_mean20": float(np.mean(hist[-20:])),
                    "data": "128x128 GRF fields (seeds 10000-10007), point-source and smooth residuals, "
                            "targets from lt_precond_solve"}
        print(f"[bench] trained U-Net: {training['seconds']:.1f} s, loss {training['final_loss_mean20']:.3f}",
              file=sys.stderr, flush=True)
        first = True
        for h, ok in zip(hs, net_2d):
            if ok:
                # one copy per handle: a network's workspace serves one solve at a time
                if first:
                    ng, first = net, False
                else:
                    ng = lt.UNet(seed=0)
                    ng.set_params(net.get_params())
                nets.append(ng)
                lt.lt_unet_attach(h, ng)
    res, fp64_samp = {}, None
    for name, prec in variants:
        opts = [lt.make_opts(tol=tol, precision=prec, n_tau=p.n_tau, maxit=args.maxit, relax=args.relax_jacobian,
                             tau_adapt=args.tau_adapt,
                             precond=lt.LT_PRECOND_UNET_GMG if (name == "learned" and ok) else lt.LT_PRECOND_GMG,
                             **({"nu1": args.nu3d, "nu2": args.nu3d} if p.ndim == 3 else {}))
                for p, ok in zip(ps, net_2d)]
        items = [dict(handle=h, sources=p.sources, q=p.q, receivers=p.receivers, times=p.times, nz=p.nz_contour,
                      opts=o, dlnK=dK, dlnS=dS) for p, h, o, (dK, dS) in zip(ps, hs, opts, outs)]
        sts, rc = None, None
        for _ in range(args.warmup):
            _, sts, rc = lt.lt_adjoint_batch(items)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, sts, rc = lt.lt_adjoint_batch(items)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        r = {"dt": dt, "tol": tol, "rc": rc, "sts": sts}
        if ref is not None:
            dK, dS = outs[0]
            rK = torch.from_numpy(ref[0]).cuda()
            rS = torch.from_numpy(ref[1]).cuda()
            r["oracle_128"] = {"dlnK": _map_err(dK, rK),
                               "dlnS_vs_scale_over_times": _map_err(dS, rS, rS.abs().amax(dim=(-2, -1))[..., None]),
                               "dlnS_per_map": _map_err(dS, rS)}
            del rK, rS
        cur = [(dK[..., i], dS[..., i]) for (dK, dS), i in zip(outs, samp)]
        if name == "fp64":
            scales = [(dK.abs().amax(dim=-1), dS.abs().amax(dim=(-2, -1))[..., None]) for dK, dS in outs]
            fp64_samp = [(a.clone(), b.clone(), sc) for (a, b), sc in zip(cur, scales)]
        else:
            r["vs_fp64_sampled"] = {
                p.name: {"dlnK": _map_err(a, fa, sk), "dlnS_vs_scale_over_times": _map_err(b, fb, ss)}
                for p, (a, b), (fa, fb, (sk, ss)) in zip(ps, cur, fp64_samp)}
        res[name] = r
        print(f"[bench] C5J {name}: {dt * 1e3:.1f} ms/step, {pairs / dt:.0f} solves/s, rc {rc}, oracle_128 "
              f"{r.get('oracle_128')}, vs fp64 {r.get('vs_fp64_sampled')}", file=sys.stderr, flush=True)
        for p, st in zip(ps, sts):
            print(f"[bench]   {p.name}: iters {st['iters_max']} vcycles {st['vcycles']} resolves "
                  f"{st['resolves']} true {st['true_relres_max']:.2e} net {st['net_applied']} "
                  f"({st['seconds'] * 1e3:.1f} ms)", file=sys.stderr, flush=True)
    # the dominant solver kernel, timed live: the one-colour Gauss-Seidel half-sweep on the fine
    # level of the largest (3D) problem, every launch bracketed by HIP events on its handle's
    # stream, in a pass of its own (the same call with the same right-hand sides, outside the
    # timed steps)
    roofline = None
    pname = "learned" if "learned" in res else "mixed"
    if pname in res:
        big = max(range(len(ps)), key=lambda i: ps[i].N)
        p, h = ps[big], hs[big]
        o = lt.make_opts(tol=tol, precision=lt.LT_PREC_MIXED, n_tau=p.n_tau, maxit=args.maxit,
                         relax=args.relax_jacobian, profile=lt.LT_PROF_SWEEP3D, tau_adapt=args.tau_adapt,
                         **({"nu1": args.nu3d, "nu2": args.nu3d} if p.ndim == 3 else {}))
        dK, dS = outs[big]
        _, _, stp = lt.lt_adjoint(h, p.sources, p.q, p.receivers, p.times, p.nz_contour, o, dlnK=dK, dlnS=dS)
        torch.cuda.synchronize()
        if stp["prof_launches"] > 0 and stp["prof_ms"] > 0:
            avg_s = stp["prof_ms"] * 1e-3 / stp["prof_launches"]
            bpl = stp["prof_bytes"] / stp["prof_launches"]
            ach = bpl / avg_s / 1e9
            roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "traffic": _measured_traffic(C5J_TRAFFIC_FILE, C5J_KERNEL_SRC),
                        "kernel": "k_gs_color_half<float> (one red-black colour of a Gauss-Seidel sweep on "
                                  "the fine level of the 128x128x64 problem, all right-hand sides of a launch)",
                        "avg_launch_us": avg_s * 1e6, "bytes_per_launch": bpl, "launches": stp["prof_launches"]}
    if args.pmc_calibrate:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 536870912 bytes read and written", file=sys.stderr, flush=True)
    hname = "learned" if "learned" in res else ("mixed" if "mixed" in res else "fp64")
    head = res[hname]
    o128 = head.get("oracle_128")
    valid = head["rc"] == 0 and (o128 is None or (o128["dlnK"] <= 1e-5 and o128["dlnS_vs_scale_over_times"] <= 1e-5))
    out = {
        "metric": "shifted solves/sec (RHS\u00d7shift, rel head err 1e-5): learned+mixed vs plain FGMRES",
        "value": pairs / head["dt"] if valid else 0.0,
        "unit": "shifted solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["dt"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "six Jacobian-assembly problems on uneven grids (128^2, 256^2, 512^2 2D; 32^3, "
                               "64^3, 128x128x64 3D), 16 wells + 32 receivers each, times {0.3, 1.2}, "
                               "24-node Talbot, sensitivities d phi / d ln kappa and d ln S of every cell, "
                               "one lt_adjoint_batch call",
                   "pairs": pairs, "rhs_per_problem": nrhs, "variant": hname, "tol": tol, "maxit": args.maxit,
                   "tau_adapt": args.tau_adapt,
                   "relax": args.relax_jacobian,
                   "accuracy": "sensitivity maps of the 128x128 problem vs the oracle, element-wise, relative "
                               "to each map's largest entry (storage: to the largest over both times)",
                   "smoother_tiles": tiles},
        "variants": {n: {"solves_per_s": pairs / r["dt"], "ms_per_step": r["dt"] * 1e3, "tol": r["tol"], "rc": r["rc"],
                         "vs_oracle_128": r.get("oracle_128"), "vs_fp64_sampled": r.get("vs_fp64_sampled"),
                         "per_problem": {p.name: {"iters": s["iters_max"], "vcycles": s["vcycles"],
                                                  "resolves": s["resolves"],
                                                  "true_relres_weighted_max": s["true_relres_max"],
                                                  "net_applied": s["net_applied"],
                                                  "net_disabled_after_iteration": s["net_disabled_at"],
                                                  "solve_ms": s["seconds"] * 1e3}
                                         for p, s in zip(ps, r["sts"])}}
                     for n, r in res.items()},
        "training": training,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "fp64" in res:
        out["vs_plain_fp64"] = res["fp64"]["dt"] / head["dt"]
    if "mixed" in res and hname == "learned":
        out["learned_vs_mixed"] = res["mixed"]["dt"] / head["dt"]
    print(json.dumps(out), flush=True)
    for h in hs:
        lt.lt_unet_attach(h, None)
    for ng in nets:
        ng.close()
    for h in hs:
        h.close()


def main_batch(args):
    """The six-grid batch (128^2, 256^2, 512^2, 32^3, 64^3, 128x128x64; 16 sources, 32 receivers,
    2 times, 24-node contour each) in one lt_solve_batch call per step."""
    import workloads as wl
    ps = wl.make_batch()
    pairs = sum(len(p.sources) * len(p.times) * (p.nz_contour // 2) for p in ps)
    cpu, ref = None, None
    small = ps[0]  # the oracle sample: the 128x128 problem, first time
    if not args.no_cpu_baseline:
        from oracle.heads import heads
        workers = min(os.cpu_count() or 1, 16)
        t0 = time.perf_counter()
        ref = heads(small.n, small.h, small.kappa, small.S, small.sources, small.receivers, small.times[:1],
                    small.nz_contour, q=small.q, bc=small.bc, workers=workers, ndim=small.ndim)
        dt = time.perf_counter() - t0
        npair = len(small.sources) * (small.nz_contour // 2)
        cpu = {"value": npair / dt, "unit": "shifted solves/s", "cores": workers, "kind": "oracle",
               "sample": f"the 128x128 problem of the batch: {len(small.sources)} sources x first time x "
                         f"{small.nz_contour // 2} shifts = {npair} pairs, SuperLU per shift ({dt:.1f} s)"}
        print(f"[bench] oracle sample: {cpu['value']:.2f} solves/s", file=sys.stderr, flush=True)
    import torch
    from paper_1409_2556_amd import binding as lt
    torch.cuda.set_device(0)
    hs, tiles = [], {}
    for p in ps:
        h, t = _handle(lt, p, not args.no_tune, len(p.sources))
        hs.append(h)
        tiles[p.name] = t
    res = {}
    # mixed tol 3e-9: the 1e-5 head bar holds on every grid of the batch (the largest 3D grid needs it)
    for name, prec, tol in (("fp64", lt.LT_PREC_FP64, 1e-9), ("mixed", lt.LT_PREC_MIXED, 3e-9)):
        opts = [lt.make_opts(tol=tol, precision=prec, n_tau=p.n_tau, maxit=64, relax=args.relax_jacobian) for p in ps]
        items = [dict(handle=h, sources=p.sources, q=p.q, times=p.times, nz=p.nz_contour, receivers=p.receivers,
                      opts=o) for p, h, o in zip(ps, hs, opts)]
        for _ in range(args.warmup):
            outs, sts, rc = lt.lt_solve_batch(items)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            outs, sts, rc = lt.lt_solve_batch(items)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        err = None
        if ref is not None:
            got = outs[0].cpu().numpy()[:, :, :1]
            e = np.linalg.norm((got - ref).reshape(len(small.sources), -1), axis=1) / \
                np.linalg.norm(ref.reshape(len(small.sources), -1), axis=1)
            err = float(e.max())
        res[name] = {"dt": dt, "tol": tol, "err": err, "rc": rc,
                     "per_problem": {p.name: {"iters": s["iters_max"], "vcycles": s["vcycles"],
                                              "true_relres_weighted_max": s["true_relres_max"],
                                              "solve_ms": s["seconds"] * 1e3} for p, s in zip(ps, sts)}}
        print(f"[bench] C5 {name}: {dt * 1e3:.1f} ms/step, {pairs / dt:.0f} solves/s, err {err}", file=sys.stderr,
              flush=True)
    head = res["mixed"]
    valid = head["rc"] == 0 and (head["err"] is None or head["err"] <= 1e-5)
    out = {
        "metric": "shifted solves/sec (RHS\u00d7shift, rel head err 1e-5): learned+mixed vs plain FGMRES",
        "value": pairs / head["dt"] if valid else 0.0,
        "unit": "shifted solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["dt"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "batch of six uneven grids (128^2, 256^2, 512^2, 32^3, 64^3, 128x128x64), "
                               "16 sources x 32 receivers each, times {0.3, 1.2}, 24-node Talbot, "
                               "lt_solve_batch (one stream per problem)",
                   "pairs": pairs, "variant": "mixed", "relax": args.relax_jacobian, "smoother_tiles": tiles},
        "variants": {n: {"solves_per_s": pairs / r["dt"], "ms_per_step": r["dt"] * 1e3, "tol": r["tol"],
                         "rel_head_err_vs_oracle_128": r["err"], "per_problem": r["per_problem"]}
                     for n, r in res.items()},
        "vs_plain_fp64": res["fp64"]["dt"] / head["dt"],
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    for h in hs:
        h.close()


def main_block(args):
    """Block flexible GMRES for shifted systems (lt_shifted_solve_block) on the 256x256 heads
    workload: its 8 wells and 16 receivers (the Jacobian's 24 right-hand sides, unit point
    sources) at the 10 contour shifts of its time nearest 0.3 t_D (4.6e-6: the fields of different
    sources overlap; at its first time, 0.01 t_D, each stays near its own cell and blocks share
    nothing), tol 1e-8 per shift, blocks of 1, 4 and 8
    columns; the exact shift-and-invert preconditioner (the paper's two-shift schedule) and
    multigrid in FP64 and in FP32 under FP64 refinement (the shift of largest real part, then the
    largest imaginary part alone)."""
    import workloads as wl
    from oracle.contour import talbot_nodes
    p = wl.make_problem(WORKLOAD)
    pts = np.vstack([p.sources, p.receivers])
    R = pts.shape[0]
    t_blk = float(p.times[np.argmin(np.abs(p.times - 0.3 * wl.configs.T_D))])
    z = talbot_nodes(p.nz_contour, t_blk)[0]
    nk = z.size
    zr, zi = z[np.argmax(z.real)], z[np.argmax(np.abs(z.imag))]
    taus = {"exact": [z[np.argmin(z.real)]] * 3 + [zr] * 2, "gmg": [zr, complex(0.0, zi.imag)]}
    taus["gmgmixed"] = taus["gmg"]
    tol = 1e-8
    cpu, sample = None, None
    if not args.no_cpu_baseline:
        # the oracle's block algorithm (SuperLU preconditioner solves) on the first block of 4
        # columns at the shifts of the first time
        from oracle.block import block_flexible_shifted
        from oracle.fv import assemble
        K, m = assemble(p.n, p.h, p.kappa, p.S, bc=p.bc, sy=p.sy)
        N = int(np.prod(p.n[:p.ndim]))
        B = np.zeros((N, 4))
        B[_cells_of(p, pts[:4]), np.arange(4)] = 1.0
        zs = z
        t0 = time.perf_counter()
        orc = block_flexible_shifted(K, m, B, taus["exact"], zs, tol=tol, maxit=60)
        dt = time.perf_counter() - t0
        sample = (zs, orc["x"])
        cpu = {"value": 4 * zs.size / dt, "unit": "shifted solves/s", "cores": 1, "kind": "oracle",
               "sample": f"block FGMRES-Sh of the oracle, first block of 4 columns x the "
                         f"{zs.size} shifts, exact preconditioner ({orc['iters']} steps, {dt:.1f} s)"}
        print(f"[bench] oracle sample: {cpu['value']:.2f} solves/s", file=sys.stderr, flush=True)
    import torch
    from paper_1409_2556_amd import binding as lt
    torch.cuda.set_device(0)
    h, _ = _handle(lt, p, False, R)
    # right-hand sides: unit vectors at the cells holding the wells and receivers (plain indexing)
    cells = _cells_of(p, pts)
    b = torch.zeros((R, 2, h.N), dtype=torch.float64, device="cuda")
    b[torch.arange(R, device="cuda"), 0, torch.tensor(cells, device="cuda")] = 1.0
    x = torch.empty((nk, R, 2, h.N), dtype=torch.float64, device="cuda")
    res = {}
    for pre in ("exact", "gmg", "gmgmixed"):
        for blk in (1, 4, 8):
            o = lt.make_opts(tol=tol, maxit=60, precond=lt.LT_PRECOND_EXACT if pre == "exact" else lt.LT_PRECOND_GMG,
                             precision=lt.LT_PREC_MIXED if pre == "gmgmixed" else lt.LT_PREC_FP64)
            for _ in range(args.warmup):
                lt.lt_shifted_solve_block(h, z, b, blk, taus[pre], o, x=x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, st = lt.lt_shifted_solve_block(h, z, b, blk, taus[pre], o, x=x)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            r = {"ms_per_step": dt * 1e3, "solves_per_s": R * nk / dt, "rc": st["rc"], "steps_max": st["iters_max"],
                 "steps_mean": float(np.mean(st["iters_per_rhs"])),
                 "precond_applications": int(np.sum(st["iters_per_rhs"])), "vcycles": st["vcycles"],
                 "true_relres_max": st["true_relres_max"]}
            if sample is not None and pre == "exact" and blk == 4:
                got = x[:sample[0].size, :4].cpu().numpy()
                got = got[:, :, 0] + 1j * got[:, :, 1]
                r["rel_err_vs_oracle_sample"] = float(max(
                    np.abs(got[k, c] - sample[1][k][:, c]).max() / np.abs(sample[1][k][:, c]).max()
                    for k in range(sample[0].size) for c in range(4)))
            res[f"{pre}_block{blk}"] = r
            print(f"[bench] BLOCK {pre} p {blk}: {r}", file=sys.stderr, flush=True)
    head = res["exact_block4"]
    valid = head["rc"] == 0 and head["true_relres_max"] <= tol and \
        head.get("rel_err_vs_oracle_sample", 0.0) <= 1e-6
    out = {
        "metric": "shifted solves/sec (RHS\u00d7shift, true residual 1e-8): block flexible GMRES",
        "value": R * nk / (head["ms_per_step"] * 1e-3) if valid else 0.0,
        "unit": "shifted solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"256x256 heads workload's {R} Jacobian right-hand sides (8 wells, 16 receivers; "
                               f"unit vectors at their cells) x {nk} contour shifts (time {t_blk:.3g}, 20-node Talbot), "
                               "lt_shifted_solve_block, exact preconditioner, blocks of 4", "tol": tol},
        "variants": res,
        "block4_vs_single_exact": res["exact_block1"]["ms_per_step"] / head["ms_per_step"],
        "block4_vs_single_gmg": res["gmg_block1"]["ms_per_step"] / res["gmg_block4"]["ms_per_step"],
        "block4_vs_single_gmg_mixed": res["gmgmixed_block1"]["ms_per_step"] / res["gmgmixed_block4"]["ms_per_step"],
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    h.close()


def _cells_of(p, pts):
    """Index of the cell holding each point (x fastest)."""
    d = p.ndim
    idx = np.zeros(len(pts), dtype=np.int64)
    stride = 1
    for a in range(d):
        i = np.clip(np.floor(pts[:, a] / p.h[a]).astype(np.int64), 0, p.n[a] - 1)
        idx += i * stride
        stride *= p.n[a]
    return idx


def _exact_problem(wl, var=1.6, n=(128, 128), t=0.3, wells=None):
    """The single-well test (W1: one well at the centre, receivers at (0.7, 0.7) and its mirror
    images, 40-node contour) with the given variance, grid and time (diffusion times)."""
    from dataclasses import replace
    p = wl.make_problem("W1", n=n, var=var)
    p = replace(p, times=np.array([t]) * wl.configs.T_D)
    if wells is not None:
        p = replace(p, sources=wells)
    return p


def main_exact(args):
    """Section 4.1's single-well test with the exact shift-and-invert preconditioner: per case, the
    'Single' solver (tau_bar_1, the contour node of smallest real part) and the 'Flexible' one
    (tau_bar_1 three times, tau_bar_2 (largest real part) twice, repeated), relative tolerance
    1e-10.  One step is one lt_solve with the factorisations of the schedule's shifts cached on the
    handle (their time, on the first call, is reported separately as factor_ms)."""
    import workloads as wl
    import workloads.configs  # noqa: F401  (T_D)
    tol = 1e-10
    head_p = _exact_problem(wl)
    nshift = head_p.nz_contour // 2
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.contour import talbot_nodes
        from oracle.fv import assemble, point_weights
        from oracle.krylov import flexible_shifted, tau_schedule
        try:
            from threadpoolctl import threadpool_limits
            threadpool_limits(1)
        except Exception:
            pass
        K, m = assemble(head_p.n, head_p.h, head_p.kappa, head_p.S)
        b = point_weights(head_p.n, head_p.h, head_p.sources).toarray()[0]
        z = talbot_nodes(head_p.nz_contour, head_p.times[0])[0]
        reps, t0 = 0, time.perf_counter()
        while reps < 3 or time.perf_counter() - t0 < 10.0:
            out = flexible_shifted(K, m, b, tau_schedule(z, 2), z, tol, 400)
            reps += 1
        dt = (time.perf_counter() - t0) / reps
        cpu = {"value": nshift / dt, "unit": "shifted solves/s", "cores": 1, "kind": "oracle",
               "sample": f"the oracle's Algorithm 1 (SuperLU per preconditioner shift, 'Flexible' schedule) on "
                         f"the headline case: 1 well x {nshift} shifts, {out['iters']} iterations, "
                         f"{reps} repetitions ({dt * reps:.1f} s)"}
        print(f"[bench] oracle Algorithm 1: {cpu['value']:.2f} solves/s ({dt * 1e3:.0f} ms/solve)", file=sys.stderr,
              flush=True)
    import torch
    from paper_1409_2556_amd import binding as lt
    from oracle.heads import heads_problem
    torch.cuda.set_device(0)

    def handle(p):
        kap = torch.tensor(p.kappa, dtype=torch.float64, device="cuda")
        S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
        return lt.lt_setup(p.ndim, p.n, p.h, kap, S, bc=p.bc, sy=p.sy)

    def run(p, n_tau, check=False, profile=0, **extra):
        h = handle(p)
        o = lt.make_opts(tol=tol, maxit=400, n_tau=n_tau, precond=lt.LT_PRECOND_EXACT, conv=lt.LT_CONV_RELATIVE,
                         **extra)
        phi, st0 = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
        for _ in range(args.warmup):
            lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        r = {"iters": int(st["iters_max"]), "ms": dt * 1e3, "factor_ms": st0["factor_ms"],
             "factorizations": st0["factorizations"], "rc": st["rc"],
             "solves_per_s": len(p.sources) * nshift / dt, "true_relres_max": st["true_relres_max"]}
        if check:
            ref = heads_problem(p)
            got = phi.cpu().numpy()
            r["rel_head_err"] = float((np.abs(got - ref).max(axis=(1, 2)) / np.abs(ref).max(axis=(1, 2))).max())
        if profile:
            op = lt.make_opts(tol=tol, maxit=400, n_tau=n_tau, precond=lt.LT_PRECOND_EXACT,
                              conv=lt.LT_CONV_RELATIVE, profile=profile)
            _, sp_ = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, op)
            r["prof"] = {"launches": sp_["prof_launches"], "ms": sp_["prof_ms"], "bytes": sp_["prof_bytes"]}
        h.close()
        return r

    tables = {"variance_128": {}, "time_128_var1.6": {}, "grid_var1.6": {}, "fom_restart_128": {}}
    for var in ((0.8, 1.6, 3.5) if args.exact_cases == "all" else ()):
        p = _exact_problem(wl, var=var)
        tables["variance_128"][str(var)] = {s: run(p, nt, check=True) for s, nt in (("single", 1), ("flexible", 2))}
        print(f"[bench] EXACT var {var}: {tables['variance_128'][str(var)]}", file=sys.stderr, flush=True)
    for t in ((0.06, 1.2) if args.exact_cases == "all" else ()):
        p = _exact_problem(wl, t=t)
        tables["time_128_var1.6"][str(t)] = {s: run(p, nt, check=True) for s, nt in (("single", 1), ("flexible", 2))}
        print(f"[bench] EXACT t {t}: {tables['time_128_var1.6'][str(t)]}", file=sys.stderr, flush=True)
    for n in ((64, 256, 512) if args.exact_cases == "all" else ()):
        p = _exact_problem(wl, n=(n, n))
        tables["grid_var1.6"][f"{n}^2"] = {s: run(p, nt) for s, nt in (("single", 1), ("flexible", 2))}
        print(f"[bench] EXACT grid {n}: {tables['grid_var1.6'][f'{n}^2']}", file=sys.stderr, flush=True)
    # the FOM variant restarted every m steps from its collinear residuals (0: never), the
    # headline problem: the basis holds m columns instead of all of them
    for m in ((0, 5, 10, 20) if args.exact_cases == "all" else ()):
        tables["fom_restart_128"][str(m)] = run(head_p, 2, check=True, method=lt.LT_METHOD_FOM, restart=m)
        print(f"[bench] EXACT FOM restart {m}: {tables['fom_restart_128'][str(m)]}", file=sys.stderr, flush=True)
    head = run(head_p, 2, check=True, profile=lt.LT_PROF_EXACT)
    wells = np.asarray(wl.configs._C2_WELLS, dtype=np.float64)
    multi = None
    if args.exact_cases != "one":
        multi = run(_exact_problem(wl, wells=wells), 2, check=True, profile=lt.LT_PROF_EXACT)
    print(f"[bench] EXACT headline {head}\n[bench] EXACT 16 wells {multi}", file=sys.stderr, flush=True)
    if args.pmc_calibrate:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 536870912 bytes read and written", file=sys.stderr, flush=True)

    def roof(r, what, traffic=None):
        pr = r["prof"]
        avg = pr["ms"] / max(pr["launches"], 1) * 1e-3
        per = pr["bytes"] / max(pr["launches"], 1)
        ach = per / avg / 1e9 if avg > 0 else 0.0
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": traffic, "kernel": f"k_ex_solve (dense block products of the exact solve, {what})",
                "avg_launch_us": avg * 1e6, "bytes_per_launch": per, "launches": pr["launches"]}

    valid = head["rc"] == 0 and head["rel_head_err"] <= 1e-5
    out = {
        "metric": "shifted solves/sec (RHS×shift, rel head err 1e-5): learned+mixed vs plain FGMRES",
        "value": head["solves_per_s"] if valid else 0.0,
        "unit": "shifted solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "single-well test of Section 4.1: 128x128 GRF (ln kappa variance 1.6, corr 0.2), "
                               "one well at the centre, 4 receivers, the 5-minute sample (0.3 diffusion times), "
                               "40-node Talbot (20 shifts), relative tolerance 1e-10, exact shift-and-invert "
                               "preconditioner, 'Flexible' schedule",
                   "precond": "exact (block cyclic reduction, factorised once per shift)",
                   "factor_ms_per_shift": head["factor_ms"] / max(head["factorizations"], 1),
                   "iters": head["iters"], "rel_head_err_vs_oracle": head["rel_head_err"]},
        "tables": tables,
        "sixteen_wells": {k: v for k, v in multi.items() if k != "prof"} if multi else None,
        "roofline": roof(head, "one well", _measured_traffic(EXACT_TRAFFIC_FILE, EXACT_KERNEL_SRC)),
        "roofline_sixteen_wells": roof(multi, "16 wells") if multi else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main_tht(args):
    """Transient hydraulic tomography (Section 5.3): the quasi-linear geostatistical inversion
    (Algorithm 2) of ln kappa on 100x100 cells from one pumping well, 36 observation wells and the
    8, 10 and 20 minute samples (108 measurements with 2 % noise), 20-node contour.  One step is
    one whole inversion of --tht-iters Gauss-Newton iterations, each: the operator for exp(s_k),
    the heads, the Jacobian by the adjoint (1 well + 36 receivers = 37 right-hand sides x 30
    shifts), Q J^T, the saddle-point system and s_{k+1}.  The data are the heads of the true field
    by the GPU's own forward solve on a finer (40-node) contour, plus the noise."""
    import workloads as wl
    p = wl.make_problem("THT")
    iters = args.tht_iters
    var, ell = 1.0, (0.2, 0.2, 0.2)
    nshift = (p.nz_contour // 2) * len(p.times)
    per_iter = (len(p.sources) + len(p.sources) + len(p.receivers)) * nshift  # forward + adjoint shifted solves
    M = len(p.sources) * len(p.receivers) * len(p.times)
    rng = np.random.default_rng(11)
    noise = rng.standard_normal(M)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.geostat import exp_covariance, gauss_newton_step
        from oracle.heads import heads
        workers = min(os.cpu_count() or 1, 16)
        y0 = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, 40, ndim=2, workers=workers).ravel()
        yc = y0 * (1 + 0.02 * noise)
        rc_ = (0.02 * np.sqrt(np.mean(y0 ** 2))) ** 2
        t0 = time.perf_counter()
        Q = exp_covariance(p.n, p.h, var, ell, 2)
        gauss_newton_step(p.n, p.h, np.zeros(p.N), p.S, p.sources, p.receivers, p.times, p.nz_contour, yc, var, ell,
                          rc_, ndim=2, Q=Q, workers=workers)
        dt = time.perf_counter() - t0
        cpu = {"value": per_iter / dt, "unit": "shifted solves/s", "cores": workers, "kind": "oracle",
               "sample": f"one Gauss-Newton step of the oracle's Algorithm 2 on the same problem (heads and "
                         f"Jacobian by SuperLU per shift, dense Q, {per_iter} shifted solves, {dt:.1f} s)"}
        print(f"[bench] oracle Gauss-Newton step: {dt:.1f} s, {cpu['value']:.1f} solves/s", file=sys.stderr,
              flush=True)
    import torch
    from paper_1409_2556_amd import binding as lt
    torch.cuda.set_device(0)
    kap = torch.tensor(p.kappa, dtype=torch.float64, device="cuda")
    S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
    h = lt.lt_setup(p.ndim, p.n, p.h, kap, S, bc=p.bc)
    data_opts = lt.make_opts(tol=1e-10, maxit=200)
    phi, _ = lt.lt_solve(h, p.sources, p.q, p.times, 40, p.receivers, data_opts)
    if args.tht_precond == "exact":
        opts = lt.make_opts(tol=1e-10, maxit=200, n_tau=2, precond=lt.LT_PRECOND_EXACT)
    else:
        opts = lt.make_opts(tol=1e-10, maxit=200)
    y0 = phi.cpu().numpy().ravel()
    y = torch.tensor(y0 * (1 + 0.02 * noise), dtype=torch.float64, device="cuda")
    r = (0.02 * np.sqrt(np.mean(y0 ** 2))) ** 2
    s0 = torch.zeros(p.N, dtype=torch.float64, device="cuda")

    def invert(k):
        return lt.lt_geostat_invert(p.ndim, p.n, p.h, S, p.sources, p.q, p.receivers, p.times, p.nz_contour, var,
                                    ell, r, y, s0, k, opts=opts)

    for _ in range(args.warmup):
        invert(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s_est, mis, stp, rc = invert(iters)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    s_true = np.log(p.kappa)
    se = s_est.cpu().numpy()
    x = (np.arange(p.n[0]) + 0.5) * p.h[0]
    X, Y = np.meshgrid(x, (np.arange(p.n[1]) + 0.5) * p.h[1], indexing="xy")
    box = ((X >= 0.2) & (X <= 0.8) & (Y >= 0.2) & (Y <= 0.8)).ravel()
    err_box = float(np.linalg.norm((se - s_true)[box]) / np.linalg.norm(s_true[box]))
    err_all = float(np.linalg.norm(se - s_true) / np.linalg.norm(s_true))
    print(f"[bench] THT: {dt * 1e3:.1f} ms per inversion of {iters} iterations, misfit {mis}, steps {stp}, "
          f"error box {err_box:.3f} all {err_all:.3f}, rc {rc}", file=sys.stderr, flush=True)
    # the covariance product, timed live on the handle's stream (torch's current stream)
    J = torch.randn(M, p.N, dtype=torch.float64, device="cuda")
    out = torch.empty_like(J)
    lt.lt_cov_apply(h, var, ell, J, out, M)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        lt.lt_cov_apply(h, var, ell, J, out, M)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / reps * 1e3
    flops = 2.0 * p.N * p.N * M  # one multiply-add per (row, column, vector)
    ach = flops / (us * 1e-6) / 1e12
    h.close()
    valid = rc == 0 and mis[-1] < mis[0]
    out_line = {
        "metric": "shifted solves/sec (RHS×shift, rel head err 1e-5): learned+mixed vs plain FGMRES",
        "value": per_iter * iters / dt if valid else 0.0,
        "unit": "shifted solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "transient hydraulic tomography of Section 5.3: geostatistical inversion "
                               "(Algorithm 2) of ln kappa on 100x100 cells, 1 pumping well, 36 observation "
                               "wells in [0.2, 0.8]^2, times 0.48/0.6/1.2 diffusion times, 108 measurements "
                               "with 2 % noise, exponential prior (var 1, length 0.2), 20-node contour, "
                               f"{iters} Gauss-Newton iterations per step",
                   "precond": args.tht_precond,
                   "shifted_solves_per_iteration": per_iter, "measurements": M,
                   "misfit_per_iteration": [float(v) for v in mis],
                   "relative_step_per_iteration": [float(v) for v in stp],
                   "rel_l2_error_box": err_box, "rel_l2_error_all": err_all},
        "roofline": {"bound": "alu", "achieved": ach, "peak": 78.6, "unit": "TFLOP/s", "frac": ach / 78.6,
                     "traffic": None,
                     "kernel": f"k_cov_apply (Q J^T for {M} rows of J: the exponential covariance evaluated in "
                               "LDS tiles, one FP64 multiply-add per (cell, cell, row))",
                     "avg_launch_us": us, "flops_per_launch": flops},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out_line), flush=True)


if __name__ == "__main__":
    main()
