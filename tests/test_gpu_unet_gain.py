"""What the trained network gains over the method without it: unseen 256x256
and 512x512 fields, 8 right-hand sides x 20 shifts, stop at 1e-5 (the
learned-preconditioner workload).  Reports iterations, V-cycles and time of
plain GMG, GMG with the network forced on, and the adaptive default.  With
N_z = 40 nodes the contour sum amplifies shift residuals by about
exp(0.171 N_z) ~ 930, so a 1e-5 residual stop bounds head errors by ~1e-2;
the test asserts that bound against a tight FP64 solve and that the network
variants are no less accurate than GMG -- the gain itself is measured, not
assumed."""
import time

import numpy as np
import pytest

import workloads as wl
from gpu_util import device_problem, rel_err_per_source, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained(lt):
    from paper_1409_2556_amd.train_unet import train
    net, hist = train(steps=400, batch=8, lr=1e-3, verbose=False)
    print("training loss (mean of last 20 steps)", float(np.mean(hist[-20:])), flush=True)
    yield net
    net.close()


def _timed(lt, h, p, o, reps=3):
    import torch
    lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, phi.cpu().numpy(), st


@pytest.mark.parametrize("name", ["C4_256", "C4_512"])
def test_network_gain_table(lt, trained, name):
    p = wl.make_problem(name)
    announce("gain", name)
    h = device_problem(lt, p)
    ref, _ = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, lt.make_opts(tol=1e-11))
    ref = ref.cpu().numpy()
    lt.lt_unet_attach(h, trained)
    rows = {}
    for label, pc, keep in (("gmg", lt.LT_PRECOND_GMG, 0.05), ("net_forced", lt.LT_PRECOND_UNET_GMG, 1.0),
                            ("net_adaptive", lt.LT_PRECOND_UNET_GMG, 0.05)):
        o = lt.make_opts(tol=1e-5, precision=lt.LT_PREC_MIXED, precond=pc, net_keep=keep)
        dt, phi, st = _timed(lt, h, p, o)
        err = rel_err_per_source(phi, ref).max()
        rows[label] = (dt, st["iters_max"], st["vcycles"], st["net_applied"], err)
        print(f"{name} {label:13s} {dt * 1e3:7.2f} ms  iters {st['iters_max']:3d}  vcycles {st['vcycles']:5d}  "
              f"net applied {st['net_applied']:4d}  err {err:.1e}", flush=True)
        assert err <= np.exp(0.171 * p.nz_contour) * 1e-5 * 2.0
    for label in ("net_forced", "net_adaptive"):
        assert rows[label][4] <= 2.0 * rows["gmg"][4] + 1e-6
    gain_v = rows["gmg"][2] - rows["net_forced"][2]
    print(f"{name}: V-cycles saved by the forced network {gain_v}, time ratio "
          f"{rows['net_forced'][0] / rows['gmg'][0]:.2f} (forced), {rows['net_adaptive'][0] / rows['gmg'][0]:.2f} "
          f"(adaptive)", flush=True)
    lt.lt_unet_attach(h, None)
    h.close()
