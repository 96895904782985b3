"""Helpers shared by the GPU tests (marshalling and error measures only)."""
import numpy as np


def device_problem(lt, p, bc=None):
    import torch
    kap = torch.tensor(p.kappa, dtype=torch.float64, device="cuda")
    S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
    return lt.lt_setup(p.ndim, p.n, p.h, kap, S, bc=bc if bc is not None else p.bc, sy=p.sy)


def rel_err_per_source(got, ref):
    """||phi - phi_ref||_2 / ||phi_ref||_2 over receivers x times, per source."""
    d = np.linalg.norm((got - ref).reshape(got.shape[0], -1), axis=1)
    n = np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)
    return d / n


def max_err_per_source(got, ref):
    """max |phi - phi_ref| / max |phi_ref| over receivers x times, per source (element-wise)."""
    d = np.abs(got - ref).reshape(got.shape[0], -1).max(axis=1)
    n = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1)
    return d / n


# Entries of a source's heads at or above this fraction of its largest magnitude are also
# compared one by one, relative to their own size (below it, early-time heads at far
# receivers are set by the contour sum's absolute error, which the weighted test bounds
# relative to the largest head, not to each entry).
ENTRY_FLOOR = 1e-2


def entry_err(got, ref, floor=ENTRY_FLOOR):
    """max over entries with |phi_ref| >= floor * max |phi_ref| (per source) of |phi - phi_ref| / |phi_ref|."""
    worst = 0.0
    for s in range(ref.shape[0]):
        r = ref[s]
        sel = np.abs(r) >= floor * np.abs(r).max()
        if sel.any():
            worst = max(worst, float((np.abs(got[s][sel] - r[sel]) / np.abs(r[sel])).max()))
    return worst


def check_heads(got, ref, bar, label="", entry_bar=None):
    """Heads parity: per source, the 2-norm error and the element-wise max error (both relative to
    the reference's size) within `bar`; entries above ENTRY_FLOOR of a source's largest head within
    `entry_bar` (default 10 * bar) of their own size.  Returns the three measures."""
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.all(np.isfinite(got))
    e2 = float(rel_err_per_source(got, ref).max())
    emax = float(max_err_per_source(got, ref).max())
    een = entry_err(got, ref)
    eb = 10.0 * bar if entry_bar is None else entry_bar
    print(f"[heads] {label} norm {e2:.2e} max {emax:.2e} entries>={ENTRY_FLOOR:g} {een:.2e} "
          f"(bars {bar:g}, {eb:g})", flush=True)
    assert e2 <= bar, (label, "norm", e2)
    assert emax <= bar, (label, "max", emax)
    assert een <= eb, (label, "entries", een)
    return e2, emax, een


def announce(*a):
    print("[case]", *a, flush=True)


def device_problem_on_stream(lt, p):
    """Handle on a new stream of its own (default priority), for concurrent batches."""
    import torch
    kap = torch.tensor(p.kappa, dtype=torch.float64, device="cuda")
    S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    h = lt.lt_setup(p.ndim, p.n, p.h, kap, S, bc=p.bc, stream=s, sy=p.sy)
    h._torch_stream = s
    return h
