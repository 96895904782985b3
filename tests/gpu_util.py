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
