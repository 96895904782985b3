"""Train the learned preconditioner on the GPU.

Training pairs (r, e = (K + tau M)^{-1} r) come from the plain multigrid
solver on random 128x128 conductivity fields (seeds 10000+): the residuals
are of the two kinds the flexible Krylov method feeds its preconditioner --
point sources (its first basis vectors) and smooth fields (later basis
vectors, images of the mass matrix applied to preconditioned vectors) -- and
the targets are accurate preconditioner solves (lt_precond_solve).  The
shifts tau are contour nodes with non-negative real part, the candidates the
solver draws its preconditioner shifts from.  Every step runs in the
library's kernels; this module only draws random numbers and marshals.

    python -m paper_1409_2556_amd.train_unet --steps 400 --out weights.npy
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def random_tau(lt, rng, nz=20):
    import workloads as wl
    t = wl.T_D * np.exp(rng.uniform(np.log(0.01), np.log(10.0)))
    z, _ = lt.lt_talbot(nz, t)
    cand = z[z.real >= 0]
    return complex(cand[rng.integers(len(cand))])


def make_batch(lt, h, p, nvec, tau, rng):
    """nvec residuals on the problem's grid and their accurate corrections."""
    import torch
    N = p.N
    r = torch.zeros((nvec, 2, N), dtype=torch.float64, device="cuda")
    n_point = nvec // 3
    # point sources with random complex amplitude (the first Krylov vectors)
    for k in range(n_point):
        for _ in range(int(rng.integers(1, 4))):
            i = int(rng.integers(N))
            ph = np.exp(1j * rng.uniform(0, 2 * np.pi))
            r[k, 0, i] += ph.real
            r[k, 1, i] += ph.imag
    # smooth fields: mass matrix times V-cycle images of noise (later Krylov vectors)
    k2 = nvec - n_point
    if k2 > 0:
        noise = torch.randn((k2, 2, N), dtype=torch.float64, device="cuda",
                            generator=torch.Generator(device="cuda").manual_seed(int(rng.integers(1 << 31))))
        x = torch.empty_like(noise)
        lt.lt_vcycle(h, tau, lt.LT_PREC_FP64, 2, 2, noise, x, k2)
        m = torch.tensor(p.S * np.prod(p.h), dtype=torch.float64, device="cuda")
        r[n_point:] = x * m
    nrm = torch.linalg.vector_norm(r.reshape(nvec, -1), dim=1).clamp_min(1e-300)
    r = (r / nrm[:, None, None]).contiguous()
    e = torch.empty_like(r)
    lt.lt_precond_solve(h, tau, r, e, nvec, tol=1e-9, maxcycles=80)
    return r, e


def train(steps=400, batch=8, lr=1e-3, seed=0, n_fields=8, grid=128, log_every=25, net=None, verbose=True):
    """Train a network (new, or `net`) and return it with the loss history."""
    import torch
    import workloads as wl
    from paper_1409_2556_amd import binding as lt

    rng = np.random.default_rng(seed)
    if net is None:
        net = lt.UNet(seed=seed)
    fields = []
    for f in range(n_fields):
        p = wl.make_problem("C4_train", n=(grid, grid), seed=10000 + f)
        kap = torch.tensor(p.kappa, dtype=torch.float64, device="cuda")
        S = torch.tensor(p.S, dtype=torch.float64, device="cuda")
        fields.append((p, lt.lt_setup(p.ndim, p.n, p.h, kap, S)))
    hist = []
    t0 = time.time()
    for s in range(steps):
        p, h = fields[int(rng.integers(len(fields)))]
        tau = random_tau(lt, rng)
        r, e = make_batch(lt, h, p, batch, tau, rng)
        lr_s = lr * (0.5 * (1 + np.cos(np.pi * s / steps)))  # cosine decay
        loss = lt.lt_unet_train_step(net, h, tau, r, e, batch, lr_s)
        hist.append(loss)
        if verbose and (s % log_every == 0 or s == steps - 1):
            print(f"[train] step {s} loss {loss:.4f} ({time.time() - t0:.1f} s)", flush=True)
    for _, h in fields:
        h.close()
    return net, np.array(hist)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    net, hist = train(args.steps, args.batch, args.lr, args.seed)
    if args.out:
        np.save(args.out, net.get_params())
        print("saved", args.out, flush=True)


if __name__ == "__main__":
    main()
