"""The GPU V-cycle (fused 2D tiles, generic 3D kernels, single-workgroup
coarse levels) equals a plain numpy V-cycle of the same definition."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import device_problem, announce
import mg_reference as ref

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n,bc,nus", [
    ("C2", (256, 256), (0,) * 6, (2, 2)),
    ("C2", (96, 80), (0, 1, 0, 0, 1, 0), (2, 2)),
    ("C2", (100, 36), (0,) * 6, (1, 3)),
    ("C1", (32, 32), (0,) * 6, (2, 2)),
    ("C3", (32, 32, 16), (0,) * 6, (2, 2)),
    ("C3", (12, 20, 10), (1, 0, 0, 0, 0, 1), (2, 1)),
    ("C3", (16, 12, 8), (0,) * 6, (2, 0)),
    ("C3", (16, 12, 8), (0, 0, 1, 0, 0, 0), (0, 3)),
    ("C3", (20, 20, 12), (0,) * 6, (1, 1)),
])
def test_vcycle_matches_reference(lt, name, n, bc, nus):
    import torch
    p = wl.make_problem(name, n=n)
    announce("vcycle-ref", n, bc, nus)
    h = device_problem(lt, p, bc=bc)
    L0 = ref.fine_level(p.n, p.h, p.kappa, p.S, bc=bc, ndim=p.ndim)
    levels, cos = ref.hierarchy(L0)
    nl, _ = lt.lt_level_shape(h, 0)
    assert nl == len(levels)
    for l, Lr in enumerate(levels):
        assert lt.lt_level_shape(h, l)[1] == Lr.n
    rng = np.random.default_rng(7)
    R = 2
    bz = rng.standard_normal((R, p.N)) + 1j * rng.standard_normal((R, p.N))
    b = torch.tensor(np.stack([bz.real, bz.imag], axis=1), dtype=torch.float64, device="cuda").contiguous()
    x = torch.empty_like(b)
    shape = (p.n[2], p.n[1], p.n[0])
    for tau in (2e5 + 6e5j, 3e7 + 1e7j):
        want = np.stack([ref.vcycle(levels, cos, bz[r].reshape(shape), tau, nus[0], nus[1], bc).ravel()
                         for r in range(R)])
        for prec, tol in ((0, 1e-11), (1, 2e-5)):
            lt.lt_vcycle(h, tau, prec, nus[0], nus[1], b, x, R)
            torch.cuda.synchronize()
            got = x.cpu().numpy()
            got = got[:, 0] + 1j * got[:, 1]
            err = np.abs(got - want).max() / np.abs(want).max()
            assert err <= tol, (tau, prec, err)
    h.close()
