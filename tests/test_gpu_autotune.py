"""Smoother tile shapes (lt_set_tiles / lt_autotune).

Every tile shape performs the same per-cell red-black arithmetic, so a
V-cycle must be bit-identical whichever shape each level uses; the tuner
must return valid shapes, keep solves at the FP64 bar against the oracle,
and its cache must hand back what it measured."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.heads import heads
from gpu_util import device_problem, check_heads, announce

pytestmark = pytest.mark.gpu

GRIDS = [("C2", (256, 256), (0,) * 6, (2, 2)), ("C2", (96, 80), (0, 1, 0, 0, 1, 0), (2, 2)),
         ("C2", (100, 36), (0,) * 6, (1, 3)), ("C2", (136, 72), (0,) * 6, (3, 1))]


@pytest.mark.parametrize("name,n,bc,nus", GRIDS)
def test_every_tile_shape_gives_the_same_vcycle(lt, name, n, bc, nus):
    p = wl.make_problem(name, n=n)
    h = device_problem(lt, p, bc=bc)
    nl, _ = lt.lt_level_shape(h, 0)
    rng = np.random.default_rng(3)
    R = 3
    b = torch.tensor(rng.standard_normal((R, 2, p.N)), dtype=torch.float64, device="cuda")
    for prec in (lt.LT_PREC_FP64, lt.LT_PREC_MIXED):
        out = []
        for t in range(4):
            announce("tiles", n, nus, prec, t)
            lt.lt_set_tiles(h, prec, [t] * nl)
            x = torch.empty_like(b)
            lt.lt_vcycle(h, 3e5 + 2e5j, prec, nus[0], nus[1], b, x, R)
            torch.cuda.synchronize()
            out.append(x)
        # mixed shapes across levels
        lt.lt_set_tiles(h, prec, [(l * 3 + 1) % 4 for l in range(nl)])
        x = torch.empty_like(b)
        lt.lt_vcycle(h, 3e5 + 2e5j, prec, nus[0], nus[1], b, x, R)
        torch.cuda.synchronize()
        out.append(x)
        for x in out[1:]:
            assert torch.equal(x, out[0])
    h.close()


def test_autotune_then_solve_matches_oracle(lt, tmp_path):
    from paper_1409_2556_amd import autotune
    p = wl.make_problem("C2", n=(128, 96), nsrc=4, ntimes=3)
    h = device_problem(lt, p)
    announce("autotune")
    path = str(tmp_path / "tiles.json")
    tiles, us, hit = autotune.tune(h, lt.LT_PREC_MIXED, 2, 2, len(p.sources), path=path)
    print("tiles", tiles, [lt.lt_tile_shape(t) for t in tiles], "us", us, flush=True)
    assert not hit and len(tiles) >= 1 and all(0 <= t < 4 for t in tiles) and us > 0
    tiles2, us2, hit2 = autotune.tune(h, lt.LT_PREC_MIXED, 2, 2, len(p.sources), path=path)
    assert hit2 and tiles2 == tiles and us2 == us
    ref = heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times, p.nz_contour, q=p.q, workers=8)
    for prec, tol, bar in ((lt.LT_PREC_FP64, 1e-9, 1e-6), (lt.LT_PREC_MIXED, 1e-8, 1e-5)):
        lt.lt_autotune(h, prec, 2, 2, len(p.sources))
        o = lt.make_opts(tol=tol, precision=prec, n_tau=1)
        phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
        assert st["rc"] == 0
        check_heads(phi.cpu().numpy(), ref, bar, f"tuned prec {prec}")
    # 3D grids have no tile shapes
    q = wl.make_problem("C3", n=(16, 16, 8))
    h3 = device_problem(lt, q)
    assert lt.lt_autotune(h3, lt.LT_PREC_MIXED) == ([], 0.0)
    h3.close()
    h.close()
