"""Host-side parts of the benchmark script (no GPU): the one-GPU refusal and the
merging of per-group statistics."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_group_statistics_merge():
    sys.path.insert(0, ROOT)
    import bench
    a = {"rc": 0, "iters_max": 21, "vcycles": 400, "true_relres_max": 3e-7, "net_applied": 1, "net_disabled_at": 1}
    b = {"rc": 1, "iters_max": 22, "vcycles": 482, "true_relres_max": 8e-7, "net_applied": 1, "net_disabled_at": 2}
    m = bench._merge_stats([a, b])
    assert m == {"rc": 1, "iters_max": 22, "vcycles": 882, "true_relres_max": 8e-7, "net_applied": 2,
                 "net_disabled_at": 2}
    assert bench._merge_stats([a]) is a


def test_water_table_and_tau_options():
    sys.path.insert(0, ROOT)
    import argparse
    import bench
    import workloads as wl
    p2 = wl.make_problem("C1")
    p3 = wl.make_problem("C3", n=(8, 6, 4))
    a = argparse.Namespace(water_table=1e-4, n_tau=3)
    q2, q3 = bench._with_boundary(p2, a), bench._with_boundary(p3, a)
    assert q2.bc == (0, 0, 0, 2, 0, 0) and q2.sy == 1e-4 and q2.n_tau == 3   # +y in 2D
    assert q3.bc == (0, 0, 0, 0, 0, 2) and q3.sy == 1e-4                      # +z in 3D
    assert bench._boundary_config(q3)["sy"] == 1e-4
    same = bench._with_boundary(p2, argparse.Namespace(water_table=None, n_tau=None))
    assert same is p2 and bench._boundary_config(same) == {}


def test_block_workload_cells_of_points():
    """The block benchmark's right-hand sides are unit vectors at the cells holding the wells and
    receivers: cell centres map to their own cell (x fastest), the far walls to the last cell."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    import workloads as wl
    p = wl.make_problem("C3", n=(8, 6, 4))
    idx = [(1, 2, 3), (7, 0, 0), (0, 5, 2)]
    pts = np.array([[(i + 0.5) * p.h[0], (j + 0.5) * p.h[1], (k + 0.5) * p.h[2]] for i, j, k in idx])
    assert list(bench._cells_of(p, pts)) == [i + 8 * (j + 6 * k) for i, j, k in idx]
    far = np.array([[8 * p.h[0], 6 * p.h[1], 4 * p.h[2]]])
    assert list(bench._cells_of(p, far)) == [8 * 6 * 4 - 1]
    # the 256x256 workload: its 8 wells sit at 8 of its 16 receivers, so the 24 columns hold 16
    # distinct cells; in the benchmark's order (wells, then receivers) every block of 4 or 8 holds
    # distinct cells, so no block starts rank deficient
    p2 = wl.make_problem("C2")
    w = np.vstack([p2.sources, p2.receivers])
    c = bench._cells_of(p2, w)
    assert len(set(c.tolist())) == 16 and c.max() < 256 * 256
    for blk in (4, 8):
        for b0 in range(0, len(c), blk):
            assert len(set(c[b0:b0 + blk].tolist())) == blk
