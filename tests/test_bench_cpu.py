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
