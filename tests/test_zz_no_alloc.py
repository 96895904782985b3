"""The allocation-free V-cycle (lt_vcycle_noalloc) against lt_vcycle, through the C ABI:
two calls in a row on one handle, the second with fewer right-hand sides, in both
precisions, and a call that needs more scratch than the library holds is refused before
any work."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import device_problem, announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n", [("C2", (96, 80)), ("C3", (24, 20, 16)), ("C3", (32, 32, 16))])
def test_noalloc_vcycle_equals_vcycle(lt, name, n):
    import torch
    p = wl.make_problem(name, n=n)
    h = device_problem(lt, p)
    rng = np.random.default_rng(11)
    for call, (R, tau) in enumerate(((3, 4e5 + 9e5j), (2, 2e7 + 3e6j))):
        bz = rng.standard_normal((R, p.N)) + 1j * rng.standard_normal((R, p.N))
        b = torch.tensor(np.stack([bz.real, bz.imag], axis=1), dtype=torch.float64, device="cuda").contiguous()
        for prec, bar in ((lt.LT_PREC_FP64, 1e-12), (lt.LT_PREC_MIXED, 1e-5)):
            announce("noalloc vcycle", name, n, "call", call, "R", R, "prec", prec)
            want = torch.empty_like(b)
            got = torch.full_like(b, float("nan"))
            lt.lt_vcycle(h, tau, prec, 2, 2, b, want, R)
            lt.lt_vcycle_noalloc(h, tau, prec, 2, 2, b, got, R)
            torch.cuda.synchronize()
            err = float((got - want).abs().max() / want.abs().max())
            print(name, n, "call", call, "prec", prec, "max rel diff", err, flush=True)
            assert torch.isfinite(got).all()
            assert err <= bar
    h.close()


def test_noalloc_refuses_oversize(lt):
    import torch
    p = wl.make_problem("C2", n=(512, 512))
    h = device_problem(lt, p)
    R = 64  # 64 right-hand sides of 512 x 512 need far more than the scratch
    b = torch.zeros((R, 2, p.N), dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 7.0)
    with pytest.raises(lt.LTError):
        lt.lt_vcycle_noalloc(h, 1e6, lt.LT_PREC_FP64, 2, 2, b, x, R)
    assert "scratch" in lt.lt_last_error()
    torch.cuda.synchronize()
    assert bool((x == 7.0).all())  # nothing ran
    h.close()
