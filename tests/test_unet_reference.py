"""Pin of the float64 reference U-Net used by the GPU network tests: its
autograd gradient agrees with central differences of its own loss."""
import numpy as np
import torch

import unet_reference as ref


def _params(seed=0):
    rng = np.random.default_rng(seed)
    n = sum(9 * ci * co + co for ci, co in ref.LAYERS) + 34
    p = np.zeros(n)
    off = 0
    for ci, co in ref.LAYERS:
        p[off:off + 9 * ci * co] = rng.standard_normal(9 * ci * co) * np.sqrt(2.0 / (9 * ci))
        off += 9 * ci * co
        p[off:off + co] = 0.05 * rng.standard_normal(co)
        off += co
    p[off:] = rng.standard_normal(34) * 0.25
    return p


def test_reference_gradient_matches_central_differences():
    nx, ny, B = 16, 8, 2
    rng = np.random.default_rng(1)
    N = nx * ny
    r = rng.standard_normal((B, 2, N))
    e = rng.standard_normal((B, 2, N))
    D = np.exp(rng.standard_normal(N) * 0.3) * 4.0
    m = np.full(N, 1e-5 / 256)
    tau = 3e5 + 1e6j
    p = _params()
    L, g = ref.loss_and_grad(p, r, e, D, m, tau, nx, ny)
    assert np.isfinite(L)
    idx = np.random.default_rng(2).choice(p.size, 24, replace=False)
    for i in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (ref.loss_and_grad(pp, r, e, D, m, tau, nx, ny)[0] - ref.loss_and_grad(pm, r, e, D, m, tau, nx, ny)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g).max()), (i, fd, g[i])


def test_reference_layout_matches_conv_definition():
    # one 3x3 layer by hand: tap t = 3 ky + kx multiplies the input at (y + ky - 1, x + kx - 1)
    ci, co = 16, 16
    W = np.zeros((9, co, ci))
    W[5, 3, 2] = 1.0  # ky = 1, kx = 2: the right neighbour
    Wt = torch.as_tensor(W).reshape(9, co, ci).permute(1, 2, 0).reshape(co, ci, 3, 3)
    x = torch.zeros(1, ci, 4, 4, dtype=torch.float64)
    x[0, 2, 1, 2] = 7.0
    y = torch.nn.functional.conv2d(x, Wt, padding=1)
    assert float(y[0, 3, 1, 1]) == 7.0 and float(y.abs().sum()) == 7.0
