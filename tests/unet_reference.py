"""Plain PyTorch-CPU float64 reference of the library's U-Net preconditioner
(test infrastructure; shares no code with the HIP kernels).

Architecture and parameter layout follow the C ABI's description: 14 3x3
convolutions with ReLU (weights [9][cout][cin], tap = 3 * ky + kx, then the
bias), 2x2 average pooling, nearest upsampling with the skip concatenated
after the upsampled channels, and a linear 1x1 head 16 -> 2.  Features of a
residual r: r / s (re, im) with s = sqrt(sum |r|^2 / N), ln D - mean ln D,
tau m / D (re, im), zeros up to 16 channels.  Target: e D / s.  Loss: mean
over vectors of the error left after the best complex multiple of the output,
1 - |<out, target>|^2 / (||out||^2 ||target||^2)."""
import numpy as np
import torch
import torch.nn.functional as F

LAYERS = [(16, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 64), (64, 64),
          (128, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16)]


def unpack(p):
    p = torch.as_tensor(np.asarray(p, dtype=np.float64))
    out, off = [], 0
    for ci, co in LAYERS:
        n = 9 * ci * co
        W = p[off:off + n].reshape(9, co, ci).permute(1, 2, 0).reshape(co, ci, 3, 3)
        off += n
        b = p[off:off + co]
        off += co
        out.append((W, b))
    Wh = p[off:off + 32].reshape(2, 16)
    off += 32
    bh = p[off:off + 2]
    return out, Wh, bh


def forward_from_tensor(p, x):
    """x: [B, 16, H, W] float64 tensor; p: flat parameter tensor (may require grad)."""
    layers, off = [], 0
    for ci, co in LAYERS:
        n = 9 * ci * co
        W = p[off:off + n].reshape(9, co, ci).permute(1, 2, 0).reshape(co, ci, 3, 3)
        off += n
        layers.append((W, p[off:off + co]))
        off += co
    Wh = p[off:off + 32].reshape(2, 16)
    bh = p[off + 32:off + 34]

    def conv(t, l):
        return torch.relu(F.conv2d(t, layers[l][0], layers[l][1], padding=1))

    def up(t):
        return t.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3)

    e0 = conv(conv(x, 0), 1)
    e1 = conv(conv(F.avg_pool2d(e0, 2), 2), 3)
    e2 = conv(conv(F.avg_pool2d(e1, 2), 4), 5)
    e3 = conv(conv(F.avg_pool2d(e2, 2), 6), 7)
    d2 = conv(conv(torch.cat([up(e3), e2], 1), 8), 9)
    d1 = conv(conv(torch.cat([up(d2), e1], 1), 10), 11)
    d0 = conv(conv(torch.cat([up(d1), e0], 1), 12), 13)
    return torch.einsum("oc,bchw->bohw", Wh, d0) + bh[None, :, None, None]


def features(r, D, m, tau, nx, ny):
    """r: [B, 2, N] numpy; returns the input tensor [B, 16, ny, nx] and the scales s."""
    B, _, N = r.shape
    s = np.sqrt((r ** 2).sum(axis=(1, 2)) / N)
    x = np.zeros((B, 16, ny, nx))
    lnD = np.log(D)
    for b in range(B):
        x[b, 0] = (r[b, 0] / s[b]).reshape(ny, nx)
        x[b, 1] = (r[b, 1] / s[b]).reshape(ny, nx)
        x[b, 2] = (lnD - lnD.mean()).reshape(ny, nx)
        x[b, 3] = (tau.real * m / D).reshape(ny, nx)
        x[b, 4] = (tau.imag * m / D).reshape(ny, nx)
    return torch.as_tensor(x), s


def apply(p, r, D, m, tau, nx, ny):
    """e = network(r) as complex planes [B, 2, N] (numpy)."""
    x, s = features(r, D, m, tau, nx, ny)
    with torch.no_grad():
        o = forward_from_tensor(torch.as_tensor(np.asarray(p, dtype=np.float64)), x).numpy()
    B = r.shape[0]
    e = np.zeros_like(r)
    for b in range(B):
        e[b, 0] = o[b, 0].ravel() * s[b] / D
        e[b, 1] = o[b, 1].ravel() * s[b] / D
    return e


def loss_and_grad(p, r, e, D, m, tau, nx, ny):
    x, s = features(r, D, m, tau, nx, ny)
    pt = torch.as_tensor(np.asarray(p, dtype=np.float64)).clone().requires_grad_(True)
    o = forward_from_tensor(pt, x)
    B = r.shape[0]
    t = torch.as_tensor(np.stack([(e[:, 0] * D / s[:, None]).reshape(B, ny, nx),
                                  (e[:, 1] * D / s[:, None]).reshape(B, ny, nx)], axis=1))
    a, b, x, y = o[:, 0], o[:, 1], t[:, 0], t[:, 1]
    P = (a * x + b * y).sum(dim=(1, 2))
    Q = (a * y - b * x).sum(dim=(1, 2))
    oo = (a * a + b * b).sum(dim=(1, 2))
    tt = (x * x + y * y).sum(dim=(1, 2))
    loss = (1.0 - (P * P + Q * Q) / (oo * tt)).mean()
    loss.backward()
    return float(loss), pt.grad.numpy()
