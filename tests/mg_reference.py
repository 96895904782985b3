"""Plain numpy V-cycle with the same definition as the library's multigrid
(test infrastructure; used to pin the GPU V-cycle to rounding).

Levels aggregate 2 cells per halved axis (axes within 1.5x of the finest
spacing, even length > 2, while the level has more than 64 cells).  Coarse
faces: sum of the fine faces on the aggregate interface times h/H; walls the
same; mass summed.  Pre-smoothing: nu1 red-black sweeps (red = even
x+y+z first) from x = 0; residual summed over each aggregate; coarsest level
solved exactly; prolongation: cell-centred linear interpolation per halved
axis with the ghost mirrored through the wall (odd for Dirichlet, even for
Neumann); post-smoothing: nu2 sweeps, black first.
"""
import numpy as np


class Level:
    pass


def fine_level(n, h, kappa, S, bc=(0,) * 6, ndim=2):
    nx, ny, nz = n
    kap = np.asarray(kappa, dtype=np.float64).reshape(nz, ny, nx)
    V = h[0] * h[1] * h[2]
    L = Level()
    L.n, L.h, L.nd = tuple(n), tuple(h), ndim
    L.T, L.W = [], []
    for a in range(3):
        ax = 2 - a
        T = np.zeros((nz, ny, nx))
        W = np.zeros((nz, ny, nx))
        if a < ndim:
            area = V / h[a]
            if n[a] > 1:
                lo = [slice(None)] * 3
                hi = [slice(None)] * 3
                lo[ax] = slice(0, n[a] - 1)
                hi[ax] = slice(1, n[a])
                ki, kj = kap[tuple(lo)], kap[tuple(hi)]
                T[tuple(lo)] = 2 * ki * kj / (ki + kj) * area / h[a]
            for side, face in ((0, 2 * a), (n[a] - 1, 2 * a + 1)):
                if bc[face] == 0:
                    sl = [slice(None)] * 3
                    sl[ax] = slice(side, side + 1)
                    W[tuple(sl)] += 2 * kap[tuple(sl)] * area / h[a]
        L.T.append(T)
        L.W.append(W)
    L.m = (np.asarray(S, dtype=np.float64) * V).reshape(nz, ny, nx)
    _finish(L)
    return L


def _finish(L):
    D = np.zeros(L.m.shape)
    for a in range(3):
        ax = 2 - a
        Tm = np.zeros_like(L.T[a])
        sl_dst = [slice(None)] * 3
        sl_src = [slice(None)] * 3
        sl_dst[ax] = slice(1, None)
        sl_src[ax] = slice(0, -1)
        Tm[tuple(sl_dst)] = L.T[a][tuple(sl_src)]
        D += L.W[a] + L.T[a] + Tm
    L.D = D
    L.color = np.indices(L.m.shape).sum(axis=0) % 2


def _agg(x, co):
    nz, ny, nx = x.shape
    return x.reshape(nz // (2 if co[2] else 1), 2 if co[2] else 1, ny // (2 if co[1] else 1),
                     2 if co[1] else 1, nx // (2 if co[0] else 1), 2 if co[0] else 1)


def coarsen(L):
    hmin = min(L.h[a] for a in range(L.nd))
    co = [a < L.nd and L.n[a] % 2 == 0 and L.n[a] > 2 and L.h[a] < 1.5 * hmin for a in range(3)]
    if not any(co):
        return None, co
    C = Level()
    C.nd = L.nd
    C.n = tuple(L.n[a] // 2 if co[a] else L.n[a] for a in range(3))
    C.h = tuple(L.h[a] * 2 if co[a] else L.h[a] for a in range(3))
    C.m = _agg(L.m, co).sum(axis=(1, 3, 5))
    C.T, C.W = [], []
    for a in range(3):
        f = 0.5 if co[a] else 1.0
        C.W.append(f * _agg(L.W[a], co).sum(axis=(1, 3, 5)))
        s = _agg(L.T[a], co)
        pos = {0: 5, 1: 3, 2: 1}[a]
        idx = [slice(None)] * 6
        idx[pos] = -1  # the child on the +a side of the aggregate
        sub = s[tuple(idx)]
        other = tuple(q - (1 if q > pos else 0) for q in (1, 3, 5) if q != pos)
        C.T.append(f * sub.sum(axis=other))
    _finish(C)
    return C, co


def hierarchy(L0, maxc=64):
    levels, cos = [L0], []
    while levels[-1].m.size > maxc:
        C, co = coarsen(levels[-1])
        if C is None:
            break
        levels.append(C)
        cos.append(co)
    return levels, cos


def _shift(x, ax, d):
    """y[i] = x[i + d] along axis ax with zero fill."""
    y = np.zeros_like(x)
    n = x.shape[ax]
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if d > 0:
        src[ax] = slice(d, n)
        dst[ax] = slice(0, n - d)
    else:
        src[ax] = slice(0, n + d)
        dst[ax] = slice(-d, n)
    y[tuple(dst)] = x[tuple(src)]
    return y


def offsum(L, x):
    y = np.zeros_like(x)
    for a in range(3):
        ax = 2 - a
        if L.n[a] == 1:
            continue
        T = L.T[a]
        y += T * _shift(x, ax, 1) + _shift(T, ax, -1) * _shift(x, ax, -1)
    return y


def apply(L, x, tau):
    return (L.D + tau * L.m) * x - offsum(L, x)


def gs(L, x, b, tau, color):
    d = L.D + tau * L.m
    msk = L.color == color
    return np.where(msk, (b + offsum(L, x)) / d, x)


def prolong(Lf, C, co, e, bc):
    out = e
    for a in range(3):
        if not co[a]:
            continue
        ax = 2 - a
        n = out.shape[ax]
        glo = 1.0 if bc[2 * a] == 1 else -1.0
        ghi = 1.0 if bc[2 * a + 1] == 1 else -1.0
        lo = _shift(out, ax, -1)
        hi = _shift(out, ax, 1)
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[ax] = slice(0, 1)
        last[ax] = slice(n - 1, n)
        lo[tuple(first)] = glo * out[tuple(first)]
        hi[tuple(last)] = ghi * out[tuple(last)]
        even = 0.75 * out + 0.25 * lo
        odd = 0.75 * out + 0.25 * hi
        out = np.stack([even, odd], axis=ax + 1)
        shape = list(out.shape[:ax]) + [2 * n] + list(out.shape[ax + 2:])
        out = out.reshape(shape)
    return out


def vcycle(levels, cos, b, tau, nu1=2, nu2=2, bc=(0,) * 6, l=0):
    L = levels[l]
    if l == len(levels) - 1:
        n = L.m.size
        A = np.zeros((n, n), complex)
        for i in range(n):
            e = np.zeros(n, complex)
            e[i] = 1
            A[:, i] = apply(L, e.reshape(L.m.shape), tau).ravel()
        return np.linalg.solve(A, b.ravel()).reshape(L.m.shape)
    x = np.zeros_like(b)
    for _ in range(nu1):
        x = gs(L, x, b, tau, 0)
        x = gs(L, x, b, tau, 1)
    r = b - apply(L, x, tau)
    co = cos[l]
    rc = _agg(r, co).sum(axis=(1, 3, 5))
    ec = vcycle(levels, cos, rc, tau, nu1, nu2, bc, l + 1)
    x = x + prolong(L, levels[l + 1], co, ec, bc)
    for _ in range(nu2):
        x = gs(L, x, b, tau, 1)
        x = gs(L, x, b, tau, 0)
    return x
