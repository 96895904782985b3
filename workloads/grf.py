"""Stationary Gaussian random fields on a regular cell-centred grid.

The paper draws its rough log-transmissivity field from an exponential
covariance kernel (Section 4.1, the field with kernel theta*exp(-r)).  The
field here is ln(kappa) with mean zero and covariance
``C(dx) = var * exp(-|dx / ell|)`` (per-axis correlation lengths), sampled
exactly on the grid by circulant embedding: the covariance is wrapped onto
a periodic grid at least twice the domain, its FFT gives the eigenvalues
of the embedding, and one complex Gaussian draw gives two independent real
samples, of which the first is returned.
"""
from __future__ import annotations

import os

import numpy as np

# embeddings of at least this many points use the threaded FFT (same transform)
_BIG = 1 << 22


def _fftn(a):
    if a.size >= _BIG:
        import scipy.fft
        return scipy.fft.fftn(a, workers=min(16, os.cpu_count() or 1))
    return np.fft.fftn(a)


def _embedding_eigs(n, h, ell, var, pad):
    axes = []
    for na, ha, la in zip(n, h, ell):
        m = int(pad * na)
        k = np.arange(m)
        d = np.minimum(k, m - k) * ha  # wrapped distance on the torus
        axes.append(d / la)
    grids = np.meshgrid(*axes, indexing="ij")
    r = np.sqrt(sum(g * g for g in grids))
    c = var * np.exp(-r)
    lam = _fftn(c).real
    return lam


def gaussian_random_field(n, h, ell, var, seed, mean=0.0):
    """Return a field of shape ``n`` (axis order as given, e.g. (nx, ny)).

    ``n``, ``h``, ``ell`` are per-axis cell counts, spacings and correlation
    lengths.  The caller transposes to its storage order.
    """
    n = tuple(int(a) for a in n)
    h = tuple(float(a) for a in h)
    ell = tuple(float(a) for a in ell)
    pad = 2
    for _ in range(6):
        lam = _embedding_eigs(n, h, ell, var, pad)
        if lam.min() >= -1e-12 * lam.max():
            break
        pad *= 2
    lam = np.clip(lam, 0.0, None)
    rng = np.random.default_rng(seed)
    shape = lam.shape
    xi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    z = _fftn(np.sqrt(lam / lam.size) * xi)
    field = z.real[tuple(slice(0, a) for a in n)]
    return mean + field
