"""The synthetic workloads: grids, fields, wells, times.

Units are nondimensional: the domain is the unit square (cube), the
geometric-mean conductivity is 1 and storage is 1e-5, so the diffusion time
``T_D = S L^2 / kappa = 1e-5``.  Measurement times are given in units of
``T_D`` and multiplied by it here, which puts them in the paper's own regime
(its 1, 5 and 20 minute samples are 0.06, 0.3 and 1.2 diffusion times of its
100 m aquifer, Section 4.1).  ``literal_times=True`` keeps the numbers as
given instead; every head then equals its steady state.

Arrays are stored with x fastest: cell (ix, iy, iz) sits at
``ix + nx * (iy + ny * iz)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from .grf import gaussian_random_field

T_D = 1e-5  # S_g L^2 / kappa_g for the unit domain


@dataclass
class Problem:
    name: str
    ndim: int
    n: tuple            # cells per axis (nx, ny, nz); nz = 1 in 2D
    h: tuple            # spacing per axis
    kappa: np.ndarray   # [N] float64, x fastest
    S: np.ndarray       # [N] float64 storage coefficient
    sources: np.ndarray     # [ns, 3] coordinates of the pumping wells
    receivers: np.ndarray   # [nr, 3] coordinates of the observation wells
    times: np.ndarray       # [nt] physical times
    nz_contour: int         # full-contour Talbot nodes per time
    q: float = 1.0          # constant pumping rate from t = 0
    bc: tuple = (0, 0, 0, 0, 0, 0)   # 0 = zero Dirichlet, 1 = zero Neumann, 2 = water table; faces -x,+x,-y,+y,-z,+z
    sy: float = 0.0                  # specific yield of the water-table faces
    n_tau: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return int(np.prod(self.n))


def _log_times(lo, hi, k):
    return np.exp(np.linspace(np.log(lo), np.log(hi), k))


def _wells_2d(vals):
    v = np.asarray(vals, dtype=float)
    return np.array([(x, y, 0.0) for y in v for x in v])


def _field(n, h, ell, var, seed):
    nd = len(n)
    f = gaussian_random_field(n, h, ell[:nd], var, seed)
    return np.exp(f).flatten(order="F")


def make_problem(name: str, n: Optional[tuple] = None, seed: Optional[int] = None,
                 literal_times: bool = False, nsrc: Optional[int] = None,
                 nrec: Optional[int] = None, ntimes: Optional[int] = None,
                 var: Optional[float] = None) -> Problem:
    """Build one of the named workloads, optionally reduced in size.

    ``n`` replaces the grid (the unit domain is kept, so the spacing
    follows), ``seed`` the field seed, ``nsrc``/``nrec``/``ntimes`` keep the
    first few sources, receivers or times, ``var`` replaces the variance of
    ln kappa.
    """
    spec = dict(CONFIGS[name])
    nn = tuple(n) if n is not None else spec["n"]
    ndim = len(nn)
    ext = spec.get("extent", (1.0,) * ndim)
    h = tuple(e / a for e, a in zip(ext, nn))
    s = spec["seed"] if seed is None else seed
    kappa = _field(nn, h, spec["ell"], spec["var"] if var is None else float(var), s)
    N = int(np.prod(nn))
    if spec.get("S_loguniform"):
        lo, hi = spec["S_loguniform"]
        rng = np.random.default_rng(spec["S_seed"] if seed is None else seed + 1)
        S = np.exp(rng.uniform(np.log(lo), np.log(hi), size=N))
    else:
        S = np.full(N, spec["S"])
    times = np.asarray(spec["times"], dtype=float)
    if not literal_times:
        times = times * T_D
    src = np.asarray(spec["sources"], dtype=float)
    rec = np.asarray(spec["receivers"], dtype=float)
    if nsrc is not None:
        src = src[:nsrc]
    if nrec is not None:
        rec = rec[:nrec]
    if ntimes is not None:
        times = times[:ntimes]
    n3 = tuple(nn) + (1,) * (3 - ndim)
    h3 = tuple(h) + (1.0,) * (3 - ndim)
    return Problem(name=name, ndim=ndim, n=n3, h=h3, kappa=kappa, S=S,
                   sources=src, receivers=rec, times=times,
                   nz_contour=spec["nz"], n_tau=spec.get("n_tau", 1),
                   meta={"seed": s, "literal_times": literal_times})


_C2_WELLS = _wells_2d([0.2, 0.4, 0.6, 0.8])
_C2_SOURCES = np.array([w for i, w in enumerate(_C2_WELLS)
                        if ((i % 4) + (i // 4)) % 2 == 0])

_C3_SOURCES = np.array([(x, y, 0.5) for y in np.linspace(0.2, 0.8, 5)
                        for x in np.linspace(0.2, 0.8, 5)])
_C3_RECEIVERS = np.array([(x, y, z) for z in (0.25, 0.5, 0.75)
                          for y in (0.2, 0.4, 0.6, 0.8) for x in (0.2, 0.4, 0.6, 0.8)])

_C5_SOURCES_2D = _wells_2d([0.2, 0.4, 0.6, 0.8])
_C5_RECEIVERS_2D = np.array([(x, y, 0.0) for y in (0.2, 0.4, 0.6, 0.8)
                             for x in (0.1, 0.2, 0.3, 0.4, 0.6, 0.7, 0.8, 0.9)])
_C5_SOURCES_3D = np.array([(x, y, 0.5) for y in (0.2, 0.4, 0.6, 0.8) for x in (0.2, 0.4, 0.6, 0.8)])
_C5_RECEIVERS_3D = np.array([(x, y, z) for z in (0.25, 0.75)
                             for y in (0.3, 0.5, 0.7, 0.9) for x in (0.3, 0.5, 0.7, 0.9)])

_THT_WELLS = _wells_2d(np.linspace(0.2, 0.8, 6))

CONFIGS = {
    # 2D 32x32, one central source, four receivers, 5 times, 16-node contour
    "C1": dict(n=(32, 32), var=1.0, ell=(0.2, 0.2, 0.2), seed=101, S=1e-5,
               sources=[(0.5, 0.5, 0.0)],
               receivers=[(0.3, 0.3, 0.0), (0.7, 0.3, 0.0), (0.3, 0.7, 0.0), (0.7, 0.7, 0.0)],
               times=_log_times(1e-2, 10.0, 5), nz=16, n_tau=1),
    # 2D 256x256, 8 sources and 16 receivers on a 4x4 well pattern, 10 times, 20 nodes
    "C2": dict(n=(256, 256), var=1.0, ell=(0.1, 0.1, 0.1), seed=201, S=1e-5,
               sources=_C2_SOURCES, receivers=_C2_WELLS,
               times=_log_times(1e-2, 10.0, 10), nz=20, n_tau=1),
    # 3D 64x64x32 on the unit cube, anisotropic field, log-uniform storage
    "C3": dict(n=(64, 64, 32), var=2.0, ell=(0.2, 0.2, 0.05), seed=301,
               S_loguniform=(1e-6, 1e-4), S_seed=302,
               sources=_C3_SOURCES, receivers=_C3_RECEIVERS,
               times=[0.3, 1.2], nz=24, n_tau=3),
    # the single-well test of Section 4.1: one well pumping at the centre, observed at (0.7, 0.7)
    # (the paper's (50, 50) and (70, 70) m in its 100 m square), ln kappa variance 1.6, the
    # 5 minute sample (0.3 diffusion times), 40-node contour, 128x128 cells
    "W1": dict(n=(128, 128), var=1.6, ell=(0.2, 0.2, 0.2), seed=401, S=1e-5,
               sources=[(0.5, 0.5, 0.0)],
               receivers=[(0.7, 0.7, 0.0), (0.3, 0.7, 0.0), (0.7, 0.3, 0.0), (0.3, 0.3, 0.0)],
               times=[0.3], nz=40, n_tau=1),
    # learned-preconditioner evaluation fields (training fields use seeds 10000+)
    "C4_256": dict(n=(256, 256), var=1.0, ell=(0.1, 0.1, 0.1), seed=20000, S=1e-5,
                   sources=_C2_SOURCES, receivers=_C2_WELLS, times=[0.3], nz=40, n_tau=1),
    "C4_512": dict(n=(512, 512), var=1.0, ell=(0.1, 0.1, 0.1), seed=20001, S=1e-5,
                   sources=_C2_SOURCES, receivers=_C2_WELLS, times=[0.3], nz=40, n_tau=1),
    # a batch of six problems on uneven grids (2D as the 256x256 workload, 3D as
    # the 64x64x32 one): 16 sources and 32 receivers each, times {0.3, 1.2}, 24 nodes
    "C5_128": dict(n=(128, 128), var=1.0, ell=(0.1, 0.1, 0.1), seed=501, S=1e-5,
                   sources=_C5_SOURCES_2D, receivers=_C5_RECEIVERS_2D, times=[0.3, 1.2], nz=24, n_tau=1),
    "C5_256": dict(n=(256, 256), var=1.0, ell=(0.1, 0.1, 0.1), seed=502, S=1e-5,
                   sources=_C5_SOURCES_2D, receivers=_C5_RECEIVERS_2D, times=[0.3, 1.2], nz=24, n_tau=1),
    "C5_512": dict(n=(512, 512), var=1.0, ell=(0.1, 0.1, 0.1), seed=503, S=1e-5,
                   sources=_C5_SOURCES_2D, receivers=_C5_RECEIVERS_2D, times=[0.3, 1.2], nz=24, n_tau=1),
    "C5_32c": dict(n=(32, 32, 32), var=2.0, ell=(0.2, 0.2, 0.05), seed=504,
                   S_loguniform=(1e-6, 1e-4), S_seed=514,
                   sources=_C5_SOURCES_3D, receivers=_C5_RECEIVERS_3D, times=[0.3, 1.2], nz=24, n_tau=3),
    "C5_64c": dict(n=(64, 64, 64), var=2.0, ell=(0.2, 0.2, 0.05), seed=505,
                   S_loguniform=(1e-6, 1e-4), S_seed=515,
                   sources=_C5_SOURCES_3D, receivers=_C5_RECEIVERS_3D, times=[0.3, 1.2], nz=24, n_tau=3),
    "C5_128x64": dict(n=(128, 128, 64), var=2.0, ell=(0.2, 0.2, 0.05), seed=506,
                      S_loguniform=(1e-6, 1e-4), S_seed=516,
                      sources=_C5_SOURCES_3D, receivers=_C5_RECEIVERS_3D, times=[0.3, 1.2], nz=24, n_tau=3),
    # transient hydraulic tomography (Section 5.3): one well pumping at the centre, 36
    # observation wells evenly in [0.2, 0.8]^2, the 8, 10 and 20 minute samples (0.48, 0.6 and
    # 1.2 diffusion times), 20-node contour, 100x100 cells (the paper: 101^2 grid points)
    "THT": dict(n=(100, 100), var=1.0, ell=(0.2, 0.2, 0.2), seed=601, S=1e-5,
                sources=[(0.5, 0.5, 0.0)], receivers=_THT_WELLS, times=[0.48, 0.6, 1.2], nz=20, n_tau=2),
    "C4_train": dict(n=(128, 128), var=1.0, ell=(0.1, 0.1, 0.1), seed=10000, S=1e-5,
                     sources=_C2_SOURCES, receivers=_C2_WELLS, times=[0.3], nz=40, n_tau=1),
}


C5_BATCH = ("C5_128", "C5_256", "C5_512", "C5_32c", "C5_64c", "C5_128x64")


def make_batch(names=C5_BATCH, **kw):
    """The problems of a batch workload (by default the six uneven grids)."""
    return [make_problem(nm, **kw) for nm in names]
