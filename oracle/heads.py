"""Heads at receivers by one sparse direct solve per contour shift.

Oracle (test infrastructure only).

The method of Section 3 approximates, to solver tolerance, the contour sum
(eqn:half) of the Laplace-domain solution F(z) = (K + z M)^{-1} (qhat(z) b +
M phi0) (Section 2.1, the transformed semi-discrete system).  This module
computes that sum directly: for every distinct shift z_k it factorises
K + z_k M once with SuperLU, solves all right-hand sides, and forms

    phi(x_r, t) = 2 Re sum_{k <= N_z/2} w_k(t) B_r (K + z_k M)^{-1} (qhat(z_k) b_s + M phi0),

with qhat(z) = q / z for a constant rate switched on at t = 0.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from .fv import assemble, point_weights
from .contour import talbot_nodes

_G = {}


def _factor_solve(z, rhs):
    K, m = _G["K"], _G["m"]
    A = (K + sp.diags(z * m)).astype(np.complex128).tocsc()
    lu = splu(A, permc_spec="MMD_AT_PLUS_A")
    return lu.solve(np.asarray(rhs, dtype=np.complex128))


def _job(args):
    z, take = args
    X = _factor_solve(z, _G["rhs"])
    if take == "gather":
        return _G["Br"] @ X
    return X


def _init_worker(K, m, rhs, Br):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    _G.update(K=K, m=m, rhs=rhs, Br=Br)


def _map_shifts(K, m, rhs, shifts, take, Br=None, workers=1):
    _G.update(K=K, m=m, rhs=rhs, Br=Br)
    jobs = [(z, take) for z in shifts]
    if workers <= 1 or len(jobs) <= 1:
        return [_job(j) for j in jobs]
    # fresh interpreters (spawn): safe even when the parent has initialised a GPU runtime
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(max_workers=min(workers, len(jobs)), mp_context=ctx,
                             initializer=_init_worker, initargs=(K, m, rhs, Br)) as ex:
        return list(ex.map(_job, jobs))


def shifted_fields(K, m, rhs, shifts, workers=1):
    """Solutions (K + z M)^{-1} rhs for each shift z (list of [N, nrhs])."""
    return _map_shifts(K, m, rhs, list(shifts), "full", workers=workers)


def heads(n, h, kappa, S, sources, receivers, times, nz, q=1.0, bc=(0,) * 6,
          phi0=None, workers=1, ndim=None, sy=0.0):
    """Heads phi[source, receiver, time] (float64).

    ``q`` is one pumping rate for every source or one per source (qhat = q_s / z).
    With ``phi0`` (an [N] initial head) the term M phi0 is added to every
    source's right-hand side with factor 1 (Section 3, the two-system split);
    ``q = 0`` leaves only the initial-value problem, and with no sources at all
    the result has one row holding it.  ``sy`` is the specific yield of the
    faces that ``bc`` marks as water table.
    """
    K, m = assemble(n, h, kappa, S, bc, ndim=ndim, sy=sy)
    N = K.shape[0]
    src = np.asarray(sources, dtype=np.float64).reshape(-1, 3)
    Br = point_weights(n, h, receivers)
    ns, nr, nt = src.shape[0], Br.shape[0], len(times)
    if ns == 0 and phi0 is None:
        raise ValueError("no sources and no initial head")
    qs = np.broadcast_to(np.asarray(q, dtype=np.float64), (ns,))
    # columns: the sources' b, then (optionally) M phi0
    cols = [point_weights(n, h, src).T.toarray() if ns > 0 else np.zeros((N, 0))]
    if phi0 is not None:
        cols.append((m * np.asarray(phi0, dtype=np.float64)).reshape(N, 1))
    rhs = np.hstack(cols)
    nodes = [talbot_nodes(nz, t) for t in times]
    shifts = np.concatenate([z for z, _ in nodes])
    gathered = _map_shifts(K, m, rhs, shifts, "gather", Br=Br, workers=workers)
    rows = max(ns, 1)
    phi = np.zeros((rows, nr, nt))
    kk = 0
    for it, (z, w) in enumerate(nodes):
        acc = np.zeros((nr, rows), dtype=np.complex128)
        for k in range(len(z)):
            G = gathered[kk]
            kk += 1
            term = np.zeros((nr, rows), dtype=np.complex128)
            if ns > 0:
                term += (qs / z[k]) * G[:, :ns]
            if phi0 is not None:
                term = term + G[:, ns:ns + 1]
            acc += w[k] * term
        phi[:, :, it] = 2.0 * acc.real.T
    return phi


def heads_problem(p, workers=1, phi0=None):
    """heads() for a workloads.Problem."""
    return heads(p.n, p.h, p.kappa, p.S, p.sources, p.receivers, p.times,
                 p.nz_contour, q=p.q, bc=p.bc, phi0=phi0, workers=workers, ndim=p.ndim,
                 sy=p.sy)


def default_workers():
    return max(1, os.cpu_count() or 1)
