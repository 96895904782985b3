"""Thin ctypes binding of the C ABI declared in include/lt.h.

Argument marshalling only: device arrays are torch tensors on the GPU (their
data pointers are passed through), host arrays are numpy arrays, and every
step of the computation runs inside the HIP library.  Importing this module
loads the built library and fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} is missing (run paper_1409_2556_amd/build.py)")
_lib = C.CDLL(LIB_PATH)

LT_OK, LT_EINVAL, LT_EHIP, LT_ENOMEM, LT_EUNSUPPORTED, LT_WNOTCONV = 0, -1, -2, -3, -4, 1
LT_BC_DIRICHLET0, LT_BC_NEUMANN0, LT_BC_WATER_TABLE = 0, 1, 2
LT_PREC_FP64, LT_PREC_MIXED = 0, 1
LT_PROF_OFF, LT_PROF_PRE_FINE, LT_PROF_POST_FINE, LT_PROF_SWEEP3D, LT_PROF_EXACT = 0, 1, 2, 3, 4
LT_PRECOND_GMG, LT_PRECOND_UNET_GMG, LT_PRECOND_EXACT = 0, 1, 2
LT_METHOD_GMRES, LT_METHOD_FOM = 0, 1
LT_CONV_WEIGHTED, LT_CONV_RELATIVE = 0, 1


class lt_grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double * 3)]


class lt_bc(C.Structure):
    _fields_ = [("face", C.c_int * 6), ("sy", C.c_double)]


class lt_points(C.Structure):
    _fields_ = [("n", C.c_int), ("xyz", C.POINTER(C.c_double))]


class lt_sources(C.Structure):
    _fields_ = [("pts", lt_points), ("q", C.POINTER(C.c_double)), ("phi0", C.c_void_p)]


class lt_contour(C.Structure):
    _fields_ = [("nz", C.c_int)]


class lt_geostat(C.Structure):
    _fields_ = [("src", lt_points), ("q", C.POINTER(C.c_double)), ("obs", lt_points),
                ("times", C.POINTER(C.c_double)), ("ntimes", C.c_int), ("contour", lt_contour),
                ("cov_var", C.c_double), ("cov_len", C.c_double * 3), ("r", C.c_double),
                ("opts", C.c_void_p)]


class lt_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("precision", C.c_int), ("n_tau", C.c_int),
                ("tau_reim", C.POINTER(C.c_double)), ("nu1", C.c_int), ("nu2", C.c_int),
                ("inner_max", C.c_int), ("relax", C.c_double), ("true_residual", C.c_int),
                ("profile", C.c_int), ("precond", C.c_int), ("net_keep", C.c_double),
                ("graph", C.c_int), ("method", C.c_int), ("conv", C.c_int), ("tau_adapt", C.c_int),
                ("restart", C.c_int)]


class lt_stats(C.Structure):
    _fields_ = [("n_rhs", C.c_int), ("n_shifts", C.c_int), ("iters_max", C.c_int), ("vcycles", C.c_int),
                ("levels", C.c_int), ("true_relres_max", C.c_double), ("seconds", C.c_double),
                ("iters_per_rhs", C.POINTER(C.c_int)), ("true_relres", C.POINTER(C.c_double)),
                ("net_applied", C.c_int), ("net_rejected", C.c_int), ("net_disabled_at", C.c_int),
                ("prof_launches", C.c_int), ("prof_ms", C.c_double), ("prof_bytes", C.c_double),
                ("resolves", C.c_int), ("factorizations", C.c_int), ("factor_ms", C.c_double)]


_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_h = C.c_void_p


class lt_solve_item(C.Structure):
    _fields_ = [("h", _h), ("src", C.POINTER(lt_sources)), ("times", _dp),
                ("ntimes", C.c_int), ("contour", C.POINTER(lt_contour)), ("receivers", C.POINTER(lt_points)),
                ("opts", C.POINTER(lt_opts)), ("phi_out", _vp), ("stats", C.POINTER(lt_stats)),
                ("status", C.c_int)]


class lt_adjoint_item(C.Structure):
    _fields_ = [("h", _h), ("src", C.POINTER(lt_sources)),
                ("receivers", C.POINTER(lt_points)), ("times", _dp), ("ntimes", C.c_int),
                ("contour", C.POINTER(lt_contour)), ("opts", C.POINTER(lt_opts)), ("dlnK", _vp), ("dlnS", _vp),
                ("stats", C.POINTER(lt_stats)), ("status", C.c_int)]

_lib.lt_opts_default.argtypes = [C.POINTER(lt_opts)]
_lib.lt_opts_default.restype = None
_lib.lt_setup.argtypes = [C.POINTER(lt_grid), _vp, _vp, C.POINTER(lt_bc), _vp, C.POINTER(_h)]
_lib.lt_setup.restype = C.c_int
_lib.lt_setup_p1.argtypes = [C.POINTER(lt_grid), _vp, _vp, _vp, C.POINTER(_h)]
_lib.lt_setup_p1.restype = C.c_int
_lib.lt_solve.argtypes = [_h, C.POINTER(lt_sources), _dp, C.c_int, C.POINTER(lt_contour),
                          C.POINTER(lt_points), C.POINTER(lt_opts), _vp, C.POINTER(lt_stats)]
_lib.lt_solve.restype = C.c_int
_lib.lt_adjoint.argtypes = [_h, C.POINTER(lt_sources), C.POINTER(lt_points), _dp, C.c_int,
                            C.POINTER(lt_contour), C.POINTER(lt_opts), _vp, _vp, C.POINTER(lt_stats)]
_lib.lt_adjoint.restype = C.c_int
_lib.lt_solve_batch.argtypes = [C.POINTER(lt_solve_item), C.c_int]
_lib.lt_solve_batch.restype = C.c_int
_lib.lt_adjoint_batch.argtypes = [C.POINTER(lt_adjoint_item), C.c_int]
_lib.lt_adjoint_batch.restype = C.c_int
_lib.lt_autotune.argtypes = [_h, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int, _dp]
_lib.lt_autotune.restype = C.c_int
_lib.lt_set_tiles.argtypes = [_h, C.c_int, C.POINTER(C.c_int), C.c_int]
_lib.lt_set_tiles.restype = C.c_int
_lib.lt_tile_shape.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
_lib.lt_tile_shape.restype = C.c_int
_lib.lt_talbot.argtypes = [C.c_int, C.c_double, _dp, _dp]
_lib.lt_talbot.restype = C.c_int
_lib.lt_apply_operator.argtypes = [_h, C.c_int, C.c_double, C.c_double, _vp, _vp, C.c_int]
_lib.lt_apply_operator.restype = C.c_int
_lib.lt_vcycle.argtypes = [_h, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int]
_lib.lt_vcycle.restype = C.c_int
_lib.lt_vcycle_noalloc.argtypes = [_h, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int]
_lib.lt_vcycle_noalloc.restype = C.c_int
_lib.lt_cov_apply.argtypes = [_h, C.c_double, _dp, C.c_int, _vp, _vp]
_lib.lt_cov_apply.restype = C.c_int
_lib.lt_geostat_step.argtypes = [_h, C.c_void_p, _vp, _vp, _vp, _vp, _dp, C.c_void_p]
_lib.lt_geostat_step.restype = C.c_int
_lib.lt_geostat_invert.argtypes = [C.c_void_p, C.c_void_p, _vp, C.c_void_p, _vp, _vp, C.c_int, _vp, _vp, _dp, _dp]
_lib.lt_geostat_invert.restype = C.c_int
_lib.lt_shift_invert.argtypes = [_h, C.c_double, C.c_double, C.c_int, _vp, _vp]
_lib.lt_shift_invert.restype = C.c_int
_lib.lt_shifted_solve_block.argtypes = [_h, C.c_int, _dp, _dp, C.c_int, _dp, C.c_int, C.c_int, _vp,
                                        C.POINTER(lt_opts), _vp, C.POINTER(lt_stats)]
_lib.lt_shifted_solve_block.restype = C.c_int
_lib.lt_krylov_basis.argtypes = [_h, C.c_int, C.c_int, _dp, _dp, _dp, C.POINTER(C.c_int)]
_lib.lt_krylov_basis.restype = C.c_int
_lib.lt_level_shape.argtypes = [_h, C.c_int, C.POINTER(C.c_int)]
_lib.lt_level_shape.restype = C.c_int
_lib.lt_strerror.argtypes = [C.c_int]
_lib.lt_strerror.restype = C.c_char_p
_lib.lt_last_error.argtypes = []
_lib.lt_last_error.restype = C.c_char_p
_lib.lt_destroy.argtypes = [_h]
_lib.lt_destroy.restype = None
_fp = C.POINTER(C.c_float)
_lib.lt_unet_create.argtypes = [C.c_ulonglong, _vp, C.POINTER(_h)]
_lib.lt_unet_create.restype = C.c_int
_lib.lt_unet_nparams.argtypes = [_h]
_lib.lt_unet_nparams.restype = C.c_longlong
_lib.lt_unet_get_params.argtypes = [_h, _fp]
_lib.lt_unet_get_params.restype = C.c_int
_lib.lt_unet_set_params.argtypes = [_h, _fp]
_lib.lt_unet_set_params.restype = C.c_int
_lib.lt_unet_apply.argtypes = [_h, _h, C.c_double, C.c_double, C.c_int, _vp, _vp]
_lib.lt_unet_apply.restype = C.c_int
_lib.lt_unet_train_step.argtypes = [_h, _h, C.c_double, C.c_double, C.c_int, _vp, _vp, C.c_float, _fp]
_lib.lt_unet_train_step.restype = C.c_int
_lib.lt_unet_grad.argtypes = [_h, _h, C.c_double, C.c_double, C.c_int, _vp, _vp, _fp]
_lib.lt_unet_grad.restype = C.c_int
_lib.lt_unet_attach.argtypes = [_h, _h]
_lib.lt_unet_attach.restype = C.c_int
_lib.lt_unet_destroy.argtypes = [_h]
_lib.lt_unet_destroy.restype = None
_lib.lt_precond_solve.argtypes = [_h, C.c_double, C.c_double, C.c_int, _vp, _vp, C.c_double, C.c_int]
_lib.lt_precond_solve.restype = C.c_int


class LTError(RuntimeError):
    def __init__(self, code):
        self.code = code
        super().__init__(f"{lt_strerror(code)} ({_lib.lt_last_error().decode()})")


def _check(rc):
    if rc < 0:
        raise LTError(rc)
    return rc


def lt_strerror(code: int) -> str:
    return _lib.lt_strerror(code).decode()


def lt_last_error() -> str:
    return _lib.lt_last_error().decode()


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _points(xyz):
    a = np.asarray(xyz, dtype=np.float64)
    a = np.ascontiguousarray(a.reshape(0, 3) if a.size == 0 else np.atleast_2d(a))
    if a.shape[1] != 3:
        raise ValueError("points must have shape [n, 3]")
    return lt_points(a.shape[0], a.ctypes.data_as(_dp)), a


def _sources(xyz, q, phi0=None):
    """lt_sources for wells at xyz pumping at rates q (scalar or one per well) and an
    optional initial head phi0 (float64 CUDA tensor [N]); returns it with what it points to."""
    sp, sa = _points(xyz)
    qa = np.ascontiguousarray(np.broadcast_to(np.asarray(q, dtype=np.float64), (sa.shape[0],)).copy())
    ptr0 = _dev_f64(phi0, "phi0") if phi0 is not None else None
    src = lt_sources(sp, qa.ctypes.data_as(_dp), ptr0)
    return src, (sp, sa, qa, phi0)


def lt_opts_default() -> lt_opts:
    o = lt_opts()
    _lib.lt_opts_default(C.byref(o))
    return o


def make_opts(**kw) -> lt_opts:
    """lt_opts with defaults overridden by keyword (tau may be a list of complex)."""
    o = lt_opts_default()
    tau = kw.pop("tau", None)
    for k, v in kw.items():
        setattr(o, k, v)
    if tau is not None:
        arr = np.ascontiguousarray(np.array([[complex(t).real, complex(t).imag] for t in tau]).ravel())
        o.tau_reim = arr.ctypes.data_as(_dp)
        o.n_tau = len(tau)
        o._keep = arr
    return o


class Handle:
    """Owns an lt_handle; lt_destroy on close or garbage collection."""

    def __init__(self, ptr, grid, stream, nparam=None):
        self.ptr = ptr
        self.grid = grid
        self.stream = stream
        self._nparam = nparam

    @property
    def N(self):
        return self.grid.n[0] * self.grid.n[1] * self.grid.n[2]

    @property
    def nparam(self):
        """Cells the sensitivities run over (the cells of a P1 handle's cell grid, else N)."""
        return self.N if self._nparam is None else self._nparam

    def close(self):
        if self.ptr:
            _lib.lt_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lt_setup(ndim, n, h, kappa, S, bc=(0, 0, 0, 0, 0, 0), stream=None, sy=0.0) -> Handle:
    g = lt_grid(int(ndim), (C.c_int * 3)(*[int(a) for a in n]), (C.c_double * 3)(*[float(a) for a in h]))
    b = lt_bc((C.c_int * 6)(*[int(a) for a in bc]), float(sy))
    out = _h()
    sp = _stream_ptr(stream)
    _check(_lib.lt_setup(C.byref(g), _dev_f64(kappa, "kappa"), _dev_f64(S, "S"), C.byref(b), sp, C.byref(out)))
    return Handle(out, g, sp)


def lt_setup_p1(n, h, kappa, S, stream=None) -> Handle:
    """P1 elements on a 2D (n[0] x n[1]) or 3D (n[0] x n[1] x n[2], n[2] > 1) cell grid (kappa, S
    per cell, float64 CUDA tensors); the handle's unknowns are the interior vertices."""
    nd = 3 if len(n) > 2 and int(n[2]) > 1 else 2
    nn = [int(v) for v in n[:nd]] + [1] * (3 - nd)
    hh = [float(v) for v in h[:nd]] + [1.0] * (3 - nd)
    g = lt_grid(nd, (C.c_int * 3)(*nn), (C.c_double * 3)(*hh))
    out = _h()
    sp = _stream_ptr(stream)
    _check(_lib.lt_setup_p1(C.byref(g), _dev_f64(kappa, "kappa"), _dev_f64(S, "S"), sp, C.byref(out)))
    gv = lt_grid(nd, (C.c_int * 3)(*[v - 1 if a < nd else 1 for a, v in enumerate(nn)]), (C.c_double * 3)(*hh))
    return Handle(out, gv, sp, nparam=nn[0] * nn[1] * nn[2])


def _stats(nrhs, nshift):
    st = lt_stats()
    it = np.zeros(nrhs, dtype=np.int32)
    tr = np.zeros(nrhs * nshift, dtype=np.float64)
    st.iters_per_rhs = it.ctypes.data_as(C.POINTER(C.c_int))
    st.true_relres = tr.ctypes.data_as(_dp)
    return st, it, tr


def _stats_dict(st, it, tr, rc, nrhs, nshift):
    return {"rc": rc, "n_rhs": st.n_rhs, "n_shifts": st.n_shifts, "iters_max": st.iters_max,
            "vcycles": st.vcycles, "levels": st.levels, "true_relres_max": st.true_relres_max,
            "seconds": st.seconds, "iters_per_rhs": it.copy(), "true_relres": tr.reshape(nrhs, nshift).copy(),
            "net_applied": st.net_applied, "net_rejected": st.net_rejected,
            "net_disabled_at": st.net_disabled_at,
            "prof_launches": st.prof_launches, "prof_ms": st.prof_ms, "prof_bytes": st.prof_bytes,
            "resolves": st.resolves, "factorizations": st.factorizations, "factor_ms": st.factor_ms}


def lt_solve(handle: Handle, sources, q, times, nz, receivers, opts: lt_opts | None = None, phi_out=None,
             phi0=None):
    """Heads [max(ns, 1), nr, nt] as a float64 CUDA tensor, plus a stats dict.

    ``q``: one rate for every well or one per well; ``phi0``: optional initial head
    (float64 CUDA tensor [N]) whose heads are added to every row."""
    import torch
    src, keep = _sources(sources, q, phi0)
    rp, ra = _points(receivers)
    t = np.ascontiguousarray(np.asarray(times, dtype=np.float64).ravel())
    ns, nr, nt = keep[1].shape[0], ra.shape[0], t.size
    nrhs = ns + (1 if phi0 is not None else 0)
    if phi_out is None:
        phi_out = torch.empty((max(ns, 1), nr, nt), dtype=torch.float64, device="cuda")
    con = lt_contour(int(nz))
    o = opts if opts is not None else lt_opts_default()
    st, it, tr = _stats(nrhs, nt * (int(nz) // 2))
    rc = _check(_lib.lt_solve(handle.ptr, C.byref(src), t.ctypes.data_as(_dp), nt, C.byref(con),
                              C.byref(rp), C.byref(o), _dev_f64(phi_out, "phi_out"), C.byref(st)))
    return phi_out, _stats_dict(st, it, tr, rc, nrhs, nt * (int(nz) // 2))


def lt_adjoint(handle: Handle, sources, q, receivers, times, nz, opts: lt_opts | None = None,
               dlnK=None, dlnS=None):
    """Sensitivities [ns, nr, nt, handle.nparam] to ln kappa and ln S (float64 CUDA tensors) and stats."""
    import torch
    src, keep = _sources(sources, q)
    rp, ra = _points(receivers)
    t = np.ascontiguousarray(np.asarray(times, dtype=np.float64).ravel())
    ns, nr, nt = keep[1].shape[0], ra.shape[0], t.size
    shape = (ns, nr, nt, handle.nparam)
    if dlnK is None:
        dlnK = torch.empty(shape, dtype=torch.float64, device="cuda")
    if dlnS is None:
        dlnS = torch.empty(shape, dtype=torch.float64, device="cuda")
    con = lt_contour(int(nz))
    o = opts if opts is not None else lt_opts_default()
    st, it, tr = _stats(ns + nr, nt * (int(nz) // 2))
    rc = _check(_lib.lt_adjoint(handle.ptr, C.byref(src), C.byref(rp), t.ctypes.data_as(_dp), nt,
                                C.byref(con), C.byref(o), _dev_f64(dlnK, "dlnK"), _dev_f64(dlnS, "dlnS"),
                                C.byref(st)))
    return dlnK, dlnS, _stats_dict(st, it, tr, rc, ns + nr, nt * (int(nz) // 2))


def lt_solve_batch(problems):
    """Solve several problems in one lt_solve_batch call.

    ``problems``: sequence of dicts with keys handle, sources, q, times, nz,
    receivers and optionally opts, phi0 and phi_out (the arguments of lt_solve).
    Returns (list of phi tensors, list of stats dicts, batch return code).
    """
    import torch
    n = len(problems)
    items = (lt_solve_item * n)()
    keep, outs, meta = [], [], []
    for i, pr in enumerate(problems):
        phi0 = pr.get("phi0")
        src, sk = _sources(pr["sources"], pr.get("q", 1.0), phi0)
        rp, ra = _points(pr["receivers"])
        t = np.ascontiguousarray(np.asarray(pr["times"], dtype=np.float64).ravel())
        ns, nr, nt = sk[1].shape[0], ra.shape[0], t.size
        nrhs = ns + (1 if phi0 is not None else 0)
        nz = int(pr["nz"])
        phi = pr.get("phi_out")
        if phi is None:
            phi = torch.empty((max(ns, 1), nr, nt), dtype=torch.float64, device="cuda")
        con = lt_contour(nz)
        o = pr.get("opts") or lt_opts_default()
        st, it, tr = _stats(nrhs, nt * (nz // 2))
        keep.append((src, sk, rp, ra, t, con, o, st, it, tr))
        items[i] = lt_solve_item(pr["handle"].ptr, C.pointer(src), t.ctypes.data_as(_dp),
                                 nt, C.pointer(con), C.pointer(rp), C.pointer(o), _dev_f64(phi, "phi_out"),
                                 C.pointer(st), 0)
        outs.append(phi)
        meta.append((nrhs, nt * (nz // 2)))
    rc = _check(_lib.lt_solve_batch(items, n))
    stats = [_stats_dict(k[7], k[8], k[9], items[i].status, *meta[i]) for i, k in enumerate(keep)]
    return outs, stats, rc


def lt_adjoint_batch(problems):
    """Sensitivities of several problems in one lt_adjoint_batch call.

    ``problems``: dicts with keys handle, sources, q, receivers, times, nz and
    optionally opts, dlnK and dlnS (output tensors).  Returns (list of (dlnK, dlnS),
    list of stats, code).
    """
    import torch
    n = len(problems)
    items = (lt_adjoint_item * n)()
    keep, outs, meta = [], [], []
    for i, pr in enumerate(problems):
        src, sk = _sources(pr["sources"], pr.get("q", 1.0))
        rp, ra = _points(pr["receivers"])
        t = np.ascontiguousarray(np.asarray(pr["times"], dtype=np.float64).ravel())
        ns, nr, nt = sk[1].shape[0], ra.shape[0], t.size
        nz = int(pr["nz"])
        shape = (ns, nr, nt, pr["handle"].nparam)
        dK = pr.get("dlnK")
        dS = pr.get("dlnS")
        if dK is None:
            dK = torch.empty(shape, dtype=torch.float64, device="cuda")
        if dS is None:
            dS = torch.empty(shape, dtype=torch.float64, device="cuda")
        con = lt_contour(nz)
        o = pr.get("opts") or lt_opts_default()
        st, it, tr = _stats(ns + nr, nt * (nz // 2))
        keep.append((src, sk, rp, ra, t, con, o, st, it, tr))
        items[i] = lt_adjoint_item(pr["handle"].ptr, C.pointer(src), C.pointer(rp),
                                   t.ctypes.data_as(_dp), nt, C.pointer(con), C.pointer(o),
                                   _dev_f64(dK, "dlnK"), _dev_f64(dS, "dlnS"), C.pointer(st), 0)
        outs.append((dK, dS))
        meta.append((ns + nr, nt * (nz // 2)))
    rc = _check(_lib.lt_adjoint_batch(items, n))
    stats = [_stats_dict(k[7], k[8], k[9], items[i].status, *meta[i]) for i, k in enumerate(keep)]
    return outs, stats, rc


def lt_autotune(handle: Handle, precision, nu1=2, nu2=2, nvec=8):
    """Tune the smoother tile shape per level; returns (shape ids of the tuned levels, us per step)."""
    tiles = (C.c_int * 16)()
    us = C.c_double()
    n = _check(_lib.lt_autotune(handle.ptr, int(precision), int(nu1), int(nu2), int(nvec), tiles, 16, C.byref(us)))
    return [tiles[i] for i in range(n)], us.value


def lt_set_tiles(handle: Handle, precision, tiles):
    arr = (C.c_int * max(1, len(tiles)))(*[int(t) for t in tiles])
    return _check(_lib.lt_set_tiles(handle.ptr, int(precision), arr, len(tiles)))


def lt_tile_shape(tile_id):
    tx, ty = C.c_int(), C.c_int()
    _check(_lib.lt_tile_shape(int(tile_id), C.byref(tx), C.byref(ty)))
    return tx.value, ty.value


def lt_talbot(nz, t):
    """Upper-half Talbot nodes and weights (complex numpy arrays) computed by the library."""
    z = np.zeros(nz, dtype=np.float64)
    w = np.zeros(nz, dtype=np.float64)
    _check(_lib.lt_talbot(int(nz), float(t), z.ctypes.data_as(_dp), w.ctypes.data_as(_dp)))
    return z[0::2] + 1j * z[1::2], w[0::2] + 1j * w[1::2]


def lt_apply_operator(handle: Handle, level, tau, x, y, nvec):
    tau = complex(tau)
    return _check(_lib.lt_apply_operator(handle.ptr, int(level), tau.real, tau.imag, _dev_f64(x, "x"),
                                         _dev_f64(y, "y"), int(nvec)))


def lt_vcycle(handle: Handle, tau, precision, nu1, nu2, b, x, nvec):
    tau = complex(tau)
    return _check(_lib.lt_vcycle(handle.ptr, tau.real, tau.imag, int(precision), int(nu1), int(nu2),
                                 _dev_f64(b, "b"), _dev_f64(x, "x"), int(nvec)))


def lt_vcycle_noalloc(handle: Handle, tau, precision, nu1, nu2, b, x, nvec):
    """lt_vcycle with every work vector in the library's scratch (allocates nothing)."""
    tau = complex(tau)
    return _check(_lib.lt_vcycle_noalloc(handle.ptr, tau.real, tau.imag, int(precision), int(nu1), int(nu2),
                                         _dev_f64(b, "b"), _dev_f64(x, "x"), int(nvec)))


def lt_shift_invert(handle: Handle, tau, b, x, nvec):
    """x = (K + tau M)^{-1} b for nvec complex vectors [nvec][2][N] (float64 CUDA tensors)."""
    tau = complex(tau)
    return _check(_lib.lt_shift_invert(handle.ptr, tau.real, tau.imag, int(nvec), _dev_f64(b, "b"),
                                       _dev_f64(x, "x")))


def lt_shifted_solve_block(handle: Handle, shifts, b, block, taus, opts: lt_opts | None = None, weights=None,
                           x=None):
    """x[k] = (K + shifts[k] M)^{-1} b for every column of b ([nvec, 2, N] float64 CUDA tensor), by
    block flexible GMRES over blocks of `block` columns (preconditioner shifts `taus`, cyclic).
    Returns (x [nshift, nvec, 2, N], stats dict)."""
    import torch
    z = np.asarray(shifts, dtype=np.complex128).ravel()
    t = np.asarray(taus, dtype=np.complex128).ravel()
    zz = np.ascontiguousarray(np.stack([z.real, z.imag], axis=1))
    tt = np.ascontiguousarray(np.stack([t.real, t.imag], axis=1))
    nvec = int(b.shape[0])
    if x is None:
        x = torch.empty((z.size, nvec, 2, handle.N), dtype=torch.float64, device="cuda")
    w = None if weights is None else np.ascontiguousarray(np.asarray(weights, dtype=np.float64).ravel())
    o = opts if opts is not None else lt_opts_default()
    st, it, tr = _stats(nvec, z.size)
    rc = _check(_lib.lt_shifted_solve_block(handle.ptr, z.size, zz.ctypes.data_as(_dp),
                                            None if w is None else w.ctypes.data_as(_dp), t.size,
                                            tt.ctypes.data_as(_dp), nvec, int(block), _dev_f64(b, "b"),
                                            C.byref(o), _dev_f64(x, "x"), C.byref(st)))
    return x, _stats_dict(st, it, tr, rc, nvec, z.size)


def lt_cov_apply(handle: Handle, var, length, v, out, nvec):
    """out = Q v for nvec float64 CUDA vectors [nvec][N] (exponential covariance, lengths per axis)."""
    ln = np.ascontiguousarray(np.broadcast_to(np.asarray(length, dtype=np.float64), (3,)).copy())
    return _check(_lib.lt_cov_apply(handle.ptr, float(var), ln.ctypes.data_as(_dp), int(nvec), _dev_f64(v, "v"),
                                    _dev_f64(out, "out")))


def _geostat(sources, q, observations, times, nz, var, length, r, opts):
    sp, sa = _points(sources)
    qa = np.ascontiguousarray(np.broadcast_to(np.asarray(q, dtype=np.float64), (sa.shape[0],)).copy())
    op, oa = _points(observations)
    t = np.ascontiguousarray(np.asarray(times, dtype=np.float64).ravel())
    ln = np.broadcast_to(np.asarray(length, dtype=np.float64), (3,))
    g = lt_geostat(sp, qa.ctypes.data_as(_dp), op, t.ctypes.data_as(_dp), t.size, lt_contour(int(nz)), float(var),
                   (C.c_double * 3)(*[float(a) for a in ln]), float(r),
                   C.cast(C.pointer(opts), C.c_void_p) if opts is not None else None)
    return g, (sp, sa, qa, op, oa, t, opts), sa.shape[0] * oa.shape[0] * t.size


def lt_geostat_step(handle: Handle, sources, q, observations, times, nz, var, length, r, y, s, s_next,
                    opts: lt_opts | None = None):
    """One Gauss-Newton step of Algorithm 2 at s (the handle's ln kappa): fills s_next (float64 CUDA
    [N]) and returns (h(s) as a float64 CUDA tensor [M], beta, return code)."""
    import torch
    g, keep, M = _geostat(sources, q, observations, times, nz, var, length, r, opts)
    hs = torch.empty(M, dtype=torch.float64, device="cuda")
    beta = C.c_double()
    rc = _check(_lib.lt_geostat_step(handle.ptr, C.byref(g), _dev_f64(y, "y"), _dev_f64(s, "s"),
                                     _dev_f64(s_next, "s_next"), _dev_f64(hs, "hs"), C.byref(beta), None))
    return hs, beta.value, rc


def lt_geostat_invert(ndim, n, h, S, sources, q, observations, times, nz, var, length, r, y, s0, iters,
                      bc=(0, 0, 0, 0, 0, 0), sy=0.0, opts: lt_opts | None = None, stream=None):
    """Algorithm 2 for iters steps from s0: (s as a float64 CUDA tensor [N], misfit per step,
    relative step size per step, return code)."""
    import torch
    gr = lt_grid(int(ndim), (C.c_int * 3)(*[int(a) for a in n]), (C.c_double * 3)(*[float(a) for a in h]))
    b = lt_bc((C.c_int * 6)(*[int(a) for a in bc]), float(sy))
    g, keep, M = _geostat(sources, q, observations, times, nz, var, length, r, opts)
    out = torch.empty_like(s0)
    mis = np.zeros(iters)
    stp = np.zeros(iters)
    rc = _check(_lib.lt_geostat_invert(C.byref(gr), C.byref(b), _dev_f64(S, "S"), C.byref(g), _dev_f64(y, "y"),
                                       _dev_f64(s0, "s0"), int(iters), _stream_ptr(stream), _dev_f64(out, "s_out"),
                                       mis.ctypes.data_as(_dp), stp.ctypes.data_as(_dp)))
    return out, mis, stp, rc


def lt_krylov_basis(handle: Handle, rhs):
    """(V [m+1, N] complex, U [m, N] complex, Hbar [m+1, m] complex) of the last solve's basis
    for right-hand side `rhs` (numpy arrays)."""
    m = C.c_int()
    rc = _lib.lt_krylov_basis(handle.ptr, int(rhs), 0, None, None, None, C.byref(m))
    mm = m.value
    if rc < 0 and mm == 0:
        raise LTError(rc)
    N = handle.N
    V = np.zeros((mm + 1) * 2 * N)
    U = np.zeros(max(mm, 1) * 2 * N)
    H = np.zeros(max(mm, 1) * (mm + 1) * 2)
    _check(_lib.lt_krylov_basis(handle.ptr, int(rhs), mm, V.ctypes.data_as(_dp), U.ctypes.data_as(_dp),
                                H.ctypes.data_as(_dp), C.byref(m)))
    V = V.reshape(mm + 1, 2, N)
    U = U.reshape(-1, 2, N)[:mm]
    Hc = H.reshape(-1, mm + 1, 2)[:mm]
    return (V[:, 0] + 1j * V[:, 1], U[:, 0] + 1j * U[:, 1], (Hc[..., 0] + 1j * Hc[..., 1]).T)


def lt_level_shape(handle: Handle, level):
    n = (C.c_int * 3)()
    nl = _check(_lib.lt_level_shape(handle.ptr, int(level), n))
    return nl, tuple(n)


def lt_destroy(handle: Handle):
    handle.close()


def exported_symbols():
    """Names the library exports among those of include/lt.h (no GPU needed)."""
    return [name for name in _ABI_NAMES if hasattr(_lib, name)]


_ABI_NAMES = ["lt_opts_default", "lt_setup", "lt_setup_p1", "lt_solve", "lt_adjoint", "lt_talbot", "lt_apply_operator",
              "lt_vcycle", "lt_level_shape", "lt_strerror", "lt_last_error", "lt_destroy", "lt_unet_create",
              "lt_unet_nparams", "lt_unet_get_params", "lt_unet_set_params", "lt_unet_apply",
              "lt_unet_train_step", "lt_unet_grad", "lt_unet_attach", "lt_unet_destroy", "lt_precond_solve",
              "lt_solve_batch", "lt_adjoint_batch", "lt_autotune", "lt_set_tiles", "lt_tile_shape",
              "lt_krylov_basis", "lt_shifted_solve_block"]


# ---------------------------------------------------------------- learned preconditioner
class UNet:
    """Owns an lt_unet (created on the current torch stream)."""

    def __init__(self, seed=0, stream=None):
        self.ptr = _h()
        _check(_lib.lt_unet_create(int(seed), _stream_ptr(stream), C.byref(self.ptr)))

    @property
    def nparams(self):
        return int(_lib.lt_unet_nparams(self.ptr))

    def get_params(self):
        p = np.zeros(self.nparams, dtype=np.float32)
        _check(_lib.lt_unet_get_params(self.ptr, p.ctypes.data_as(_fp)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        if p.size != self.nparams:
            raise ValueError("wrong parameter count")
        _check(_lib.lt_unet_set_params(self.ptr, p.ctypes.data_as(_fp)))

    def close(self):
        if self.ptr:
            _lib.lt_unet_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lt_unet_apply(net: UNet, handle: Handle, tau, r, e, nvec):
    tau = complex(tau)
    return _check(_lib.lt_unet_apply(net.ptr, handle.ptr, tau.real, tau.imag, int(nvec), _dev_f64(r, "r"),
                                     _dev_f64(e, "e")))


def lt_unet_train_step(net: UNet, handle: Handle, tau, r, e, nvec, lr):
    tau = complex(tau)
    loss = C.c_float(0.0)
    _check(_lib.lt_unet_train_step(net.ptr, handle.ptr, tau.real, tau.imag, int(nvec), _dev_f64(r, "r"),
                                   _dev_f64(e, "e"), float(lr), C.byref(loss)))
    return float(loss.value)


def lt_unet_grad(net: UNet, handle: Handle, tau, r, e, nvec):
    tau = complex(tau)
    g = np.zeros(net.nparams, dtype=np.float32)
    _check(_lib.lt_unet_grad(net.ptr, handle.ptr, tau.real, tau.imag, int(nvec), _dev_f64(r, "r"),
                             _dev_f64(e, "e"), g.ctypes.data_as(_fp)))
    return g


def lt_unet_attach(handle: Handle, net):
    return _check(_lib.lt_unet_attach(handle.ptr, net.ptr if net is not None else None))


def lt_precond_solve(handle: Handle, tau, r, e, nvec, tol=1e-10, maxcycles=60):
    tau = complex(tau)
    return _check(_lib.lt_precond_solve(handle.ptr, tau.real, tau.imag, int(nvec), _dev_f64(r, "r"),
                                        _dev_f64(e, "e"), float(tol), int(maxcycles)))


# ---------------------------------------------------------------- complex SoA helpers
def to_planes(zc):
    """complex torch tensor [..., N] -> float64 planes [..., 2, N] (contiguous)."""
    import torch
    return torch.stack([zc.real, zc.imag], dim=-2).to(torch.float64).contiguous()


def from_planes(p):
    return p[..., 0, :] + 1j * p[..., 1, :]
