"""The C ABI library loads without a GPU and exports every function that
include/lt.h declares; host-only entry points behave (no GPU compute)."""
import ctypes
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lt_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1409_2556_amd import binding
    return binding


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "lt_setup" in names and "lt_solve" in names and "lt_adjoint" in names
    so = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing


def test_host_talbot_table_matches_oracle(lib):
    from oracle.contour import talbot_nodes
    for nz in (16, 20, 24, 40):
        for t in (1e-7, 3e-6, 1.0):
            z, w = talbot_nodes(nz, t)
            z2, w2 = lib.lt_talbot(nz, t)
            np.testing.assert_allclose(z2, z, rtol=1e-14)
            np.testing.assert_allclose(w2, w, rtol=1e-13, atol=1e-15 * np.abs(w).max())


def test_error_codes_without_gpu(lib):
    so = lib._lib
    assert so.lt_setup(None, None, None, None, None, None) == lib.LT_EINVAL
    z = np.zeros(8)
    assert so.lt_talbot(7, 1.0, z.ctypes.data_as(lib._dp), z.ctypes.data_as(lib._dp)) == lib.LT_EINVAL
    assert so.lt_talbot(8, -1.0, z.ctypes.data_as(lib._dp), z.ctypes.data_as(lib._dp)) == lib.LT_EINVAL
    for c in (0, -1, -2, -3, -4, 1):
        assert lib.lt_strerror(c).startswith("LT_")
    o = lib.lt_opts_default()
    assert o.tol == 1e-10 and o.nu1 == 2 and o.nu2 == 2 and o.precision == lib.LT_PREC_FP64
    assert o.method == lib.LT_METHOD_GMRES and o.graph == 0 and o.conv == lib.LT_CONV_WEIGHTED
    so.lt_destroy(None)  # accepted
    # batches are checked before any GPU work: no items, too many, a missing handle
    items = (lib.lt_solve_item * 2)()
    assert so.lt_solve_batch(None, 1) == lib.LT_EINVAL
    assert so.lt_solve_batch(items, 0) == lib.LT_EINVAL
    assert so.lt_solve_batch(items, 65) == lib.LT_EINVAL
    assert so.lt_solve_batch(items, 2) == lib.LT_EINVAL
    assert "no handle" in lib.lt_last_error()
    adj = (lib.lt_adjoint_item * 1)()
    assert so.lt_adjoint_batch(adj, 1) == lib.LT_EINVAL
    # tile shapes
    assert [lib.lt_tile_shape(i) for i in range(4)] == [(32, 16), (64, 8), (16, 16), (16, 8)]
    tx = lib.C.c_int()
    assert so.lt_tile_shape(4, lib.C.byref(tx), lib.C.byref(tx)) == lib.LT_EINVAL
    assert so.lt_autotune(None, 0, 2, 2, 1, None, 0, None) == lib.LT_EINVAL
    assert so.lt_set_tiles(None, 0, None, 0) == lib.LT_EINVAL


def test_setup_rejects_bad_water_table_without_gpu(lib):
    """Boundary arguments are checked before any device call."""
    so = lib._lib
    buf = np.ones(16)
    ptr = buf.ctypes.data_as(lib._vp) if hasattr(lib, "_vp") else buf.ctypes.data
    g = lib.lt_grid(2, (C.c_int * 3)(4, 4, 1), (C.c_double * 3)(0.25, 0.25, 1.0))
    out = lib._h()
    assert C.sizeof(lib.lt_bc) == 32
    for faces, sy in (((0, 0, 0, 0, 0, 2), 0.1),        # water table on a wall a 2D grid lacks
                      ((0, 0, 0, 2, 0, 0), -1.0),       # negative specific yield
                      ((0, 0, 0, 2, 0, 0), float("nan")),
                      ((0, 0, 0, 3, 0, 0), 0.0)):       # unknown type
        b = lib.lt_bc((C.c_int * 6)(*faces), sy)
        assert so.lt_setup(C.byref(g), ptr, ptr, C.byref(b), None, C.byref(out)) == lib.LT_EINVAL
    # a valid water table passes the checks and stops only at the missing device
    b = lib.lt_bc((C.c_int * 6)(0, 0, 0, 2, 0, 0), 0.1)
    assert so.lt_setup(C.byref(g), ptr, ptr, C.byref(b), None, C.byref(out)) == lib.LT_EHIP


def test_setup_rejects_grids_beyond_the_cell_limit_without_gpu(lib):
    """More than 2^28 cells would overflow the smoothers' 32-bit byte offsets of an FP64
    vector plane; lt_setup refuses such a grid before touching the device."""
    so = lib._lib
    buf = np.ones(16)
    ptr = buf.ctypes.data
    out = lib._h()
    big = lib.lt_grid(3, (C.c_int * 3)(1024, 1024, 257), (C.c_double * 3)(1.0, 1.0, 1.0))
    assert so.lt_setup(C.byref(big), ptr, ptr, None, None, C.byref(out)) == lib.LT_EINVAL
    assert "2^28" in lib.lt_last_error()
    # exactly 2^28 cells passes the size check and stops only at the missing device
    edge = lib.lt_grid(3, (C.c_int * 3)(1024, 1024, 256), (C.c_double * 3)(1.0, 1.0, 1.0))
    assert so.lt_setup(C.byref(edge), ptr, ptr, None, None, C.byref(out)) == lib.LT_EHIP


def test_block_solver_checks_arguments_without_gpu(lib):
    """lt_shifted_solve_block refuses a missing handle, shift list or right-hand side before any
    device call."""
    so = lib._lib
    z = np.zeros(4)
    zp = z.ctypes.data_as(lib._dp)
    o = lib.lt_opts_default()
    assert so.lt_shifted_solve_block(None, 2, zp, None, 1, zp, 4, 2, z.ctypes.data, C.byref(o),
                                     z.ctypes.data, None) == lib.LT_EINVAL
    assert "lt_shifted_solve_block" in lib.lt_last_error()
    assert so.lt_shifted_solve_block(None, 0, None, None, 0, None, 0, 0, None, None, None, None) == lib.LT_EINVAL
