"""CPU checks of the C ABI: the library loads, exports every entry point that
include/cryosgd.h declares, and rejects invalid arguments on the host before
any GPU work is enqueued (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cryosgd.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def b():
    from paper_2311_16100_amd import binding
    binding.lib()
    return binding


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("csg_project", "csg_backproject", "csg_hvp", "csg_hutchinson_diag", "csg_precond_sgd_step",
                     "csg_gradient", "csg_workspace_bytes", "csg_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(b):
    lib = ctypes.CDLL(b.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # and the binding knows every one of them
    assert set(declared_functions()) <= set(b.EXPORTS)


def test_workspace_sizes(b):
    g = b.Grid(256)
    vol = 256 ** 3 * 8
    # trilinear: only the brick tables (the probe pair is regenerated from
    # its hash and z (.) Hz is formed in the brick kernel); the
    # nearest-neighbour kernels keep the pair and its product
    assert 0 < b.workspace_bytes(g, 1024, b.CSG_WS_HUTCHINSON) == b.workspace_bytes(g, 1024, b.CSG_WS_GRADIENT)
    assert b.workspace_bytes(b.Grid(256, interp=0), 1024, b.CSG_WS_HUTCHINSON) >= 2 * vol
    # deterministic adjoint: the 64-bit fixed-point volume on trilinear
    # grids, one image per batch image (owner-computes kernel) on
    # nearest-neighbour grids
    for kind in (b.CSG_WS_GRADIENT_DETERMINISTIC, b.CSG_WS_BACKPROJECT_DETERMINISTIC):
        assert b.workspace_bytes(g, 1024, kind) >= 2 * vol
    nn = b.Grid(256, interp=0)
    assert b.workspace_bytes(nn, 1024, b.CSG_WS_GRADIENT_DETERMINISTIC) >= 1024 * 256 * 256 * 8
    assert b.workspace_bytes(nn, 1024, b.CSG_WS_BACKPROJECT_DETERMINISTIC) == 0
    assert b.workspace_bytes(g, 1024, b.CSG_WS_GRADIENT) > 0
    assert b.workspace_bytes(b.Grid(7), 1, b.CSG_WS_HUTCHINSON) == 0


def _call_project(b, grid, optics, n=1):
    L = b.lib()
    p = b._Poses(n, None, None)
    return L.csg_project(ctypes.byref(grid), ctypes.byref(optics), ctypes.byref(p), None, None, None, None, None, 0,
                         None)


@pytest.mark.parametrize("M,rmax,interp", [(7, 2.0, 1), (2, 0.0, 1), (2048, 10.0, 1), (32, 16.0, 1),
                                           (32, -1.0, 1), (32, 10.0, 2)])
def test_invalid_grid_rejected(b, M, rmax, interp):
    rc = _call_project(b, b._Grid(M, rmax, interp), b.Optics().c())
    assert rc == -1
    assert b.lib().csg_last_error()


@pytest.mark.parametrize("field,value", [("kv", 0.0), ("pixel_A", -1.0), ("amp_contrast", 1.0), ("cs_mm", -2.0)])
def test_invalid_optics_rejected(b, field, value):
    o = b.Optics().c()
    setattr(o, field, value)
    assert _call_project(b, b.Grid(32).c(), o) == -1


def test_null_pointers_rejected(b):
    # n > 0 with NULL rotations
    assert _call_project(b, b.Grid(32).c(), b.Optics().c(), n=3) == -1
    assert b"non-NULL" in b.lib().csg_last_error()
    L = b.lib()
    stats = None
    assert L.csg_precond_sgd_step(10, None, None, None, None, None, 1, 0.9, 1.0, 1.0, None, None, stats, None) == -1
    assert L.csg_rademacher(-1, 0, 0, None, None) == -1
    # a zero-length request is a no-op and succeeds without touching the GPU
    assert L.csg_rademacher(0, 0, 0, None, None) == 0
    p = b._Poses(0, None, None)
    g, o = b.Grid(16).c(), b.Optics().c()
    assert L.csg_project(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), None, None, None, None, None, 0,
                         None) == 0


def test_bad_ctf_power_rejected(b):
    L = b.lib()
    g, o = b.Grid(16).c(), b.Optics().c()
    p = b._Poses(0, None, None)
    assert L.csg_backproject(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), None, 3, 1.0, None, 0, None, 0,
                             None) == -1


def test_timing_arguments_checked(b):
    L = b.lib()
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    assert L.csg_timing_read(7, ctypes.byref(ms), ctypes.byref(n)) == -1
    assert L.csg_timing_read(-1, ctypes.byref(ms), ctypes.byref(n)) == -1
    assert L.csg_timing_read(0, None, ctypes.byref(n)) == -1
    # nothing recorded: zero launches, and reading needs no device
    assert b.timing_read("gradient") == (0.0, 0)
    assert b.timing_read("gradient_probe") == (0.0, 0)
    b.timing_enable(False)


def test_noalloc_gradient_checks_arguments_on_the_host(b):
    """The allocation-free gradient rejects bad arguments before it looks up
    its static scratch or enqueues anything."""
    L = b.lib()
    g, o = b.Grid(32).c(), b.Optics().c()
    p = b._Poses(4, None, None)
    assert L.csg_gradient_noalloc(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), None, None, 1.0, 0.0, None,
                                  None, None) == -1
    bad = b._Grid(33, 10.0, 1)
    assert L.csg_gradient_noalloc(ctypes.byref(bad), ctypes.byref(o), ctypes.byref(p), None, None, 1.0, 0.0, None,
                                  None, None) == -1
    assert b"must be even" in L.csg_last_error()


def test_gradient_hutchinson_checks_arguments_on_the_host(b):
    """The one-call gradient and Hutchinson diagonal rejects bad arguments
    and a missing workspace before anything is enqueued (the pointers below
    are host buffers that no kernel ever sees)."""
    L = b.lib()
    g, o = b.Grid(32).c(), b.Optics().c()
    bufs = [ctypes.create_string_buffer(64) for _ in range(5)]
    rot, df, vol, x, out = (ctypes.cast(u, ctypes.c_void_p) for u in bufs)
    p = b._Poses(4, rot, df, None)
    diag = ctypes.c_void_p(ctypes.addressof(bufs[4]) + 32)

    def call(n_probe=2, grad=out, dg=diag, ws=None, wn=0, v=vol):
        return L.csg_gradient_hutchinson(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), v, x, 1.0, 0.1, grad,
                                         None, n_probe, 7, 0, dg, ws, wn, None)

    assert call(n_probe=0) == -1 and b"n_probe" in L.csg_last_error()
    assert call(dg=None) == -1 and b"non-NULL" in L.csg_last_error()
    assert call(grad=diag) == -1 and b"alias" in L.csg_last_error()
    assert call(v=out) == -1 and b"alias" in L.csg_last_error()
    assert call() == -3 and b"workspace" in L.csg_last_error()
    need = b.workspace_bytes(b.Grid(32), 4, b.CSG_WS_GRADIENT_HUTCHINSON)
    assert need == max(b.workspace_bytes(b.Grid(32), 4, b.CSG_WS_GRADIENT),
                       b.workspace_bytes(b.Grid(32), 4, b.CSG_WS_HUTCHINSON))
    # nearest-neighbour grids run the two calls in the same workspace: it
    # holds either one's, also where the brick tables of many images exceed
    # the two volumes of the probe product (a small grid)
    for M, n in ((32, 4), (16, 2048), (64, 300)):
        nn = b.Grid(M, interp=0)
        need = b.workspace_bytes(nn, n, b.CSG_WS_GRADIENT_HUTCHINSON)
        assert need == max(b.workspace_bytes(nn, n, b.CSG_WS_HUTCHINSON), b.workspace_bytes(nn, n, b.CSG_WS_GRADIENT))
