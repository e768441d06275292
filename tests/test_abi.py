"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/nf.h declares, and rejects invalid arguments on the host side before
touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nf.h")
LIB = os.path.join(ROOT, "paper_2606_06720_amd", "libnf.so")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nf_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnf.so not built: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for s in ("nf_create_grid", "nf_destroy_grid", "nf_pressure_solve", "nf_step", "nf_run", "nf_energy",
              "nf_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_version_string(lib):
    lib.nf_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.nf_version()


@pytest.mark.parametrize("n", [(7, 8), (8, 6), (4, 8), (8192, 8), (8, 0), (12, 16)])
def test_create_grid_rejects_bad_sizes_on_host(lib, n):
    h = ctypes.c_void_p()
    nn = (ctypes.c_int64 * 3)(n[0], n[1], 1)
    L = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    rc = lib.nf_create_grid(ctypes.byref(h), 2, nn, L, 0, None)
    assert rc == -1 and not h.value


def test_create_grid_rejects_bad_geometry_on_host(lib):
    h = ctypes.c_void_p()
    nn = (ctypes.c_int64 * 3)(16, 16, 1)
    for L, ndim, dtype in (((0.0, 1.0, 1.0), 2, 0), ((1.0, -1.0, 1.0), 2, 0), ((1.0, 1.0, 1.0), 4, 0),
                           ((1.0, 1.0, 1.0), 2, 7)):
        LL = (ctypes.c_double * 3)(*L)
        assert lib.nf_create_grid(ctypes.byref(h), ndim, nn, LL, dtype, None) == -1


def test_null_handle_calls_are_rejected(lib):
    lib.nf_pressure_solve.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
    assert lib.nf_pressure_solve(None, None, None, None, None, 1e-10, 10, None) == -1
    assert lib.nf_destroy_grid(None) == 0
    lib.nf_set_inner_tolerance.argtypes = [ctypes.c_void_p, ctypes.c_double]
    assert lib.nf_set_inner_tolerance(None, 1e-5) == -1
    lib.nf_batch_set_partitions.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert lib.nf_batch_set_partitions(None, 1) == -1
    lib.nf_batch_partitions.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.nf_batch_partitions(None, None) == -1
    lib.nf_batch_set_graphs.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert lib.nf_batch_set_graphs(None, 1) == -1


def test_batch_create_rejects_bad_sizes_on_host(lib):
    # the failure path frees a partly built ensemble (instances not created yet)
    lib.nf_batch_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    for sizes in ((32, 33), (7, 64, 32, 32)):
        h = ctypes.c_void_p()
        nn = (ctypes.c_int64 * len(sizes))(*sizes)
        LL = (ctypes.c_double * len(sizes))(*([1.0] * len(sizes)))
        assert lib.nf_batch_create(ctypes.byref(h), len(sizes) // 2, nn, LL, 0, None) == -1
        assert not h.value


@pytest.mark.parametrize("n", [(512, 256), (256, 512), (4096, 32), (50, 50), (12, 16), (8192, 8)])
def test_noalloc_solve_rejects_sizes_beyond_its_workspace_on_host(lib, n):
    # the size check comes before any device work, so it runs without a GPU
    nn = (ctypes.c_int64 * 2)(*n)
    L = (ctypes.c_double * 2)(1.0, 1.0)
    dummy = ctypes.c_void_p(16)
    lib.nf_pressure_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                              ctypes.c_int, ctypes.c_void_p]
    lib.nf_last_error.restype = ctypes.c_char_p
    lib.nf_last_error.argtypes = [ctypes.c_void_p]
    rc = lib.nf_pressure_solve_noalloc(nn, L, None, dummy, dummy, dummy, dummy, 1e-10, 100, None)
    assert rc == -1
    assert b"allocation-free" in lib.nf_last_error(None)
