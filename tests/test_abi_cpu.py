"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol declared in include/isdf.h, rejects invalid arguments before
touching a device, and its memory planner reproduces the paper's storage
model (N_k N_IP^2 + N_k N_IP N_AO complex numbers; 2.11 GB for diamond at
N_k = 1000, N_IP = 14 x 26, N_AO = 26)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2601_16379_amd as pkg
from paper_2601_16379_amd import isdf as binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "isdf.h")).read()
    return sorted(set(re.findall(r"\b(isdf_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = pkg.load_library()
    declared = _declared_symbols()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(binding.EXPORTS)


def test_version_string():
    assert pkg.isdf_version().startswith("isdf-gfx950")


def test_storage_model_matches_paper_number():
    b = pkg.isdf_storage_model_bytes(1000, 14 * 26, 26)
    assert abs(b / 2 ** 30 - 2.11) < 0.01


def test_plan_bytes_at_most_linear_in_nk():
    # resident data is at most linear in N_k (q-indexed data grows with the
    # classes {q, -q}: 8 of the 2x2x2 mesh, 12 of the 4x2x2 mesh); the r-tile
    # scratch is capped at 2 GiB
    b1 = pkg.isdf_plan_bytes((32, 32, 32), (2, 2, 2), 26, 520)
    b2 = pkg.isdf_plan_bytes((32, 32, 32), (4, 2, 2), 26, 520)
    assert 1.2 < b2 / b1 <= 2.0
    # workload 5 shapes: the orbitals alone are ~53 GB, and eta of all 504
    # classes (FP64, 537 GB) exceeds one GPU, hence the q batches
    b5 = pkg.isdf_plan_bytes((40, 40, 40), (10, 10, 10), 52, 1040)
    assert b5 > 53e9 + 504 * 1040 * 64000 * 16


def test_create_rejects_invalid_arguments_without_device():
    lib = pkg.load_library()
    h = ctypes.c_void_p()
    lat = np.eye(3) * 6.0
    grid = np.array([16, 16, 16], np.int32)
    km = np.array([1, 1, 1], np.int32)
    orb = np.zeros((1, 2, 4096), np.complex128)
    ip = np.arange(4, dtype=np.int32)
    P = ctypes.c_void_p
    # null output handle / null pointers
    assert lib.isdf_create(None, lat.ctypes.data, grid.ctypes.data, km.ctypes.data, 2,
                           orb.ctypes.data, ip.ctypes.data, 4, 0, None) == -1
    assert lib.isdf_create(ctypes.byref(h), None, grid.ctypes.data, km.ctypes.data, 2,
                           orb.ctypes.data, ip.ctypes.data, 4, 0, None) == -1
    # grid with a prime factor above 7, k mesh too large, bad counts
    bad = np.array([16, 16, 11], np.int32)
    assert lib.isdf_create(ctypes.byref(h), lat.ctypes.data, bad.ctypes.data, km.ctypes.data, 2,
                           orb.ctypes.data, ip.ctypes.data, 4, 0, None) == -1
    bigk = np.array([17, 1, 1], np.int32)
    assert lib.isdf_create(ctypes.byref(h), lat.ctypes.data, grid.ctypes.data, bigk.ctypes.data, 2,
                           orb.ctypes.data, ip.ctypes.data, 4, 0, None) == -1
    assert lib.isdf_create(ctypes.byref(h), lat.ctypes.data, grid.ctypes.data, km.ctypes.data, 0,
                           orb.ctypes.data, ip.ctypes.data, 4, 0, None) == -1
    assert lib.isdf_create(ctypes.byref(h), lat.ctypes.data, grid.ctypes.data, km.ctypes.data, 2,
                           orb.ctypes.data, ip.ctypes.data, 0, 0, None) == -1
    assert h.value is None
    assert b"n_ip" in lib.isdf_last_error(None)


def test_calls_on_null_context_fail_cleanly():
    lib = pkg.load_library()
    assert lib.isdf_fit(None, 0) == -1
    assert lib.isdf_fit(None, 2) == -1
    assert lib.isdf_coulomb_kernel(None, 0) == -1
    assert lib.isdf_destroy(None) == -1
    assert isinstance(lib.isdf_last_error(None), bytes)
    st = ctypes.c_int32()
    assert lib.isdf_poll(None, ctypes.c_uint64(1), ctypes.byref(st), None) == -1
    assert lib.isdf_stage_ms(None, b"chol") == -1.0
    # batch graphs and launch tiling
    h = ctypes.c_void_p()
    nf = (ctypes.c_int32 * 1)(4)
    ptrs = (ctypes.c_void_p * 1)(None)
    assert lib.isdf_graph_create(None, 2, 1, nf, ptrs, ptrs, ctypes.byref(h)) == -1 and not h.value
    assert lib.isdf_graph_launch(None) == -1
    assert lib.isdf_graph_destroy(None) == -1
    assert lib.isdf_autotune(None, 2, 1, nf, ptrs, ptrs, None) == -1
    assert lib.isdf_set_tiling(None, 12, 2) == -1


def test_select_points_rejects_invalid_arguments_without_device():
    lib = pkg.load_library()
    grid = np.array([8, 8, 8], np.int32)
    km = np.array([1, 1, 1], np.int32)
    orb = np.zeros((1, 2, 512), np.complex128)
    ip = np.zeros(4, np.int32)
    assert lib.isdf_select_points(None, km.ctypes.data, 2, orb.ctypes.data, 4, ip.ctypes.data, None, 0,
                                  None) == -1
    assert lib.isdf_select_points(grid.ctypes.data, km.ctypes.data, 2, orb.ctypes.data, 4, None, None, 0,
                                  None) == -1
    assert b"null" in lib.isdf_last_error(None)
    # more points than grid points; bad grid; bad orbital count
    assert lib.isdf_select_points(grid.ctypes.data, km.ctypes.data, 2, orb.ctypes.data, 513,
                                  ip.ctypes.data, None, 0, None) == -1
    assert b"exceeds" in lib.isdf_last_error(None)
    bad = np.array([8, 8, 13], np.int32)
    assert lib.isdf_select_points(bad.ctypes.data, km.ctypes.data, 2, orb.ctypes.data, 4, ip.ctypes.data,
                                  None, 0, None) == -1
    assert lib.isdf_select_points(grid.ctypes.data, km.ctypes.data, 0, orb.ctypes.data, 4, ip.ctypes.data,
                                  None, 0, None) == -1
    with pytest.raises(ValueError):
        pkg.select_points([8, 8, 8], [1, 1, 1], np.zeros((1, 2, 500), np.complex128), 4)
