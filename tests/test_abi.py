"""The C ABI: the built library exports every entry point include/exm.h
declares, and host-side validation rejects bad input before any device work
(these calls never reach the GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1604_05937_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "exm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(exm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert set(_declared()) == set(_abi.EXPORTED)


def test_library_exports_every_symbol():
    lib = _abi.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.exm_abi_version() == 1


def test_mesh_validation_errors():
    lib = _abi.load()
    h = ctypes.c_void_p()
    cv = np.array([[0, 1, 2], [0, 2, 5]], dtype=np.int32)   # vertex 5 out of range for 4 vertices
    st = lib.exm_mesh_create(4, 0, 2, cv.ctypes.data_as(ctypes.c_void_p), None, 3, ctypes.byref(h))
    assert st == _abi.EXM_ERANGE and "outside" in _abi.last_error()
    cv = np.array([[0, 1, 2]], dtype=np.int32)
    assert lib.exm_mesh_create(3, 0, 1, cv.ctypes.data_as(ctypes.c_void_p), None, 0, ctypes.byref(h)) == _abi.EXM_ERANGE
    cv = np.array([[0, 1, 1]], dtype=np.int32)
    assert lib.exm_mesh_create(3, 0, 1, cv.ctypes.data_as(ctypes.c_void_p), None, 2, ctypes.byref(h)) == _abi.EXM_EINVAL
    assert lib.exm_mesh_create(3, 0, 1, None, None, 2, ctypes.byref(h)) == _abi.EXM_EINVAL
    assert lib.exm_space_create(None, None, 0, None, ctypes.byref(h)) == _abi.EXM_EINVAL
    assert lib.exm_par_loop(99, None, 0, None, None, None) == _abi.EXM_EINVAL
    assert lib.exm_stream_triad(None, None, None, 1.0, 10, 256, 0, None) == _abi.EXM_EINVAL
    assert lib.exm_batch_create(0, None, None, None, ctypes.byref(h)) == _abi.EXM_EINVAL
    assert lib.exm_batch_tiles(None, _abi.EXM_ELEMENT_P1P1, None, None) == _abi.EXM_EINVAL


def test_python_wrappers_raise():
    with pytest.raises(_abi.ExmError) as e:
        _abi.exm_par_loop(99, None, 0, None, None, None)
    assert e.value.status == _abi.EXM_EINVAL


def test_new_entry_points_validate_on_the_host():
    lib = _abi.load()
    h = ctypes.c_void_p()
    cv = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    # layer ranges: empty, reversed and beyond n_layers are refused before any device work
    for bad in ([[0, 0], [0, 3]], [[2, 1], [0, 3]], [[0, 4], [0, 3]], [[-1, 2], [0, 3]]):
        lay = np.array(bad, dtype=np.int32)
        st = lib.exm_mesh_create_var(4, 0, 2, cv.ctypes.data_as(ctypes.c_void_p), None, 3,
                                     lay.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
        assert st == _abi.EXM_ERANGE, (bad, st)
    assert lib.exm_mesh_create_var(4, 0, 2, cv.ctypes.data_as(ctypes.c_void_p), None, 3, None,
                                   ctypes.byref(h)) == _abi.EXM_EINVAL
    assert lib.exm_mesh_entity_layers(None, 0, None, None) == _abi.EXM_EINVAL
    assert lib.exm_matrix_create(None, ctypes.byref(h)) == _abi.EXM_EINVAL
    assert lib.exm_matrix_info(None, None, None, None, None) == _abi.EXM_EINVAL
    assert lib.exm_matrix_assemble(_abi.EXM_K_MASS, None, 0, None, None) == _abi.EXM_EINVAL
    assert lib.exm_matrix_spmv(None, None, None, _abi.EXM_WRITE, None) == _abi.EXM_EINVAL
    assert lib.exm_matrix_csr(None, None, None, None, None) == _abi.EXM_EINVAL
    # the Jacobian and the facet loop are kernels of their own entry points only
    assert lib.exm_par_loop(_abi.EXM_K_CUBIC_JAC, None, 0, None, None, None) == _abi.EXM_EINVAL
    assert lib.exm_par_loop(_abi.EXM_K_FACET_JUMP, None, 0, None, None, None) == _abi.EXM_EINVAL


def test_stored_launch_table_loads(tmp_path):
    # the shipped table of tuned launches parses and passes the loader's range
    # checks; a line with a chunk length no schedule takes is refused
    lib = _abi.load()
    table = os.path.join(ROOT, "paper_1604_05937_amd", "tuned_mi355x.txt")
    assert lib.exm_autotune_load(table.encode()) == _abi.EXM_OK, _abi.last_error()
    bad = tmp_path / "bad.txt"
    bad.write_text("# kernel element n_layers log2_cells race schedule cpw wpb tile_cells chunk_layers\n"
                   "1 2 100 19 1 4 0 4 30 33\n")
    assert lib.exm_autotune_load(str(bad).encode()) == _abi.EXM_ERANGE
    assert "out of range" in _abi.last_error()
    bad.write_text("1 2 100 19 1 4 0 4 30\n")
    assert lib.exm_autotune_load(str(bad).encode()) == _abi.EXM_EINVAL


def test_edge_convention_is_checked():
    # two triangles sharing the edge (1, 2); edge a of a cell joins its
    # vertices (a+1)%3 and (a+2)%3.  A consistent map is [[0, 1, 2], [3, 4, 0]]
    # (it reaches the device upload, so it is exercised by the GPU tests).
    lib = _abi.load()
    h = ctypes.c_void_p()
    cv = np.array([[0, 1, 2], [2, 1, 3]], dtype=np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    # cell 1 names edge 1 (0-2 in cell 0) for its edge joining 2 and 1
    ce = np.array([[0, 1, 2], [3, 4, 1]], dtype=np.int32)
    assert lib.exm_mesh_create(4, 5, 2, ptr(cv), ptr(ce), 3, ctypes.byref(h)) == _abi.EXM_EINVAL
    assert "joins vertices" in _abi.last_error() and "earlier cell" in _abi.last_error()
    # a sixth edge joining 1 and 2 again: the shared edge would get two columns
    ce = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    assert lib.exm_mesh_create(4, 6, 2, ptr(cv), ptr(ce), 3, ctypes.byref(h)) == _abi.EXM_EINVAL
    assert "two edges join vertices 1 and 2" in _abi.last_error()
    # an edge index out of range is a range error, as before
    ce = np.array([[0, 1, 2], [3, 4, 7]], dtype=np.int32)
    assert lib.exm_mesh_create(4, 5, 2, ptr(cv), ptr(ce), 3, ctypes.byref(h)) == _abi.EXM_ERANGE
    # the same checks on the variable-height entry point
    lay = np.array([[0, 3], [1, 3]], dtype=np.int32)
    ce = np.array([[0, 1, 2], [3, 4, 1]], dtype=np.int32)
    assert lib.exm_mesh_create_var(4, 5, 2, ptr(cv), ptr(ce), 3, ptr(lay), ctypes.byref(h)) == _abi.EXM_EINVAL
