"""ctypes binding of libexm.so: the C entry points under their own names.

Argument marshalling only: every step of the numbering and of the column
loop runs in the library's HIP kernels.  PyTorch is used by callers for device
memory and streams; this module passes raw pointers and stream handles.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexm.so")

# constants mirrored from include/exm.h
EXM_OK = 0
EXM_EINVAL = -1
EXM_ERANGE = -2
EXM_EOVERFLOW = -3
EXM_ENOMEM = -4
EXM_EHIP = -5
EXM_EUNSUPPORTED = -6

EXM_ELEMENT_NONE = 0
EXM_ELEMENT_P1P1 = 1
EXM_ELEMENT_DG0DG0 = 2
EXM_ELEMENT_DG1DG1 = 3
EXM_ELEMENT_P2P2 = 4
EXM_ELEMENT_P1DG0 = 5
EXM_ELEMENT_P1DG1 = 6
EXM_ELEMENT_DG0P1 = 7
EXM_ELEMENT_DG0DG1 = 8
EXM_ELEMENT_DG1P1 = 9
EXM_ELEMENT_DG1DG0 = 10
EXM_ELEMENT_DGMIX = 11

EXM_READ = 1
EXM_WRITE = 2
EXM_INC = 3

EXM_K_MASS = 1
EXM_K_CUBIC = 2
EXM_K_CUBIC_VJP = 3
EXM_K_CUBIC_FUSED = 4
EXM_K_CUBIC_JAC = 5
EXM_K_FACET_JUMP = 6

EXM_RACE_AUTO = 0
EXM_RACE_ATOMIC = 1
EXM_RACE_COLOUR = 2
EXM_RACE_OWNER = 3

EXM_SCHED_AUTO = 0
EXM_SCHED_DIRECT = 1
EXM_SCHED_TILED = 2
EXM_SCHED_STAGED = 3
EXM_SCHED_PIPELINED = 4
EXM_SCHED_CHUNKED = 5
EXM_SCHED_GATHER = 6

STATUS_NAMES = {0: "EXM_OK", -1: "EXM_EINVAL", -2: "EXM_ERANGE", -3: "EXM_EOVERFLOW", -4: "EXM_ENOMEM",
                -5: "EXM_EHIP", -6: "EXM_EUNSUPPORTED"}


class ExmError(RuntimeError):
    def __init__(self, status: int, message: str, func: str):
        self.status = status
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {message}")


class exm_arg(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("space", c_void_p), ("dim", c_int32), ("access", c_int32)]


class exm_loop_opts(ctypes.Structure):
    _fields_ = [("race", c_int32), ("schedule", c_int32), ("cols_per_wave", c_int32), ("waves_per_block", c_int32),
                ("tile_cells", c_int32), ("chunk_layers", c_int32)]


class exm_batch_item(ctypes.Structure):
    _fields_ = [("space", c_void_p), ("coord_space", c_void_p), ("coords", c_void_p), ("n_fields", c_int32),
                ("f", POINTER(c_void_p)), ("b", POINTER(c_void_p)), ("w", POINTER(c_void_p)),
                ("g", POINTER(c_void_p))]


EXM_PLAN_CELL_COLOURS = 1
EXM_PLAN_TILES = 2
EXM_PLAN_OWNER = 3


class exm_plan_info(ctypes.Structure):
    _fields_ = [("n_units", c_int32), ("n_colours", c_int32), ("n_cell_entries", c_int64),
                ("n_vert_entries", c_int64), ("n_edge_entries", c_int64)]


class exm_plan_arrays(ctypes.Structure):
    _fields_ = [(n, c_void_p) for n in ("colour", "cell_off", "cells", "vert_off", "verts", "owned", "edge_off",
                                        "edges", "local_cv", "local_ce")]


# name -> (restype, argtypes); status-returning functions raise ExmError
_PROTOS = {
    "exm_last_error": (c_char_p, []),
    "exm_abi_version": (c_int32, []),
    "exm_sync": (c_int32, [c_void_p]),
    "exm_mesh_create": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int32, POINTER(c_void_p)]),
    "exm_mesh_create_var": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                      POINTER(c_void_p)]),
    "exm_mesh_create_device": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                         POINTER(c_void_p)]),
    "exm_mesh_entity_layers": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "exm_mesh_destroy": (None, [c_void_p]),
    "exm_space_create": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, POINTER(c_void_p)]),
    "exm_space_info": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int32)]),
    "exm_space_offsets": (c_int32, [c_void_p, c_void_p]),
    "exm_space_column_starts": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "exm_space_bottom_map": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "exm_space_destroy": (None, [c_void_p]),
    "exm_space_coordinates": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "exm_coordinates_verify": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "exm_par_loop": (c_int32, [c_int32, c_void_p, c_int32, POINTER(exm_arg), POINTER(exm_loop_opts), c_void_p]),
    "exm_par_loop_config": (c_int32, [c_int32, c_void_p, c_int32, POINTER(exm_arg), POINTER(exm_loop_opts),
                                      POINTER(exm_loop_opts)]),
    "exm_mesh_colours": (c_int32, [c_void_p, POINTER(c_int32)]),
    "exm_mesh_plan_info": (c_int32, [c_void_p, c_int32, c_int32, POINTER(exm_plan_info)]),
    "exm_mesh_plan_read": (c_int32, [c_void_p, c_int32, c_int32, POINTER(exm_plan_arrays)]),
    "exm_autotune": (c_int32, [c_int32, c_void_p, c_int32, POINTER(exm_arg), c_void_p, POINTER(exm_loop_opts)]),
    "exm_autotune_save": (c_int32, [c_char_p]),
    "exm_autotune_load": (c_int32, [c_char_p]),
    "exm_batch_create": (c_int32, [c_int32, POINTER(exm_batch_item), POINTER(exm_loop_opts), c_void_p,
                                   POINTER(c_void_p)]),
    "exm_batch_launch": (c_int32, [c_void_p, c_void_p]),
    "exm_batch_info": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int32)]),
    "exm_batch_tiles": (c_int32, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "exm_batch_destroy": (None, [c_void_p]),
    "exm_space_create_mixed": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                         POINTER(c_void_p)]),
    "exm_space_list_size": (c_int32, [c_void_p, POINTER(c_int64)]),
    "exm_space_lists": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "exm_matrix_create": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "exm_matrix_info": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]),
    "exm_matrix_assemble": (c_int32, [c_int32, c_void_p, c_int32, c_void_p, c_void_p]),
    "exm_matrix_spmv": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "exm_matrix_csr": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "exm_matrix_csr_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "exm_matrix_destroy": (None, [c_void_p]),
    "exm_stream_triad": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_int64, c_int32, c_int32, c_void_p]),
}

EXPORTED = tuple(_PROTOS)

_lib = None


def load(path: str = LIB_PATH):
    """Load libexm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libexm.so not found at {path}: build it with `python -m paper_1604_05937_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().exm_last_error().decode()


def call(name: str, *args) -> int:
    """Call a status-returning entry point; raise ExmError on a negative status."""
    st = getattr(load(), name)(*args)
    if st != EXM_OK:
        raise ExmError(st, last_error(), name)
    return st


def _mk(name):
    def f(*args):
        fn = getattr(load(), name)
        if fn.restype is c_int32 and name not in ("exm_abi_version",):
            st = fn(*args)
            if st != EXM_OK:
                raise ExmError(st, last_error(), name)
            return st
        return fn(*args)
    f.__name__ = name
    return f


# thin wrappers under the C names
for _n in _PROTOS:
    globals()[_n] = _mk(_n)
