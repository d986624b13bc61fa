"""exm: extruded-mesh numbering and column iteration on AMD MI355X.

Python face of libexm.so (hand-written HIP for gfx950).  The classes here hold
library handles and marshal torch tensors (device memory) and torch streams
into the C ABI; all numbering and assembly work runs in the library.  There is
no CPU fallback: without the built library every call raises.

Method: Bercea et al., arXiv 1604.05937 -- vertical-innermost numbering
(Algorithm 1), vertical offsets (Algorithm 2), column iteration by direct
addressing (Algorithm 3).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import (EXM_ELEMENT_DG0DG0, EXM_ELEMENT_DG1DG1, EXM_ELEMENT_DGMIX, EXM_ELEMENT_NONE, EXM_ELEMENT_P1P1, EXM_ELEMENT_P2P2,
                   EXM_INC, EXM_K_CUBIC, EXM_K_CUBIC_FUSED, EXM_K_CUBIC_JAC, EXM_K_CUBIC_VJP, EXM_K_FACET_JUMP,
                   EXM_K_MASS,
                   EXM_RACE_ATOMIC,
                   EXM_RACE_AUTO, EXM_RACE_COLOUR, EXM_RACE_OWNER, EXM_READ, EXM_SCHED_AUTO, EXM_SCHED_CHUNKED, EXM_SCHED_DIRECT, EXM_SCHED_GATHER, EXM_SCHED_PIPELINED,
                   EXM_SCHED_STAGED, EXM_SCHED_TILED, EXM_WRITE, ExmError)

__all__ = ["Mesh", "Space", "Matrix", "par_loop", "ExmError", "ELEMENTS", "DELTA", "load_library", "stream_handle"]

# delta((d1, d2)) tables, flattened as d1 * 2 + d2 (Section 3.2)
DELTA = {
    _abi.EXM_ELEMENT_P1DG0: (0, 1, 0, 0, 0, 0),
    _abi.EXM_ELEMENT_P1DG1: (0, 2, 0, 0, 0, 0),
    _abi.EXM_ELEMENT_DG0P1: (0, 0, 0, 0, 1, 0),
    _abi.EXM_ELEMENT_DG0DG1: (0, 0, 0, 0, 0, 2),
    _abi.EXM_ELEMENT_DG1P1: (0, 0, 0, 0, 3, 0),
    _abi.EXM_ELEMENT_DG1DG0: (0, 0, 0, 0, 0, 3),
    EXM_ELEMENT_P1P1: (1, 0, 0, 0, 0, 0),
    EXM_ELEMENT_DG0DG0: (0, 0, 0, 0, 0, 1),
    EXM_ELEMENT_DG1DG1: (0, 0, 0, 0, 0, 6),
    EXM_ELEMENT_P2P2: (1, 1, 1, 1, 0, 0),
}
ELEMENTS = {"P1": EXM_ELEMENT_P1P1, "DG0": EXM_ELEMENT_DG0DG0, "DG1": EXM_ELEMENT_DG1DG1, "P2": EXM_ELEMENT_P2P2,
            # the other horizontal x vertical products of {CG1, DG0, DG1}
            "CG1xDG0": _abi.EXM_ELEMENT_P1DG0, "CG1xDG1": _abi.EXM_ELEMENT_P1DG1,
            "DG0xCG1": _abi.EXM_ELEMENT_DG0P1, "DG0xDG1": _abi.EXM_ELEMENT_DG0DG1,
            "DG1xCG1": _abi.EXM_ELEMENT_DG1P1, "DG1xDG0": _abi.EXM_ELEMENT_DG1DG0}

# spaces whose DoFs are shared between cells or layers (outputs must be INC)
CONTINUOUS = {"P1", "P2", "CG1xDG0", "CG1xDG1", "DG0xCG1", "DG1xCG1"}


def load_library():
    return _abi.load()


def stream_handle(stream=None) -> int | None:
    """Raw HIP stream handle of a torch stream (default: the current stream)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


class Mesh:
    """An extruded mesh: triangular base mesh (cell->vertex, cell->edge) and
    a layer count, or a layer range per cell column (``layers`` [N2, 2]: the
    prisms of layers layers[c, 0] .. layers[c, 1] - 1).  Wraps exm_mesh."""

    def __init__(self, base, n_layers: int, layers=None):
        _abi.load()
        self.base = base
        self.n_layers = int(n_layers)
        self.layers = None if layers is None else _i32(layers).reshape(-1, 2)
        cv = _i32(base.cell_vertex)
        ce = _i32(base.cell_edge) if getattr(base, "cell_edge", None) is not None else None
        h = ctypes.c_void_p()
        args = (int(base.n_vertices), int(base.n_edges), int(base.n_cells), cv.ctypes.data_as(ctypes.c_void_p),
                None if ce is None else ce.ctypes.data_as(ctypes.c_void_p), self.n_layers)
        if self.layers is None:
            _abi.exm_mesh_create(*args, ctypes.byref(h))
        else:
            _abi.exm_mesh_create_var(*args, self.layers.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
        self.handle = h

    @classmethod
    def from_device(cls, base, n_layers: int, cell_vertex, cell_edge=None, layers=None):
        """The same mesh from device-resident int32 adjacency tensors
        (exm_mesh_create_device); `base` supplies the entity counts."""
        import torch
        _abi.load()
        self = cls.__new__(cls)
        self.base = base
        self.n_layers = int(n_layers)
        for t in (cell_vertex, cell_edge, layers):
            assert t is None or (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous())
        self.layers = None if layers is None else layers.cpu().numpy().reshape(-1, 2)
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        h = ctypes.c_void_p()
        _abi.exm_mesh_create_device(int(base.n_vertices), int(base.n_edges), int(base.n_cells), ptr(cell_vertex),
                                    ptr(cell_edge), self.n_layers, ptr(layers), ctypes.byref(h))
        self.handle = h
        return self

    def entity_layers(self, d1: int):
        """Layer range (lo, hi) of the column of every base entity of dimension d1."""
        n = int(self.base.counts[d1])
        lo = np.zeros(n, dtype=np.int32)
        hi = np.zeros(n, dtype=np.int32)
        _abi.exm_mesh_entity_layers(self.handle, d1, lo.ctypes.data_as(ctypes.c_void_p),
                                    hi.ctypes.data_as(ctypes.c_void_p))
        return lo, hi

    @property
    def n_cells(self) -> int:
        return int(self.base.n_cells)

    def colours(self) -> int:
        n = ctypes.c_int32()
        _abi.exm_mesh_colours(self.handle, ctypes.byref(n))
        return n.value

    def plan(self, kind: str, target: int = 0) -> dict:
        """A race-resolution plan as host arrays (exm_mesh_plan_read): kind
        "colours" (base cells), "tiles" or "owner" (tiles of about `target`
        cells)."""
        k = {"colours": _abi.EXM_PLAN_CELL_COLOURS, "tiles": _abi.EXM_PLAN_TILES, "owner": _abi.EXM_PLAN_OWNER}[kind]
        info = _abi.exm_plan_info()
        _abi.exm_mesh_plan_info(self.handle, k, int(target), ctypes.byref(info))
        nu = info.n_units
        edges = info.n_edge_entries > 0
        out = {"n_colours": info.n_colours,
               "colour": np.zeros(nu, np.int32), "cell_off": np.zeros(nu + 1, np.int32),
               "cells": np.zeros(info.n_cell_entries, np.int32), "vert_off": np.zeros(nu + 1, np.int32),
               "verts": np.zeros(info.n_vert_entries, np.int32), "owned": np.zeros(nu, np.int32),
               "local_cv": np.zeros(info.n_cell_entries * 3, np.uint16)}
        if edges:
            out.update(edge_off=np.zeros(nu + 1, np.int32), edges=np.zeros(info.n_edge_entries, np.int32),
                       local_ce=np.zeros(info.n_cell_entries * 3, np.uint16))
        arr = _abi.exm_plan_arrays(*[out[n].ctypes.data if n in out else None
                                     for n, _ in _abi.exm_plan_arrays._fields_])
        _abi.exm_mesh_plan_read(self.handle, k, int(target), ctypes.byref(arr))
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _abi is not None and _abi._lib is not None:
            _abi._lib.exm_mesh_destroy(h)
        self.handle = None


class Space:
    """A function space on an extruded mesh (numbering of Algorithm 1, lists
    and offsets of Algorithm 2).  Wraps exm_space; built on the device."""

    def __init__(self, mesh: Mesh, element, delta=None, stream=None):
        if isinstance(element, str):
            element = ELEMENTS[element]
        self.mesh = mesh
        self.element = element
        d = np.asarray(delta if delta is not None else DELTA[element], dtype=np.int32).reshape(6)
        self.delta = d
        h = ctypes.c_void_p()
        _abi.exm_space_create(mesh.handle, d.ctypes.data_as(ctypes.c_void_p), int(element),
                              stream_handle(stream), ctypes.byref(h))
        self.handle = h
        n = ctypes.c_int64()
        k = ctypes.c_int32()
        _abi.exm_space_info(h, ctypes.byref(n), ctypes.byref(k))
        self.n_dofs = n.value
        self.arity = k.value

    @classmethod
    def mixed(cls, mesh: Mesh, dofs, element: int = EXM_ELEMENT_NONE, stream=None):
        """A space with a DoF count per entity: dofs[d] is [N_d, 2] (DoFs on
        every horizontal and vertical entity of each base entity of dimension
        d), or None for none."""
        self = cls.__new__(cls)
        self.mesh = mesh
        self.element = element
        self.delta = None
        arrs = [None if d is None else np.ascontiguousarray(np.asarray(d, dtype=np.int32).reshape(-1, 2))
                for d in dofs]
        ptrs = [None if a is None else a.ctypes.data_as(ctypes.c_void_p) for a in arrs]
        h = ctypes.c_void_p()
        _abi.exm_space_create_mixed(mesh.handle, ptrs[0], ptrs[1], ptrs[2], int(element), stream_handle(stream),
                                    ctypes.byref(h))
        self.handle = h
        n = ctypes.c_int64()
        k = ctypes.c_int32()
        _abi.exm_space_info(h, ctypes.byref(n), ctypes.byref(k))
        self.n_dofs = n.value
        self.arity = k.value
        return self

    def lists(self, stream=None):
        """(list_off [n_cells + 1], lists [total], entry_offsets [total]), int32 device tensors."""
        import torch
        total = ctypes.c_int64()
        _abi.exm_space_list_size(self.handle, ctypes.byref(total))
        off = torch.empty(self.mesh.n_cells + 1, dtype=torch.int32, device="cuda")
        lst = torch.empty(max(total.value, 1), dtype=torch.int32, device="cuda")
        eo = torch.empty(max(total.value, 1), dtype=torch.int32, device="cuda")
        _abi.exm_space_lists(self.handle, ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(lst.data_ptr()),
                             ctypes.c_void_p(eo.data_ptr()), stream_handle(stream))
        return off, lst[:total.value], eo[:total.value]

    def offsets(self) -> np.ndarray:
        out = np.zeros(self.arity, dtype=np.int32)
        _abi.exm_space_offsets(self.handle, out.ctypes.data_as(ctypes.c_void_p))
        return out

    def column_starts(self, d1: int, stream=None):
        import torch
        n = [self.mesh.base.n_vertices, self.mesh.base.n_edges, self.mesh.base.n_cells][d1]
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        _abi.exm_space_column_starts(self.handle, d1, ctypes.c_void_p(out.data_ptr()), stream_handle(stream))
        return out

    def bottom_map(self, stream=None):
        import torch
        out = torch.empty((self.mesh.n_cells, self.arity), dtype=torch.int32, device="cuda")
        _abi.exm_space_bottom_map(self.handle, ctypes.c_void_p(out.data_ptr()), stream_handle(stream))
        return out

    def zeros(self, dim: int = 1):
        import torch
        shape = (self.n_dofs,) if dim == 1 else (self.n_dofs, dim)
        return torch.zeros(shape, dtype=torch.float64, device="cuda")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _abi is not None and _abi._lib is not None:
            _abi._lib.exm_space_destroy(h)
        self.handle = None


def coordinate_field(space: Space, vertex_coords, stream=None):
    """Coordinate field (FP64, device, component-major [3, n_dofs]) of a P1 x P1
    space from per-vertex, per-level coordinates [N0, lambda+1, 3] (a numpy
    array or a device tensor), placed by the library (exm_space_coordinates),
    which refuses columns whose x or y changes with the level."""
    import torch
    out = torch.empty(3 * space.n_dofs, dtype=torch.float64, device="cuda")
    if isinstance(vertex_coords, torch.Tensor):
        src = vertex_coords.detach().to(dtype=torch.float64).contiguous()
        assert src.is_cuda and src.numel() == space.mesh.base.n_vertices * (space.mesh.n_layers + 1) * 3
        _abi.exm_space_coordinates(space.handle, ctypes.c_void_p(src.data_ptr()), 1, ctypes.c_void_p(out.data_ptr()),
                                   stream_handle(stream))
    else:
        src = np.ascontiguousarray(vertex_coords, dtype=np.float64)
        assert src.size == space.mesh.base.n_vertices * (space.mesh.n_layers + 1) * 3
        _abi.exm_space_coordinates(space.handle, src.ctypes.data_as(ctypes.c_void_p), 0,
                                   ctypes.c_void_p(out.data_ptr()), stream_handle(stream))
    return out.view(3, space.n_dofs)


def verify_coordinates(space: Space, X, stream=None):
    """Check a coordinate field for vertical columns (exm_coordinates_verify)."""
    _abi.exm_coordinates_verify(space.handle, ctypes.c_void_p(X.data_ptr()), stream_handle(stream))


def _arg(t, space: Space, access: int, dim: int = 1) -> _abi.exm_arg:
    import torch
    assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous(), "fields are contiguous FP64 device tensors"
    assert t.numel() == space.n_dofs * dim, "field size does not match its space"
    return _abi.exm_arg(ctypes.c_void_p(t.data_ptr()), space.handle, dim, access)


def make_args(coords, coord_space: Space, fields):
    """exm_arg array: coordinates first, then (tensor, space, access) triples."""
    arr = (_abi.exm_arg * (1 + len(fields)))()
    arr[0] = _arg(coords, coord_space, EXM_READ, 3)
    for i, (t, sp, acc) in enumerate(fields):
        arr[1 + i] = _arg(t, sp, acc)
    return arr


OPT_FIELDS = ("race", "schedule", "cols_per_wave", "waves_per_block", "tile_cells", "chunk_layers")


def loop_opts(race: int = 0, schedule: int = 0, cols_per_wave: int = 0, waves_per_block: int = 0,
              tile_cells: int = 0, chunk_layers: int = 0):
    return _abi.exm_loop_opts(race, schedule, cols_per_wave, waves_per_block, tile_cells, chunk_layers)


def _opts_dict(o) -> dict:
    return {k: getattr(o, k) for k in OPT_FIELDS}


def par_loop(kernel: int, mesh: Mesh, coords, coord_space: Space, fields, stream=None, **opts):
    """exm_par_loop on the current torch stream (opts: exm_loop_opts fields)."""
    args = make_args(coords, coord_space, fields)
    o = loop_opts(**opts)
    _abi.exm_par_loop(kernel, mesh.handle, len(args), args, ctypes.byref(o), stream_handle(stream))


def par_loop_config(kernel: int, mesh: Mesh, coords, coord_space: Space, fields, **opts) -> dict:
    """The launch configuration exm_par_loop would use."""
    args = make_args(coords, coord_space, fields)
    o = loop_opts(**opts)
    ch = _abi.exm_loop_opts()
    _abi.exm_par_loop_config(kernel, mesh.handle, len(args), args, ctypes.byref(o), ctypes.byref(ch))
    return _opts_dict(ch)


def autotune(kernel: int, mesh: Mesh, coords, coord_space: Space, fields, stream=None) -> dict:
    args = make_args(coords, coord_space, fields)
    best = _abi.exm_loop_opts()
    _abi.exm_autotune(kernel, mesh.handle, len(args), args, stream_handle(stream), ctypes.byref(best))
    return _opts_dict(best)


def autotune_save(path: str):
    """Write the launches the autotuner has chosen (a text table)."""
    _abi.exm_autotune_save(path.encode())


def autotune_load(path: str):
    """Read a table written by autotune_save: loops without explicit options
    take its launches."""
    _abi.exm_autotune_load(path.encode())


def sync(stream=None):
    _abi.exm_sync(stream_handle(stream))


def stream_triad(a, b, c, alpha: float, block: int = 256, grid: int = 0, stream=None):
    _abi.exm_stream_triad(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                          float(alpha), a.numel(), block, grid, stream_handle(stream))


class Matrix:
    """exm_matrix: the matrix of a bilinear form on one space in the
    vertically aligned layout (classes of DoFs at a fixed stride, a pattern
    over base entities, three values per slot), assembled, applied and
    exported to CSR on the device."""

    def __init__(self, space: Space):
        self.space = space
        h = ctypes.c_void_p()
        _abi.exm_matrix_create(space.handle, ctypes.byref(h))
        self.handle = h
        n, nnz, npat, nst = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _abi.exm_matrix_info(h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(npat), ctypes.byref(nst))
        self.n_rows, self.nnz, self.n_pattern, self.n_stored = n.value, nnz.value, npat.value, nst.value

    def assemble(self, kernel: int, coords, coord_space: Space, u=None, stream=None):
        """Overwrite the values with the matrix of EXM_K_MASS (no field) or
        EXM_K_CUBIC_JAC (the Jacobian at u)."""
        fields = [] if u is None else [(u, self.space, EXM_READ)]
        args = make_args(coords, coord_space, fields)
        _abi.exm_matrix_assemble(kernel, self.handle, len(args), args, stream_handle(stream))

    def spmv(self, x, y=None, access: int = EXM_WRITE, stream=None):
        import torch
        assert x.dtype == torch.float64 and x.is_cuda and x.is_contiguous() and x.numel() == self.n_rows
        if y is None:
            y = torch.empty_like(x)
        assert y.dtype == torch.float64 and y.is_cuda and y.is_contiguous() and y.numel() == self.n_rows
        _abi.exm_matrix_spmv(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), access,
                             stream_handle(stream))
        return y

    def csr(self, stream=None):
        """(rowptr int64 [n + 1], col int32 [nnz], val float64 [nnz]) on the device."""
        import torch
        rowptr = torch.empty(self.n_rows + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(self.nnz, 1), dtype=torch.float64, device="cuda")
        _abi.exm_matrix_csr(self.handle, ctypes.c_void_p(rowptr.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                            ctypes.c_void_p(val.data_ptr()), stream_handle(stream))
        return rowptr, col[:self.nnz], val[:self.nnz]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _abi is not None and _abi._lib is not None:
            _abi._lib.exm_matrix_destroy(h)
        self.handle = None


class Batch:
    """exm_batch: forward residual b = M f and adjoint g = M w for several
    fields on many extruded meshes, one launch per kind of item (P1, DG0) in
    a HIP graph.

    items: list of dicts with keys space, coord_space, coords, f, b and
    optionally w, g (lists of device FP64 tensors on `space`)."""

    def __init__(self, items, cols_per_wave: int = 0, unit_cells: int = 0, schedule: int = 0,
                 chunk_layers: int = 0, race: int = 0, stream=None):
        _abi.load()
        self._keep = []
        arr = (_abi.exm_batch_item * len(items))()
        for i, it in enumerate(items):
            nf = len(it["f"])
            ptr_arrays = []
            for key in ("f", "b", "w", "g"):
                ts = it.get(key)
                if ts is None:
                    ptr_arrays.append(None)
                    continue
                assert len(ts) == nf
                for t in ts:
                    assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous()
                    assert t.numel() == it["space"].n_dofs
                pa = (ctypes.c_void_p * nf)(*[t.data_ptr() for t in ts])
                ptr_arrays.append(pa)
                self._keep.append(pa)
            f, b, w, g = ptr_arrays
            P = ctypes.POINTER(ctypes.c_void_p)
            arr[i] = _abi.exm_batch_item(it["space"].handle, it["coord_space"].handle,
                                         ctypes.c_void_p(it["coords"].data_ptr()), nf,
                                         ctypes.cast(f, P), ctypes.cast(b, P),
                                         ctypes.cast(w, P) if w is not None else None,
                                         ctypes.cast(g, P) if g is not None else None)
        self._keep.append(arr)
        self.items = items
        opts = loop_opts(cols_per_wave=cols_per_wave, tile_cells=unit_cells, schedule=schedule,
                         chunk_layers=chunk_layers, race=race)
        h = ctypes.c_void_p()
        _abi.exm_batch_create(len(items), arr, ctypes.byref(opts), stream_handle(stream), ctypes.byref(h))
        self.handle = h

    def launch(self, stream=None):
        _abi.exm_batch_launch(self.handle, stream_handle(stream))

    def info(self):
        n = ctypes.c_int64()
        b = ctypes.c_int32()
        _abi.exm_batch_info(self.handle, ctypes.byref(n), ctypes.byref(b))
        return n.value, b.value

    def tiles(self, name: str):
        """(tile_cells, chunk_layers) of the tiles of the "P1" or "DG0" items;
        (0, 0) when that kind runs on work units."""
        t = ctypes.c_int32()
        c = ctypes.c_int32()
        el = {"P1": EXM_ELEMENT_P1P1, "DG0": EXM_ELEMENT_DG0DG0}[name]
        _abi.exm_batch_tiles(self.handle, el, ctypes.byref(t), ctypes.byref(c))
        return t.value, c.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _abi is not None and _abi._lib is not None:
            _abi._lib.exm_batch_destroy(h)
        self.handle = None
