"""The benchmark workloads as seeded synthetic inputs on the device, and their
algorithmic byte counts.

Input preparation and bookkeeping only: meshes come from ``meshgen``, the
numbering and every assembly run in libexm.

Algorithmic bytes of one column loop = the bytes it must move at least once:
input fields, the output (read and written for INC, written for WRITE), the
z coordinate of every extruded vertex, (x, y) once per base vertex (columns
are vertical), and the explicit lists it reads (field lists and the
coordinate list, int32).  The paper's valuable data volume (input, output and
the full coordinate field, Section 4.2.1) is reported beside it.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass, field

import numpy as np

from . import (CONTINUOUS, EXM_INC, EXM_K_CUBIC, EXM_K_CUBIC_FUSED, EXM_K_MASS, EXM_READ, EXM_WRITE, Mesh, Space,
               coordinate_field, par_loop)
from . import meshgen

_PKG = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    """Hash of the HIP sources and the C header (identifies a kernel build)."""
    h = hashlib.sha256()
    files = sorted(os.path.join(_PKG, "csrc", f) for f in os.listdir(os.path.join(_PKG, "csrc")))
    files.append(os.path.join(os.path.dirname(_PKG), "include", "exm.h"))
    for p in files:
        with open(p, "rb") as fh:
            h.update(os.path.basename(p).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


@dataclass
class Extruded:
    base: meshgen.BaseMesh
    n_layers: int
    mesh: Mesh
    Vx: Space
    X: object                         # device coordinates [3, n]
    spaces: dict = field(default_factory=dict)
    vc: np.ndarray | None = None      # host vertex coordinates [N0, lambda+1, 3]
    layers: np.ndarray | None = None  # layer range of every cell column (meshes with columns of different heights)

    @property
    def n_prisms(self) -> int:
        if self.layers is not None:
            return int((self.layers[:, 1] - self.layers[:, 0]).sum())
        return self.base.n_cells * self.n_layers

    def space(self, name: str) -> Space:
        if name == "P1":
            return self.Vx
        if name not in self.spaces:
            self.spaces[name] = Space(self.mesh, name)
        return self.spaces[name]


def extruded(n: int, n_layers: int, order: str = "rcm", keep_host_coords: bool = False, terrain: float = 0.0,
             layer_kind: str | None = None):
    """n x n triangulated square extruded to n_layers; with ``layer_kind`` the
    cell columns take the layer ranges of meshgen.layer_ranges."""
    base = meshgen.tri_square(n, order=order)
    layers = meshgen.layer_ranges(base, n_layers, layer_kind) if layer_kind else None
    mesh = Mesh(base, n_layers, layers=layers)
    Vx = Space(mesh, "P1")
    vc = meshgen.extruded_vertex_coords(base, n_layers, terrain=terrain)
    X = coordinate_field(Vx, vc)
    return Extruded(base, n_layers, mesh, Vx, X, {}, vc if keep_host_coords else None, layers)


def device_values(n: int, seed: int):
    """n FP64 values U[-1, 1] from numpy's seeded PCG64, on the device."""
    import torch
    return torch.from_numpy(meshgen.uniform_values(n, seed=seed)).to("cuda")


ARITY = {"P1": 6, "DG0": 1, "DG1": 6, "P2": 18, "CG1xDG0": 3, "CG1xDG1": 6, "DG0xCG1": 2, "DG0xDG1": 2,
         "DG1xCG1": 6, "DG1xDG0": 3}


def map_bytes(e: Extruded, name: str) -> int:
    lists = 4 * e.base.n_cells * ARITY[name]
    if name != "P1":
        lists += 4 * e.base.n_cells * 6   # the coordinate list
    return lists


def coord_bytes(e: Extruded) -> int:
    """z at every extruded vertex + (x, y) per base vertex."""
    return 8 * e.Vx.n_dofs + 16 * e.base.n_vertices


def mass_bytes_counts(base, n_layers: int, name: str) -> dict:
    """mass_bytes of a uniform extruded mesh from the entity counts alone
    (n_dofs = sum over d of N_d ((lambda + 1) delta(d, 0) + lambda delta(d, 1)))."""
    from . import DELTA, ELEMENTS
    d = DELTA[ELEMENTS[name]]
    counts = (base.n_vertices, base.n_edges, base.n_cells)
    n = sum(counts[k] * ((n_layers + 1) * d[2 * k] + n_layers * d[2 * k + 1]) for k in range(3))
    nx = base.n_vertices * (n_layers + 1)
    lists = 4 * base.n_cells * ARITY[name] + (4 * base.n_cells * 6 if name != "P1" else 0)
    inc = name in CONTINUOUS
    alg = 8 * n + 8 * n * (2 if inc else 1) + 8 * nx + 16 * base.n_vertices + lists
    return dict(algorithmic=alg, valuable=8 * n * 2 + 24 * nx, n_dofs=n)


def mass_bytes(e: Extruded, name: str) -> dict:
    """Byte counts of one y = M x / residual assembly on space `name`:
    ``algorithmic`` (what the loop must move, with (x, y) once per vertex
    column, since columns are vertical), ``algorithmic_full_coords`` (the
    same with all three coordinate components at every extruded vertex, as
    if the field were read whole), and the paper's ``valuable`` volume."""
    n = e.space(name).n_dofs
    inc = name in CONTINUOUS
    io = 8 * n + 8 * n * (2 if inc else 1) + map_bytes(e, name)
    return dict(algorithmic=io + coord_bytes(e), algorithmic_full_coords=io + 24 * e.Vx.n_dofs,
                valuable=8 * n * 2 + 24 * e.Vx.n_dofs, n_dofs=n)


def cubic_bytes(e: Extruded, fused: bool) -> dict:
    n = e.Vx.n_dofs
    n_in = 3 if fused else 2
    n_out = 3 if fused else 1
    alg = 8 * n * n_in + 16 * n * n_out + coord_bytes(e) + map_bytes(e, "P1")
    valuable = 8 * n * (n_in + n_out) + 24 * n
    return dict(algorithmic=alg, valuable=valuable, n_dofs=n)


# Algorithmic FP64 operations per prism of the cubic forms: the count of a
# sum-factorised evaluation (triangle points times closed-form column
# integrals, the linear terms as the P1 mass action), about 400 per prism for
# the residual and 750 for the fused residual and adjoint.
CUBIC_FLOPS_PER_PRISM = {"forward": 400, "fused": 750}


def cubic_flops(e: Extruded, fused: bool) -> int:
    return CUBIC_FLOPS_PER_PRISM["fused" if fused else "forward"] * e.base.n_cells * e.n_layers


def mass_args(e: Extruded, name: str, x, y):
    acc = EXM_INC if name in CONTINUOUS else EXM_WRITE
    V = e.space(name)
    return [(x, V, EXM_READ), (y, V, acc)]


def run_mass(e: Extruded, name: str, x, y, **opts):
    par_loop(EXM_K_MASS, e.mesh, e.X, e.Vx, mass_args(e, name, x, y), **opts)


def run_cubic(e: Extruded, u, f, F, **opts):
    V = e.Vx
    par_loop(EXM_K_CUBIC, e.mesh, e.X, V, [(u, V, EXM_READ), (f, V, EXM_READ), (F, V, EXM_INC)], **opts)


def run_fused(e: Extruded, u, f, w, F, gu, gf, **opts):
    V = e.Vx
    par_loop(EXM_K_CUBIC_FUSED, e.mesh, e.X, V, [(u, V, EXM_READ), (f, V, EXM_READ), (w, V, EXM_READ),
                                                (F, V, EXM_INC), (gu, V, EXM_INC), (gf, V, EXM_INC)], **opts)
