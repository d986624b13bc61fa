"""Seeded synthetic inputs: triangulated base meshes, their orderings, extruded
vertex coordinates and field values.

This module holds input preparation only.  It contains none of the numbering,
iteration or element arithmetic of the method, and it is the only module that
both the HIP path and the CPU oracle are fed from.

Base mesh conventions (the paper's base mesh is an unstructured 2D mesh given
by explicit adjacency lists, Section 2.2; its cell-to-vertex relation is the
one from which the others are derived):

* vertices, edges and triangles are numbered 0..N_d-1;
* ``cell_vertex[c] = (v0, v1, v2)`` is counter-clockwise;
* ``cell_edge[c, a]`` is the edge opposite local vertex ``a``, i.e. the edge
  joining ``cell_vertex[c, (a+1)%3]`` and ``cell_vertex[c, (a+2)%3]``;
* edges are listed sorted by (min vertex, max vertex) after the vertices have
  been renumbered.

The workloads stand in for the paper's Gmsh unit-cube meshes (Section 4.1.1),
which are not available: a unit square cut into n x n quads, each split along
the (i,j)-(i+1,j+1) diagonal, interior vertices jittered by U[-0.2h, 0.2h]
in x and y, reordered by reverse Cuthill-McKee or by a seeded random
permutation (Section 4.1.4).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

# Seeds used across tests and benchmarks.
SEED_MESH = 0      # vertex jitter
SEED_FIELD = 1     # field values
SEED_ORDER = 2     # random base ordering
SEED_COTAN = 3     # cotangents / adjoint seeds
SEED_BATCH = 4     # batch sizes and types


@dataclass
class BaseMesh:
    """A 2D triangular base mesh with explicit adjacency lists."""

    xy: np.ndarray            # [N0, 2] float64 vertex coordinates
    cell_vertex: np.ndarray   # [N2, 3] int32, counter-clockwise
    cell_edge: np.ndarray     # [N2, 3] int32, edge a opposite vertex a
    edge_vertex: np.ndarray   # [N1, 2] int32, sorted pair
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edge_vertex.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cell_vertex.shape[0])

    @property
    def counts(self) -> tuple[int, int, int]:
        return (self.n_vertices, self.n_edges, self.n_cells)


def _structured_rectangle(nx: int, ny: int, h: float):
    """Vertices and ccw triangles of an nx x ny quad grid of spacing h."""
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    xy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)

    def vid(i, j):
        return j * (nx + 1) + i

    qi, qj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    qi = qi.ravel()
    qj = qj.ravel()
    a = vid(qi, qj)
    b = vid(qi + 1, qj)
    c = vid(qi + 1, qj + 1)
    d = vid(qi, qj + 1)
    t1 = np.stack([a, b, c], axis=1)   # lower-right triangle, ccw
    t2 = np.stack([a, c, d], axis=1)   # upper-left triangle, ccw
    cells = np.empty((2 * qi.size, 3), dtype=np.int64)
    cells[0::2] = t1
    cells[1::2] = t2
    boundary = (ii.ravel() == 0) | (ii.ravel() == nx) | (jj.ravel() == 0) | (jj.ravel() == ny)
    return xy, cells, boundary


def _jitter(xy: np.ndarray, boundary: np.ndarray, h: float, amount: float, seed: int) -> np.ndarray:
    """Move interior vertices by independent U[-amount*h, amount*h] in x and y.

    With amount <= 0.2 every triangle keeps a positive area: the legs from the
    right-angle vertex change by at most 0.4h per coordinate, so twice the area
    stays >= (0.6h)^2 - (0.4h)^2 > 0.
    """
    if amount == 0.0:
        return xy.copy()
    rng = np.random.default_rng(seed)
    d = rng.uniform(-amount * h, amount * h, size=xy.shape)
    out = xy.copy()
    out[~boundary] += d[~boundary]
    return out


def _vertex_graph(cells: np.ndarray, nv: int) -> sp.csr_matrix:
    r = np.concatenate([cells[:, 0], cells[:, 1], cells[:, 2], cells[:, 1], cells[:, 2], cells[:, 0]])
    c = np.concatenate([cells[:, 1], cells[:, 2], cells[:, 0], cells[:, 0], cells[:, 1], cells[:, 2]])
    g = sp.csr_matrix((np.ones(r.size, dtype=np.int8), (r, c)), shape=(nv, nv))
    g.data[:] = 1
    return g


def _edges_of(cells: np.ndarray):
    """Unique edges (sorted pairs) and the cell->edge map, edge a opposite vertex a."""
    n2 = cells.shape[0]
    pairs = np.empty((n2, 3, 2), dtype=np.int64)
    for a in range(3):
        p = cells[:, (a + 1) % 3]
        q = cells[:, (a + 2) % 3]
        pairs[:, a, 0] = np.minimum(p, q)
        pairs[:, a, 1] = np.maximum(p, q)
    flat = pairs.reshape(-1, 2)
    uniq, inv = np.unique(flat, axis=0, return_inverse=True)   # sorted by (min, max)
    return uniq, inv.reshape(n2, 3)


def _dual_graph(cell_edge: np.ndarray, n_edges: int) -> sp.csr_matrix:
    """Cells adjacent when they share an edge."""
    n2 = cell_edge.shape[0]
    rows = np.repeat(np.arange(n2), 3)
    inc = sp.csr_matrix((np.ones(rows.size, dtype=np.int32), (rows, cell_edge.ravel())), shape=(n2, n_edges))
    g = (inc @ inc.T).tocsr()
    g.setdiag(0)
    g.eliminate_zeros()
    return g


def _assemble(xy, cells, order: str, seed_order: int, meta: dict) -> BaseMesh:
    nv = xy.shape[0]
    if order == "rcm":
        vperm = reverse_cuthill_mckee(_vertex_graph(cells, nv), symmetric_mode=True)
    elif order == "random":
        vperm = np.random.default_rng(seed_order).permutation(nv)
    elif order == "natural":
        vperm = np.arange(nv)
    else:
        raise ValueError(f"unknown ordering {order!r}")
    # vperm[new] = old
    vinv = np.empty(nv, dtype=np.int64)
    vinv[vperm] = np.arange(nv)
    xy = xy[vperm]
    cells = vinv[cells]
    edges, cell_edge = _edges_of(cells)
    if order == "rcm":
        cperm = reverse_cuthill_mckee(_dual_graph(cell_edge, edges.shape[0]), symmetric_mode=True)
    elif order == "random":
        cperm = np.random.default_rng(seed_order + 1).permutation(cells.shape[0])
    else:
        cperm = np.arange(cells.shape[0])
    cells = cells[cperm]
    cell_edge = cell_edge[cperm]
    if order == "random":
        eperm = np.random.default_rng(seed_order + 2).permutation(edges.shape[0])
        einv = np.empty_like(eperm)
        einv[eperm] = np.arange(eperm.size)
        edges = edges[eperm]
        cell_edge = einv[cell_edge]
    meta = dict(meta, order=order)
    return BaseMesh(
        xy=np.ascontiguousarray(xy, dtype=np.float64),
        cell_vertex=np.ascontiguousarray(cells, dtype=np.int32),
        cell_edge=np.ascontiguousarray(cell_edge, dtype=np.int32),
        edge_vertex=np.ascontiguousarray(edges, dtype=np.int32),
        meta=meta,
    )


def tri_square(n: int, jitter: float = 0.2, seed: int = SEED_MESH, order: str = "rcm",
               seed_order: int = SEED_ORDER) -> BaseMesh:
    """Unit square cut into n x n quads, two ccw triangles each."""
    return tri_rectangle(n, n, 1.0 / n, jitter=jitter, seed=seed, order=order, seed_order=seed_order)


def tri_rectangle(nx: int, ny: int, h: float, jitter: float = 0.2, seed: int = SEED_MESH,
                  order: str = "rcm", seed_order: int = SEED_ORDER) -> BaseMesh:
    """[0, nx*h] x [0, ny*h] cut into nx x ny quads, two ccw triangles each."""
    if nx < 1 or ny < 1:
        raise ValueError("need at least one quad in each direction")
    xy, cells, boundary = _structured_rectangle(nx, ny, h)
    xy = _jitter(xy, boundary, h, jitter, seed)
    meta = dict(nx=nx, ny=ny, h=h, jitter=jitter, seed=seed)
    return _assemble(xy, cells, order, seed_order, meta)


def tri_checkerboard(n: int, order: str = "rcm", seed_order: int = SEED_ORDER) -> BaseMesh:
    """The n x n square with every other quad removed (a checkerboard): the
    cells around an interior vertex form two fans that meet only at it."""
    xy, cells, _ = _structured_rectangle(n, n, 1.0 / n)
    q = np.arange(cells.shape[0]) // 2
    keep = ((q % n) + (q // n)) % 2 == 0
    meta = dict(nx=n, ny=n, h=1.0 / n, jitter=0.0, checkerboard=True)
    return _assemble(xy, cells[keep], order, seed_order, meta)


def level_heights(n_layers: int, height: float = 1.0) -> np.ndarray:
    """z of the n_layers+1 levels of a flat extrusion: l * height / n_layers."""
    return np.arange(n_layers + 1, dtype=np.float64) * (height / n_layers)


def extruded_vertex_coords(mesh: BaseMesh, n_layers: int, height: float = 1.0,
                           terrain: float = 0.0, seed: int = SEED_MESH + 10) -> np.ndarray:
    """Coordinates of every extruded vertex, indexed [vertex, level, xyz].

    Columns are vertical: (x, y) of vertex v is the same at every level.  With
    ``terrain == 0`` the levels are flat, z = l * height / n_layers.  With
    ``terrain > 0`` column v is stretched to height * (1 + terrain * r_v),
    r_v ~ U[-1, 1] (a terrain-following mesh with non-uniform prism heights).
    """
    nv = mesh.n_vertices
    out = np.empty((nv, n_layers + 1, 3), dtype=np.float64)
    out[:, :, 0] = mesh.xy[:, 0:1]
    out[:, :, 1] = mesh.xy[:, 1:2]
    z = level_heights(n_layers, height)
    if terrain == 0.0:
        out[:, :, 2] = z[None, :]
    else:
        r = np.random.default_rng(seed).uniform(-1.0, 1.0, size=nv)
        out[:, :, 2] = z[None, :] * (1.0 + terrain * r)[:, None]
    return out


def layer_ranges(mesh: BaseMesh, n_layers: int, kind: str = "bathymetry", depth: float = 0.5,
                 seed: int = SEED_MESH + 20) -> np.ndarray:
    """Layer range [b_c, t_c) of every cell column (int32 [n_cells, 2]) for a
    mesh whose columns differ in height.

    ``bathymetry``: every column reaches the top level; the bottom of column c
    sits at b_c = floor(depth * n_layers * s(x_c, y_c)), s a smooth bump in
    [0, 1) over the cell centroid, so neighbouring columns differ by few layers
    (an ocean over uneven ground).  ``random``: b_c and n_layers - t_c are
    independent, uniform in 0 .. floor(depth * n_layers) / 2 (ragged at both
    ends, neighbours unrelated).
    """
    cent = mesh.xy[mesh.cell_vertex].mean(axis=1)
    lo = mesh.xy.min(axis=0)
    span = np.maximum(mesh.xy.max(axis=0) - lo, 1e-300)
    u = (cent - lo) / span
    if kind == "bathymetry":
        s = 0.5 * (1.0 + np.sin(2.0 * np.pi * u[:, 0]) * np.sin(3.0 * np.pi * u[:, 1])) * (1.0 - 1e-12)
        b = np.floor(depth * n_layers * s).astype(np.int64)
        t = np.full(mesh.n_cells, n_layers, np.int64)
    elif kind == "random":
        k = int(depth * n_layers) // 2
        rng = np.random.default_rng(seed)
        b = rng.integers(0, k + 1, mesh.n_cells)
        t = n_layers - rng.integers(0, k + 1, mesh.n_cells)
    else:
        raise ValueError(f"unknown layer-range kind {kind!r}")
    b = np.minimum(b, n_layers - 1)
    t = np.maximum(t, b + 1)
    return np.stack([b, t], axis=1).astype(np.int32)


def cell_degrees(mesh: BaseMesh, frac_dg1: float = 0.5, seed: int = SEED_MESH + 30) -> np.ndarray:
    """DoFs per layer of every cell of a mixed-degree DG space: 6 (DG1 x DG1)
    on a seeded random fraction frac_dg1 of the cells, 1 (DG0 x DG0) on the
    rest."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random(mesh.n_cells) < frac_dg1, 6, 1).astype(np.int32)


def entity_dofs(mesh: BaseMesh, hi: int = 3, seed: int = SEED_MESH + 31) -> list:
    """A DoF count per entity, uniform in 0 .. hi - 1 for the horizontal and the
    vertical entities of every base vertex, edge and cell: [N_d, 2] each."""
    rng = np.random.default_rng(seed)
    return [rng.integers(0, hi, (n, 2)).astype(np.int32) for n in mesh.counts]


def uniform_values(n: int, seed: int = SEED_FIELD, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """n float64 values, U[lo, hi], from numpy's PCG64 with the given seed."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


# ---------------------------------------------------------------------------
# Batch of uneven meshes

@dataclass
class BatchItem:
    mesh: BaseMesh
    n_layers: int
    space: str          # "P1" (CG1 x CG1) or "DG0" (DG0 x DG0)


def batch_meshes(n_meshes: int = 64, seed: int = SEED_BATCH, tri_lo: float = 2e3, tri_hi: float = 2e5,
                 layers_lo: int = 10, layers_hi: int = 150, scale: float = 1.0) -> list[BatchItem]:
    """Uneven extruded meshes: base triangle counts log-uniform in
    [tri_lo, tri_hi] (times ``scale``), layer counts uniform integers in
    [layers_lo, layers_hi]; even index -> P1xP1, odd -> DG0xDG0.  Each base is a
    jittered triangulated rectangle of aspect r ~ U[1, 4], RCM-ordered."""
    rng = np.random.default_rng(seed)
    items = []
    for m in range(n_meshes):
        target = float(np.exp(rng.uniform(np.log(tri_lo), np.log(tri_hi)))) * scale
        r = rng.uniform(1.0, 4.0)
        ny = max(1, int(round(np.sqrt(target / (2.0 * r)))))
        nx = max(1, int(round(target / (2.0 * ny))))
        lam = int(rng.integers(layers_lo, layers_hi + 1))
        mesh = tri_rectangle(nx, ny, 1.0 / ny, jitter=0.2, seed=seed * 1000 + m, order="rcm")
        items.append(BatchItem(mesh=mesh, n_layers=lam, space="P1" if m % 2 == 0 else "DG0"))
    return items
