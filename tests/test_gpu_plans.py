"""The race-resolution plans the library builds, read back through the C ABI
and checked entry by entry: the cell colouring (no two cells of one colour
share a vertex), the tile plans (every cell in exactly one tile, the tile's
vertex and edge lists, the shared flags, tile colours without a shared
vertex) and the owner plans (every vertex owned by exactly one tile, a
tile's cells exactly those with an owned vertex).  A plan that broke one of
these would let two units increment one DoF at once, which a parity test
could miss by timing luck."""
import numpy as np
import pytest

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

SHARED = np.int32(-2 ** 31)


def _units(off):
    return np.repeat(np.arange(off.size - 1), np.diff(off))


def _check_cell_colours(base, mesh):
    p = mesh.plan("colours")
    col = p["colour"]
    assert p["n_colours"] == mesh.colours()
    assert col.min() == 0 and col.max() == p["n_colours"] - 1
    assert np.unique(col).size == p["n_colours"]
    # every (vertex, colour) pair at most once over the cell-vertex incidences
    keys = base.cell_vertex.astype(np.int64) * p["n_colours"] + col[:, None]
    assert np.unique(keys).size == keys.size, "two cells of one colour share a vertex"
    return p["n_colours"]


def _check_lists(unit_of_cell, cells, off, ids, local, cell_ent, n_ent, what, lone=None):
    """The entity list of every unit is the union of its cells' entities,
    without repeats, and the local indices point into it.  `lone` flags the
    entities that may be listed without a cell (an owned vertex no cell
    touches)."""
    unit_of_ent = _units(off)
    keys = unit_of_ent.astype(np.int64) * n_ent + ids
    assert np.unique(keys).size == keys.size, f"{what}: an entity repeats within a unit"
    if lone is not None:
        keys = keys[~lone[ids]]
    want = np.unique(unit_of_cell[:, None].astype(np.int64) * n_ent + cell_ent[cells])
    np.testing.assert_array_equal(np.sort(keys), want, err_msg=f"{what}: list is not the union of its cells")
    pos = off[unit_of_cell][:, None] + local.reshape(-1, 3).astype(np.int64)
    assert np.all(local.reshape(-1, 3) < np.diff(off)[unit_of_cell][:, None])
    np.testing.assert_array_equal(ids[pos], cell_ent[cells], err_msg=f"{what}: local index")
    return unit_of_ent


def _check_tiles(base, mesh, target):
    p = mesh.plan("tiles", target)
    nt = p["cell_off"].size - 1
    cells = p["cells"]
    np.testing.assert_array_equal(np.sort(cells), np.arange(base.n_cells), err_msg="a cell not in exactly one tile")
    assert np.diff(p["cell_off"]).min() >= 1 and np.diff(p["cell_off"]).max() <= target
    tile_of_cell = _units(p["cell_off"])
    verts = p["verts"] & 0x7FFFFFFF
    tile_of_vert = _check_lists(tile_of_cell, cells, p["vert_off"], verts, p["local_cv"], base.cell_vertex,
                                base.n_vertices, "tile vertices")
    touched = np.bincount(verts, minlength=base.n_vertices)
    np.testing.assert_array_equal(p["verts"] < 0, touched[verts] > 1, err_msg="shared vertex flag")
    if "edges" in p:
        edges = p["edges"] & 0x7FFFFFFF
        _check_lists(tile_of_cell, cells, p["edge_off"], edges, p["local_ce"], base.cell_edge, base.n_edges,
                     "tile edges")
        touched_e = np.bincount(edges, minlength=base.n_edges)
        np.testing.assert_array_equal(p["edges"] < 0, touched_e[edges] > 1, err_msg="shared edge flag")
    col = p["colour"]
    assert col.min() == 0 and col.max() == p["n_colours"] - 1
    keys = verts.astype(np.int64) * p["n_colours"] + col[tile_of_vert]
    assert np.unique(keys).size == keys.size, "two tiles of one colour share a vertex"
    return nt, p["n_colours"]


def _check_owner(base, mesh, target):
    p = mesh.plan("owner", target)
    nt = p["cell_off"].size - 1
    owned = p["owned"]
    assert owned.min() >= 1
    tile_of_cell = _units(p["cell_off"])
    verts = p["verts"]
    assert verts.min() >= 0
    lone = np.bincount(base.cell_vertex.ravel(), minlength=base.n_vertices) == 0
    tile_of_vert = _check_lists(tile_of_cell, p["cells"], p["vert_off"], verts, p["local_cv"], base.cell_vertex,
                                base.n_vertices, "owner tile vertices", lone=lone)
    rank = np.arange(verts.size) - p["vert_off"][tile_of_vert]
    mine = rank < owned[tile_of_vert]
    np.testing.assert_array_equal(np.sort(verts[mine]), np.arange(base.n_vertices),
                                  err_msg="a vertex not owned by exactly one tile")
    owner = np.empty(base.n_vertices, np.int64)
    owner[verts[mine]] = tile_of_vert[mine]
    assert not np.any(lone[verts[~mine]]), "a vertex without cells listed as read-only"
    assert np.all(owner[verts[~mine]] != tile_of_vert[~mine]), "an owned vertex listed again as read-only"
    # the cells of a tile are exactly those with a vertex it owns
    want = np.unique(owner[base.cell_vertex] * base.n_cells + np.arange(base.n_cells)[:, None])
    got = tile_of_cell.astype(np.int64) * base.n_cells + p["cells"]
    assert np.unique(got).size == got.size, "a cell repeats within an owner tile"
    np.testing.assert_array_equal(np.sort(got), want, err_msg="owner tile cells")
    assert p["n_colours"] == 1
    return nt


@pytest.mark.parametrize("n,order", [(7, "rcm"), (16, "random"), (33, "rcm")])
def test_plans_small(n, order):
    base = meshgen.tri_square(n, order=order)
    mesh = exm.Mesh(base, 3)
    _check_cell_colours(base, mesh)
    for target in (8, 32, 64, 1000):
        _check_tiles(base, mesh, target)
        _check_owner(base, mesh, target)


def test_plans_checkerboard():
    # vertices whose cells form two fans that meet only at the vertex
    base = meshgen.tri_checkerboard(12)
    mesh = exm.Mesh(base, 2)
    _check_cell_colours(base, mesh)
    for target in (8, 64):
        _check_tiles(base, mesh, target)
        _check_owner(base, mesh, target)


def test_plans_batch_rectangle():
    it = meshgen.batch_meshes(n_meshes=3, scale=0.02)[1]
    mesh = exm.Mesh(it.mesh, it.n_layers)
    _check_cell_colours(it.mesh, mesh)
    _check_tiles(it.mesh, mesh, 64)
    _check_owner(it.mesh, mesh, 64)


def test_plans_config2():
    """The plans behind the benchmark's launches on the 512 x 512 base."""
    say("plans 512x512")
    base = meshgen.tri_square(512)
    mesh = exm.Mesh(base, 100)
    ncol = _check_cell_colours(base, mesh)
    nt, tcol = _check_tiles(base, mesh, 64)
    no = _check_owner(base, mesh, 64)
    _check_tiles(base, mesh, 32)
    say(f"  cell colours {ncol}, 64-cell tiles {nt} in {tcol} colours, owner tiles {no}")
