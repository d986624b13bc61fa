"""Input generator checks (counts, orientation, conventions, orderings)."""
import numpy as np
import pytest

from paper_1604_05937_amd import meshgen


@pytest.mark.parametrize("order", ["rcm", "random", "natural"])
def test_counts_and_euler(order):
    m = meshgen.tri_square(16, order=order)
    assert m.counts == (289, 800, 512)
    assert m.n_vertices - m.n_edges + m.n_cells == 1


@pytest.mark.parametrize("order", ["rcm", "random"])
def test_orientation_and_edge_convention(order):
    m = meshgen.tri_square(12, order=order)
    p = m.xy[m.cell_vertex]
    twoA = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    assert np.all(twoA > 0)
    for a in range(3):
        ev = m.edge_vertex[m.cell_edge[:, a]]
        pq = np.sort(np.stack([m.cell_vertex[:, (a + 1) % 3], m.cell_vertex[:, (a + 2) % 3]], axis=1), axis=1)
        np.testing.assert_array_equal(ev, pq)
    assert abs(0.5 * twoA.sum() - 1.0) < 1e-12


def test_rcm_reduces_bandwidth():
    r = meshgen.tri_square(20, order="rcm")
    x = meshgen.tri_square(20, order="random")
    bw = lambda m: np.abs(m.cell_vertex[:, :, None] - m.cell_vertex[:, None, :]).max()
    assert bw(r) < bw(x) / 5


def test_seeded():
    a = meshgen.tri_square(8)
    b = meshgen.tri_square(8)
    np.testing.assert_array_equal(a.xy, b.xy)
    np.testing.assert_array_equal(a.cell_vertex, b.cell_vertex)
    np.testing.assert_array_equal(meshgen.uniform_values(10, 3), meshgen.uniform_values(10, 3))


def test_batch_shapes():
    items = meshgen.batch_meshes(n_meshes=6, scale=0.02)
    assert [it.space for it in items] == ["P1", "DG0"] * 3
    for it in items:
        assert 10 <= it.n_layers <= 150
        assert it.mesh.n_cells >= 2


def test_byte_counts_from_entity_counts():
    # the closed-form DoF counts of the byte model (no device needed)
    from paper_1604_05937_amd import workloads as W
    base = meshgen.tri_square(512)
    p1 = W.mass_bytes_counts(base, 100, "P1")
    d0 = W.mass_bytes_counts(base, 100, "DG0")
    assert p1["n_dofs"] == 26580069 and d0["n_dofs"] == 52428800
    # K1: f + b (read and written) + z + (x, y) per base vertex + the 6-entry lists
    assert p1["algorithmic"] == 867355824
    assert p1["valuable"] == 8 * 26580069 * 2 + 24 * 26580069
