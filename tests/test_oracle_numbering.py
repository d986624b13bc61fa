"""Pins of the oracle's numbering (Algorithm 1), explicit lists and offsets
(Algorithm 2) and direct addressing (the n-th application formula of Section
3.3) against a brute-force numbering of the explicit 3D mesh."""
import numpy as np
import pytest

import oracle
from paper_1604_05937_amd import meshgen
from tests import bruteforce

SPACES = [("CG1", "CG1"), ("DG0", "DG0"), ("DG1", "DG1"), ("CG2", "CG2"),
          ("CG1", "DG0"), ("CG1", "DG1"), ("DG0", "CG1"), ("DG0", "DG1"),
          ("DG1", "CG1"), ("DG1", "DG0")]


@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("order", ["rcm", "random"])
def test_numbering_matches_bruteforce(space, order):
    mesh = meshgen.tri_square(3, order=order)
    lam = 3
    delta = oracle.delta_table(*space)
    num = oracle.number(mesh.counts, lam, delta, mesh.cell_vertex, mesh.cell_edge)
    n, first, stencils, entities = bruteforce.bruteforce_numbering(mesh, lam, delta)
    assert num.n_dofs == n
    # every entity of the explicit 3D mesh gets the same first DoF
    for ((d1, d2), i, l), f in first.items():
        assert num.first[d1][i, l, d2] == f
    # every prism's stencil is L(c) + l * offset (Section 3.3, n-th application)
    for (c, l), row in stencils.items():
        np.testing.assert_array_equal(num.lmap[c] + l * num.offsets, row)


@pytest.mark.parametrize("space", SPACES)
def test_entity_set_sizes_and_bijection(space):
    mesh = meshgen.tri_square(4)
    lam = 5
    delta = oracle.delta_table(*space)
    num = oracle.number(mesh.counts, lam, delta, mesh.cell_vertex, mesh.cell_edge)
    # |V_{d1,d2}| = N_d1 (lam + 1 - d2) (Section 3.1.3); the DoF count follows
    expect = sum(mesh.counts[d1] * (lam + 1 - d2) * delta[d1, d2] for d1 in range(3) for d2 in range(2))
    assert num.n_dofs == expect
    # DoFs form a bijection onto [0, n_dofs)
    seen = np.zeros(num.n_dofs, dtype=np.int64)
    for d1 in range(3):
        for d2 in range(2):
            nd = int(delta[d1, d2])
            if nd == 0:
                continue
            for i in range(mesh.counts[d1]):
                for l in range(lam + 1 - d2):
                    f = num.first[d1][i, l, d2]
                    seen[f:f + nd] += 1
    assert np.all(seen == 1)


def test_vertically_adjacent_entities_have_adjacent_numbers():
    # Section 3.2: DoFs of vertically adjacent entities have adjacent numbers,
    # i.e. each entity column is one contiguous block walked bottom to top.
    mesh = meshgen.tri_square(3)
    lam = 4
    delta = oracle.delta_table("CG2", "CG2")
    num = oracle.number(mesh.counts, lam, delta, mesh.cell_vertex, mesh.cell_edge)
    for d1 in range(2):
        for i in range(mesh.counts[d1]):
            seq = []
            for l in range(lam + 1):
                for d2 in range(2 if l < lam else 1):
                    f = num.first[d1][i, l, d2]
                    seq += list(range(f, f + int(delta[d1, d2])))
            assert seq == list(range(seq[0], seq[0] + len(seq)))


@pytest.mark.parametrize("space,k,off", [
    (("CG1", "CG1"), 6, 1), (("DG0", "DG0"), 1, 1), (("DG1", "DG1"), 6, 6), (("CG2", "CG2"), 18, 2),
    (("CG1", "DG0"), 3, 1), (("CG1", "DG1"), 6, 2), (("DG0", "CG1"), 2, 1), (("DG0", "DG1"), 2, 2),
    (("DG1", "CG1"), 6, 3), (("DG1", "DG0"), 3, 3)])
def test_stencil_sizes_and_offsets(space, k, off):
    # DoFs per cell 1/2/3/6 for the nine low-order pairs (Section 4.3), 18 for
    # P2 x P2; Algorithm 2 gives delta(d,0) + delta(d,1) for every position.
    mesh = meshgen.tri_square(2)
    num = oracle.number(mesh.counts, 2, oracle.delta_table(*space), mesh.cell_vertex, mesh.cell_edge)
    assert num.k == k
    assert np.all(num.offsets == off)


def test_lists_reduce_by_lambda():
    # Section 3.3: one explicit list per column instead of one per layer.
    mesh = meshgen.tri_square(3)
    for lam in (1, 2, 7):
        num = oracle.number(mesh.counts, lam, oracle.delta_table("CG1", "CG1"), mesh.cell_vertex, mesh.cell_edge)
        assert num.lmap.shape == (mesh.n_cells, 6)


def test_p1_row_layout():
    # P1 x P1: column of vertex v starts at v (lam + 1); the row of a cell is
    # (S(v0), S(v0)+1, S(v1), S(v1)+1, S(v2), S(v2)+1).
    mesh = meshgen.tri_square(3)
    lam = 4
    num = oracle.number(mesh.counts, lam, oracle.delta_table("CG1", "CG1"), mesh.cell_vertex, mesh.cell_edge)
    S = num.column_starts(0)
    np.testing.assert_array_equal(S, np.arange(mesh.n_vertices) * (lam + 1))
    for c in range(mesh.n_cells):
        v = mesh.cell_vertex[c]
        np.testing.assert_array_equal(num.lmap[c], [S[v[0]], S[v[0]] + 1, S[v[1]], S[v[1]] + 1, S[v[2]], S[v[2]] + 1])


def _ranges(mesh, lam, seed):
    """Seeded layer ranges whose columns around any vertex overlap (every
    range starts at or below 2 and ends at or above lam - 2)."""
    rng = np.random.default_rng(seed)
    lo = rng.integers(0, 3, mesh.n_cells)
    hi = lam - rng.integers(0, 3, mesh.n_cells)
    return np.stack([lo, hi], axis=1).astype(np.int32)


@pytest.mark.parametrize("space", SPACES)
def test_variable_layers_match_bruteforce(space):
    mesh = meshgen.tri_square(3, order="random")
    lam = 6
    layers = _ranges(mesh, lam, 5)
    delta = oracle.delta_table(*space)
    num = oracle.number(mesh.counts, lam, delta, mesh.cell_vertex, mesh.cell_edge, layers=layers)
    n, first, stencils, entities = bruteforce.bruteforce_numbering(mesh, lam, delta, layers)
    assert num.n_dofs == n
    for ((d1, d2), i, l), f in first.items():
        assert num.first[d1][i, l, d2] == f
    # direct addressing from the column's bottom prism
    for (c, l), row in stencils.items():
        np.testing.assert_array_equal(num.lmap[c] + (l - layers[c, 0]) * num.offsets, row)
    # bijection onto 0 .. n_dofs - 1 and per-cell layer counts
    assert sorted({int(x) for row in stencils.values() for x in row}) == list(range(n))
    np.testing.assert_array_equal(num.cell_lam, layers[:, 1] - layers[:, 0])


def test_variable_layers_reduce_to_uniform():
    mesh = meshgen.tri_square(4)
    lam = 5
    full = np.tile(np.array([[0, lam]], np.int32), (mesh.n_cells, 1))
    for space in SPACES:
        delta = oracle.delta_table(*space)
        a = oracle.number(mesh.counts, lam, delta, mesh.cell_vertex, mesh.cell_edge)
        b = oracle.number(mesh.counts, lam, delta, mesh.cell_vertex, mesh.cell_edge, layers=full)
        assert a.n_dofs == b.n_dofs
        np.testing.assert_array_equal(a.lmap, b.lmap)
        for d in range(3):
            if a.first[d] is not None:
                np.testing.assert_array_equal(a.first[d], b.first[d])


def _random_entity_dofs(mesh, seed, hi=3):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, hi, (n, 2)).astype(np.int32) for n in mesh.counts]


@pytest.mark.parametrize("lam", [1, 3, 4])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_entity_dofs_match_bruteforce(lam, seed):
    # a DoF count per entity (the per-type constant of the exposition relaxed):
    # the counter loop against sorting every (entity, j) key of the explicit mesh
    mesh = meshgen.tri_square(3, jitter=0.2, order="random")
    dofs = _random_entity_dofs(mesh, seed)
    num = oracle.number_mixed(mesh.counts, lam, dofs, mesh.cell_vertex, mesh.cell_edge)
    n, first, stencils, _ = bruteforce.bruteforce_numbering(mesh, lam, np.zeros((3, 2)), dofs=dofs)
    assert num.n_dofs == n
    for ((d1, d2), i, l), f in first.items():
        assert num.first[d1][i, l, d2] == f
    for (c, l), row in stencils.items():
        a, b = num.list_off[c], num.list_off[c + 1]
        got = num.lmap[a:b] + l * num.offsets[a:b].astype(np.int64)
        assert got.tolist() == row, (c, l)


def test_entity_dofs_reduce_to_the_type_table():
    mesh = meshgen.tri_square(4)
    lam = 5
    for space in ("P1", "P2", "DG1", "DG1xCG1", "CG1xDG1"):
        delta = oracle.delta_table(*oracle.SPACES[space])
        dofs = [np.tile(delta[d], (mesh.counts[d], 1)) for d in range(3)]
        mix = oracle.number_mixed(mesh.counts, lam, dofs, mesh.cell_vertex, mesh.cell_edge)
        uni = oracle.number(mesh.counts, lam, delta, mesh.cell_vertex, mesh.cell_edge)
        assert mix.n_dofs == uni.n_dofs
        k = uni.k
        np.testing.assert_array_equal(mix.list_off, np.arange(mesh.n_cells + 1) * k)
        np.testing.assert_array_equal(mix.lmap.reshape(-1, k), uni.lmap)
        np.testing.assert_array_equal(mix.offsets.reshape(-1, k), np.tile(uni.offsets, (mesh.n_cells, 1)))
        for d in range(3):
            if uni.first[d] is not None:
                np.testing.assert_array_equal(mix.column_starts(d), uni.column_starts(d))


def test_entity_dofs_count_formula():
    # n_dofs = sum over entities of (lam + 1) n_h + lam n_v
    mesh = meshgen.tri_square(5)
    lam = 7
    dofs = _random_entity_dofs(mesh, 9, hi=5)
    num = oracle.number_mixed(mesh.counts, lam, dofs, mesh.cell_vertex, mesh.cell_edge)
    assert num.n_dofs == sum(int(((lam + 1) * d[:, 0] + lam * d[:, 1]).sum()) for d in dofs)
