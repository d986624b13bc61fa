"""The oracle on several host threads (the all-core CPU baseline): its own
greedy colouring is valid, and the threaded runs give the sequential
oracle's values up to the order of summation (bit for bit where every DoF
has one contributing cell)."""
import numpy as np
import pytest

import oracle
from paper_1604_05937_amd import meshgen


@pytest.mark.parametrize("order", ["rcm", "random"])
def test_greedy_colouring_separates_cells_sharing_a_vertex(order):
    base = meshgen.tri_square(24, order=order)
    colour, n = oracle.greedy_colour(base.cell_vertex, base.n_vertices)
    assert colour.min() == 0 and colour.max() == n - 1
    keys = base.cell_vertex.astype(np.int64) * n + colour[:, None]
    assert np.unique(keys).size == keys.size
    # greedy in base order: each cell's colour is the smallest free one, so
    # every smaller colour is held by a neighbour visited earlier
    for c in range(0, base.n_cells, 37):
        nb = np.nonzero(np.isin(base.cell_vertex, base.cell_vertex[c]).any(axis=1))[0]
        earlier = set(colour[nb[nb < c]].tolist())
        assert all(k in earlier for k in range(colour[c]))


@pytest.mark.parametrize("space", ["P1", "P2", "DG0", "DG1", "CG1xDG1"])
@pytest.mark.parametrize("threads", [3, 8])
def test_threaded_oracle_matches_sequential(space, threads):
    base = meshgen.tri_square(12)
    lam = 7
    vc = meshgen.extruded_vertex_coords(base, lam, terrain=0.1)
    pr = oracle.Problem(base, lam, space, vc)
    x = meshgen.uniform_values(pr.n_dofs, seed=5)
    want = pr.mass(x)
    write = not oracle.is_continuous(pr.space)
    got = np.zeros(pr.n_dofs)
    colour, _ = oracle.greedy_colour(base.cell_vertex, base.n_vertices)
    oracle.par_loop_threaded(oracle.FORM_MASS, pr.space, pr.num_v, pr.num_x, pr.X, [x], [got], write=write,
                             threads=threads, colour=colour)
    if write:
        np.testing.assert_array_equal(got, want)
    else:
        scale = pr.mass_abs(x)
        assert np.all(np.abs(got - want) <= 1e-13 * scale)
