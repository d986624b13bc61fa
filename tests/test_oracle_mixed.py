"""Pins of the oracle's mixed-degree DG mass action (cells DG0 x DG0 or
DG1 x DG1, numbered with a DoF count per entity): the uniform spaces at both
ends, the volume, and cell-by-cell agreement with the pure spaces."""
import numpy as np
import pytest

import oracle
from paper_1604_05937_amd import meshgen


def _setup(n=4, lam=3, terrain=0.3):
    mesh = meshgen.tri_square(n, jitter=0.2)
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=terrain)
    return mesh, lam, vc


@pytest.mark.parametrize("k,name", [(1, "DG0"), (6, "DG1")])
def test_one_degree_everywhere_is_the_uniform_space(k, name):
    mesh, lam, vc = _setup()
    nd = np.full(mesh.n_cells, k, np.int32)
    pr = oracle.Problem(mesh, lam, name, vc)
    x = meshgen.uniform_values(pr.n_dofs, seed=71)
    y, num = oracle.mixed_dg_mass(mesh, lam, vc, nd, x)
    assert num.n_dofs == pr.n_dofs
    np.testing.assert_array_equal(num.lmap, pr.num_v.lmap[:, 0] if k == 1 else pr.num_v.lmap.ravel())
    np.testing.assert_array_equal(y, pr.mass(x))


def test_mixed_degrees_integrate_the_constant():
    # the constant 1 (every nodal value 1): the residual sums to the volume
    mesh, lam, vc = _setup(terrain=0.4)
    nd = meshgen.cell_degrees(mesh, frac_dg1=0.4)
    y, num = oracle.mixed_dg_mass(mesh, lam, vc, nd, np.ones(int(((lam) * nd).sum())))
    vol = 0.0
    for c in range(mesh.n_cells):
        a, b, d = mesh.cell_vertex[c]
        xy = mesh.xy
        twoA = abs((xy[b, 0] - xy[a, 0]) * (xy[d, 1] - xy[a, 1]) - (xy[d, 0] - xy[a, 0]) * (xy[b, 1] - xy[a, 1]))
        for l in range(lam):
            vol += twoA * sum(vc[v, l + 1, 2] - vc[v, l, 2] for v in (a, b, d)) / 6.0
    assert abs(y.sum() - vol) < 1e-14


def test_mixed_columns_match_the_pure_spaces_cell_by_cell():
    mesh, lam, vc = _setup()
    nd = meshgen.cell_degrees(mesh, frac_dg1=0.5)
    x = meshgen.uniform_values(int((lam * nd).sum()), seed=72)
    y, num = oracle.mixed_dg_mass(mesh, lam, vc, nd, x)
    pure = {1: oracle.Problem(mesh, lam, "DG0", vc), 6: oracle.Problem(mesh, lam, "DG1", vc)}
    for c in range(mesh.n_cells):
        k = int(nd[c])
        s = num.lmap[num.list_off[c]]
        pr = pure[k]
        xu = np.zeros(pr.n_dofs)
        u0 = pr.num_v.lmap[c, 0]
        xu[u0:u0 + k * lam] = x[s:s + k * lam]
        yu = pr.mass(xu, cells=np.array([c]))
        np.testing.assert_allclose(y[s:s + k * lam], yu[u0:u0 + k * lam], rtol=0, atol=1e-16)
