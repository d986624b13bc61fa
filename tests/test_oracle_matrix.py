"""Pins of the oracle's matrix assembly (the bilinear forms behind the
residuals: the mass matrix on the paper's nine spaces plus P2, and the
Jacobian of the cubic residual): exact rational entries, the sparsity
pattern of brute-force prism enumeration, the matrix-free actions, symmetry,
volume, and finite differences."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1604_05937_amd import meshgen
from tests import bruteforce

SPACES = ["P1", "DG0", "DG1", "P2", "CG1xDG0", "CG1xDG1", "DG0xCG1", "DG0xDG1", "DG1xCG1", "DG1xDG0"]


def _problem(space, n=3, lam=3, terrain=0.3):
    mesh = meshgen.tri_square(n, jitter=0.2)
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=terrain)
    return mesh, vc, oracle.Problem(mesh, lam, space, vc)


@pytest.mark.parametrize("space", SPACES)
def test_mass_matrix_entries_are_exact(space):
    # column j of M is the exact mass action on the unit vector e_j
    mesh, vc, pr = _problem(space, n=1, lam=2)
    M = pr.mass_matrix().toarray()
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, 2, oracle.delta_table(*pr.space))
    assert n == pr.n_dofs
    exact = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        exact[:, j] = [float(x) for x in bruteforce.exact_mass(mesh, vc, 2, pr.space, stencils, n, e)]
    assert np.abs(M - exact).max() <= 1e-14 * np.abs(exact).max()


@pytest.mark.parametrize("space", SPACES)
def test_pattern_is_the_prism_sharing_relation(space):
    # (i, j) is stored iff DoFs i and j belong to one prism, by enumeration of
    # the explicit 3D mesh
    mesh, vc, pr = _problem(space, n=3, lam=3)
    M = pr.mass_matrix().tocoo()
    got = set(zip(M.row.tolist(), M.col.tolist()))
    _, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, 3, oracle.delta_table(*pr.space))
    want = {(a, b) for row in stencils.values() for a in row for b in row}
    assert got == want


@pytest.mark.parametrize("space", SPACES)
def test_mass_matrix_is_the_mass_action(space):
    mesh, vc, pr = _problem(space, n=4, lam=5)
    M = pr.mass_matrix()
    x = meshgen.uniform_values(pr.n_dofs, seed=11)
    np.testing.assert_allclose(M @ x, pr.mass(x), rtol=0, atol=1e-15 * np.abs(M).sum(axis=1).max())
    assert abs(M - M.T).max() <= 1e-16
    # 1^T M 1 is the volume of the extruded domain (for a space holding the constants)
    one = np.ones(pr.n_dofs)
    if space in ("P1", "DG0", "DG1", "P2", "DG1xCG1", "DG0xCG1"):
        vol = 0.0
        for c in range(mesh.n_cells):
            a, b, d = mesh.cell_vertex[c]
            xy = mesh.xy
            twoA = abs((xy[b, 0] - xy[a, 0]) * (xy[d, 1] - xy[a, 1]) - (xy[d, 0] - xy[a, 0]) * (xy[b, 1] - xy[a, 1]))
            for l in range(5):
                vol += twoA * sum(vc[v, l + 1, 2] - vc[v, l, 2] for v in (a, b, d)) / 6.0
        assert abs(one @ (M @ one) - vol) < 1e-14


def test_mass_matrix_of_dg0_is_the_prism_volumes():
    mesh, vc, pr = _problem("DG0", n=3, lam=4, terrain=0.0)
    M = pr.mass_matrix()
    assert M.nnz == pr.n_dofs
    d = M.diagonal()
    for c in range(mesh.n_cells):
        a, b, e = mesh.cell_vertex[c]
        xy = mesh.xy
        area = 0.5 * abs((xy[b, 0] - xy[a, 0]) * (xy[e, 1] - xy[a, 1]) - (xy[e, 0] - xy[a, 0]) * (xy[b, 1] - xy[a, 1]))
        np.testing.assert_allclose(d[pr.num_v.lmap[c, 0]:pr.num_v.lmap[c, 0] + 4], area / 4.0, rtol=1e-14)


def test_cubic_jacobian_is_the_derivative():
    mesh, vc, pr = _problem("P1", n=3, lam=4)
    u = meshgen.uniform_values(pr.n_dofs, seed=12)
    du = meshgen.uniform_values(pr.n_dofs, seed=13)
    f = meshgen.uniform_values(pr.n_dofs, seed=14)
    J = pr.cubic_jacobian(u)
    # the tangent map of the residual (pinned against exact rationals elsewhere)
    np.testing.assert_allclose(J @ du, pr.cubic_jvp(u, du, np.zeros(pr.n_dofs)), rtol=0, atol=1e-15)
    # central differences of the residual: F is cubic in u, so the O(h^2)
    # error is (h^2 / 6) F'''[du, du, du]
    h = 1e-4
    fd = (pr.cubic(u + h * du, f) - pr.cubic(u - h * du, f)) / (2 * h)
    assert np.abs(J @ du - fd).max() < 1e-8
    # J is symmetric (the residual is the gradient of integral u^4 / 4 - f u)
    assert abs(J - J.T).max() <= 1e-16
    # with u = 1 the Jacobian is three times the mass matrix
    J1 = pr.cubic_jacobian(np.ones(pr.n_dofs))
    assert abs(J1 - 3.0 * pr.mass_matrix()).max() <= 1e-15


def test_cubic_jacobian_entries_are_exact():
    # column j of J is the exact tangent of the cubic residual along e_j:
    # d/dt F(u + t e_j) at t = 0, from the exact rational residual at
    # t = +-1/2 and +-1 (F is cubic in t: a five-point stencil is exact)
    mesh, vc, pr = _problem("P1", n=1, lam=2, terrain=0.2)
    # u on a 2^-20 grid, so that u + t below is exact in binary64
    u = np.round(meshgen.uniform_values(pr.n_dofs, seed=15) * 2.0**20) / 2.0**20
    J = pr.cubic_jacobian(u).toarray()
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, 2, oracle.delta_table("CG1", "CG1"))
    f0 = np.zeros(n)
    for j in range(n):
        vals = {}
        for t in (Fraction(-1), Fraction(-1, 2), Fraction(1, 2), Fraction(1)):
            ut = u.copy()
            ut[j] += float(t)
            assert Fraction(float(ut[j])) == Fraction(float(u[j])) + t
            vals[t] = bruteforce.exact_cubic(mesh, vc, 2, stencils, n, ut, f0)
        col = [(8 * (vals[Fraction(1, 2)][i] - vals[Fraction(-1, 2)][i]) - (vals[Fraction(1)][i] - vals[Fraction(-1)][i]))
               / 6 for i in range(n)]
        np.testing.assert_allclose(J[:, j], [float(c) for c in col], rtol=0, atol=1e-14)


def test_abs_forms_bound_the_entries():
    mesh, vc, pr = _problem("P2", n=2, lam=2)
    M = pr.mass_matrix()
    S = pr.mass_matrix_abs()
    assert (S.indices == M.indices).all() and (S.indptr == M.indptr).all()
    assert (np.abs(M.data) <= S.data * (1 + 1e-15)).all()
