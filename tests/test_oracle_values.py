"""Pins of the oracle's element kernels: exact rational assembly (no
quadrature), closed-form integrals, partition of unity, symmetry, the DG0
closed form and the derivatives of the cubic residual."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1604_05937_amd import meshgen
from tests import bruteforce


def _rel_close(got, exact, tol=1e-13):
    exact = np.array([float(x) for x in exact])
    scale = max(1.0, np.abs(exact).max())
    err = np.abs(got - exact).max() / scale
    assert err <= tol, err


@pytest.mark.parametrize("space", ["P1", "DG0", "DG1", "P2", ("CG1", "DG0"), ("DG0", "CG1"), ("DG1", "CG1"), ("CG1", "DG1"),
                                   ("DG0", "DG1"), ("DG1", "DG0")])
@pytest.mark.parametrize("terrain", [0.0, 0.3])
def test_mass_matches_exact_rationals(space, terrain):
    mesh = meshgen.tri_square(3, jitter=0.2)
    lam = 2
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=terrain)
    pr = oracle.Problem(mesh, lam, space, vc)
    f = meshgen.uniform_values(pr.n_dofs, seed=7)
    got = pr.mass(f)
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, lam, oracle.delta_table(*pr.space))
    exact = bruteforce.exact_mass(mesh, vc, lam, pr.space, stencils, n, f)
    _rel_close(got, exact)


@pytest.mark.parametrize("terrain", [0.0, 0.3])
def test_cubic_matches_exact_rationals(terrain):
    mesh = meshgen.tri_square(2, jitter=0.2)
    lam = 2
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=terrain)
    pr = oracle.Problem(mesh, lam, "P1", vc)
    u = meshgen.uniform_values(pr.n_dofs, seed=8)
    f = meshgen.uniform_values(pr.n_dofs, seed=9)
    got = pr.cubic(u, f)
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, lam, oracle.delta_table("CG1", "CG1"))
    exact = bruteforce.exact_cubic(mesh, vc, lam, stencils, n, u, f)
    _rel_close(got, exact)


def _interp(pr, func):
    """Interpolate func(x, y, z) at the nodes of P1/P2 x P1/P2 (node coordinates
    from the explicit lists: every DoF sits on one node of one prism)."""
    h, v = pr.space
    lay = oracle.stencil_layout(h, v)
    vals = np.zeros(pr.n_dofs)
    xy = pr.mesh.xy
    z = meshgen.level_heights(pr.n_layers)
    for c in range(pr.mesh.n_cells):
        cv = pr.mesh.cell_vertex[c]
        for l in range(pr.n_layers):
            row = pr.num_v.lmap[c] + l * pr.num_v.offsets
            for p, (d, ent, part, alpha, beta) in enumerate(lay):
                if d == 0:
                    x = xy[cv[ent]]
                elif d == 1:
                    x = 0.5 * (xy[cv[(ent + 1) % 3]] + xy[cv[(ent + 2) % 3]])
                else:
                    x = xy[cv[alpha]]        # DG1 node alpha sits at vertex alpha
                zz = {"bot": z[l], "top": z[l + 1]}.get(part)
                if zz is None:
                    if v == "CG2":
                        zz = 0.5 * (z[l] + z[l + 1])
                    elif v == "DG1":
                        zz = z[l] if beta == 0 else z[l + 1]
                    else:
                        zz = 0.5 * (z[l] + z[l + 1])
                vals[row[p]] = func(x[0], x[1], zz)
    return vals


@pytest.mark.parametrize("space,func,exact", [
    ("P1", lambda x, y, z: x * z, 0.25),
    ("P1", lambda x, y, z: 1.0, 1.0),
    ("DG1", lambda x, y, z: x * z, 0.25),
    ("P2", lambda x, y, z: x * x * z * z, 1.0 / 9.0),
    ("P2", lambda x, y, z: y * y + x * z, 1.0 / 3.0 + 0.25),
    ("DG0", lambda x, y, z: 1.0, 1.0),
])
def test_closed_form_integrals(space, func, exact):
    # Sum_i integral(f v_i) = integral(f) over the unit cube (partition of
    # unity), for f in the space so interpolation is exact.
    mesh = meshgen.tri_square(5, jitter=0.2)
    lam = 3
    pr = oracle.Problem(mesh, lam, space, meshgen.extruded_vertex_coords(mesh, lam))
    f = _interp(pr, func)
    assert abs(pr.mass(f).sum() - exact) < 1e-13


def test_p1_interior_vertex_integral():
    # Unjittered mesh: an interior vertex at an interior level has
    # integral(v_i) = h^2 dz (patch area 3h^2, hat function mean 1/3).
    n, lam = 6, 4
    mesh = meshgen.tri_square(n, jitter=0.0, order="natural")
    pr = oracle.Problem(mesh, lam, "P1", meshgen.extruded_vertex_coords(mesh, lam))
    b = pr.mass(np.ones(pr.n_dofs))
    h, dz = 1.0 / n, 1.0 / lam
    v = 3 * (n + 1) + 3
    S = pr.num_v.column_starts(0)
    for l in range(1, lam):
        assert abs(b[S[v] + l] - h * h * dz) < 1e-15


def test_dg0_closed_form():
    # DG0: b_c = f_c * |A_c| * dz, a single-point closed form.
    mesh = meshgen.tri_square(4)
    lam = 3
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=0.3)
    pr = oracle.Problem(mesh, lam, "DG0", vc)
    f = meshgen.uniform_values(pr.n_dofs)
    b = pr.mass(f)
    for c in range(mesh.n_cells):
        p = mesh.xy[mesh.cell_vertex[c]]
        A = 0.5 * abs((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[2, 0] - p[0, 0]) * (p[1, 1] - p[0, 1]))
        for l in range(lam):
            hts = vc[mesh.cell_vertex[c], l + 1, 2] - vc[mesh.cell_vertex[c], l, 2]
            dof = pr.num_v.lmap[c, 0] + l
            assert abs(b[dof] - f[dof] * A * hts.mean()) < 1e-15


@pytest.mark.parametrize("space", ["P1", "DG1", "P2", "CG1xDG0", "CG1xDG1", "DG0xCG1", "DG0xDG1", "DG1xCG1", "DG1xDG0"])
def test_mass_symmetric_and_volume(space):
    mesh = meshgen.tri_square(4)
    lam = 3
    pr = oracle.Problem(mesh, lam, space, meshgen.extruded_vertex_coords(mesh, lam, terrain=0.2))
    x1 = meshgen.uniform_values(pr.n_dofs, seed=11)
    x2 = meshgen.uniform_values(pr.n_dofs, seed=12)
    assert abs(x1 @ pr.mass(x2) - pr.mass(x1) @ x2) < 1e-14
    one = np.ones(pr.n_dofs)
    vol = pr.mass(one).sum()
    # volume of the terrain-following column mesh: sum over cells of |A| * mean height
    assert vol > 0.5 and one @ pr.mass(one) == pytest.approx(vol, rel=1e-14)


def test_dg1_block_diagonal():
    # DG1 x DG1: the mass matrix couples only the 6 DoFs of one prism.
    mesh = meshgen.tri_square(3)
    lam = 2
    pr = oracle.Problem(mesh, lam, "DG1", meshgen.extruded_vertex_coords(mesh, lam))
    x = np.zeros(pr.n_dofs)
    row = pr.num_v.lmap[4] + 1 * pr.num_v.offsets
    x[row[2]] = 1.0
    y = pr.mass(x)
    nz = np.nonzero(y)[0]
    assert set(nz) <= set(row)


def test_cubic_constant_fields():
    # u = c, f = d  =>  F_i = (c^3 - d) integral(v_i)
    mesh = meshgen.tri_square(4)
    lam = 3
    pr = oracle.Problem(mesh, lam, "P1", meshgen.extruded_vertex_coords(mesh, lam, terrain=0.2))
    c, d = 0.7, -0.3
    F = pr.cubic(np.full(pr.n_dofs, c), np.full(pr.n_dofs, d))
    ref = (c ** 3 - d) * pr.mass(np.ones(pr.n_dofs))
    np.testing.assert_allclose(F, ref, rtol=1e-13, atol=1e-16)


def test_cubic_integral_closed_form():
    # u = x, f = z on the unit cube: integral(x^3 - z) = 1/4 - 1/2.
    mesh = meshgen.tri_square(6)
    lam = 4
    pr = oracle.Problem(mesh, lam, "P1", meshgen.extruded_vertex_coords(mesh, lam))
    u = _interp(pr, lambda x, y, z: x)
    f = _interp(pr, lambda x, y, z: z)
    # u^3 is not in P1, but the oracle integrates u_h^3 exactly; u_h = x exactly
    assert abs(pr.cubic(u, f).sum() - (0.25 - 0.5)) < 1e-13


def test_cubic_vjp_dot_product_and_fd():
    mesh = meshgen.tri_square(4)
    lam = 3
    pr = oracle.Problem(mesh, lam, "P1", meshgen.extruded_vertex_coords(mesh, lam, terrain=0.2))
    n = pr.n_dofs
    u = meshgen.uniform_values(n, seed=21)
    f = meshgen.uniform_values(n, seed=22)
    w = meshgen.uniform_values(n, seed=23)
    du = meshgen.uniform_values(n, seed=24)
    df = meshgen.uniform_values(n, seed=25)
    gu, gf = pr.cubic_vjp(u, w)
    # dot-product test against the independent linearisation
    lhs = w @ pr.cubic_jvp(u, du, df)
    rhs = gu @ du + gf @ df
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))
    # g_f = -M w
    np.testing.assert_allclose(gf, -pr.mass(w), rtol=1e-13, atol=1e-16)
    # central finite differences, h = 1e-6
    h = 1e-6
    fd_u = (w @ pr.cubic(u + h * du, f) - w @ pr.cubic(u - h * du, f)) / (2 * h)
    fd_f = (w @ pr.cubic(u, f + h * df) - w @ pr.cubic(u, f - h * df)) / (2 * h)
    assert abs(fd_u - gu @ du) <= 1e-6 * abs(gu @ du)
    assert abs(fd_f - gf @ df) <= 1e-6 * abs(gf @ df)
    # the fused form gives the same three vectors
    F2, gu2, gf2 = pr.cubic_fused(u, f, w)
    np.testing.assert_allclose(F2, pr.cubic(u, f), rtol=0, atol=1e-15)
    np.testing.assert_allclose(gu2, gu, rtol=0, atol=1e-15)
    np.testing.assert_allclose(gf2, gf, rtol=0, atol=1e-15)


def test_subset_iteration_matches_full():
    # Running Algorithm 3 over a subset of columns gives the full result on
    # every DoF whose support lies inside the subset.
    mesh = meshgen.tri_square(5)
    lam = 3
    pr = oracle.Problem(mesh, lam, "P1", meshgen.extruded_vertex_coords(mesh, lam))
    f = meshgen.uniform_values(pr.n_dofs)
    full = pr.mass(f)
    v = 17
    cells = np.nonzero((mesh.cell_vertex == v).any(axis=1))[0]
    part = pr.mass(f, cells=cells)
    S = pr.num_v.column_starts(0)[v]
    np.testing.assert_array_equal(part[S:S + lam + 1], full[S:S + lam + 1])


@pytest.mark.parametrize("space", ["P1", "DG0", ("CG1", "DG0"), ("DG1", "CG1"), "P2"])
def test_variable_layers_mass_matches_exact_rationals(space):
    mesh = meshgen.tri_square(3, jitter=0.2)
    lam = 5
    rng = np.random.default_rng(21)
    layers = np.stack([rng.integers(0, 3, mesh.n_cells), lam - rng.integers(0, 3, mesh.n_cells)], 1).astype(np.int32)
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=0.3)
    pr = oracle.Problem(mesh, lam, space, vc, layers=layers)
    f = meshgen.uniform_values(pr.n_dofs, seed=8)
    got = pr.mass(f)
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, lam, oracle.delta_table(*pr.space), layers)
    exact = bruteforce.exact_mass(mesh, vc, lam, pr.space, stencils, n, f)
    _rel_close(got, exact)
    # the sum of the residual of f = 1 is the volume of the prisms present
    ones = pr.mass(np.ones(pr.n_dofs))
    xy = mesh.xy
    vol = 0.0
    for c in range(mesh.n_cells):
        a, b, d = mesh.cell_vertex[c]
        twoA = abs((xy[b, 0] - xy[a, 0]) * (xy[d, 1] - xy[a, 1]) - (xy[d, 0] - xy[a, 0]) * (xy[b, 1] - xy[a, 1]))
        for l in range(layers[c, 0], layers[c, 1]):
            h = [vc[v, l + 1, 2] - vc[v, l, 2] for v in (a, b, d)]
            vol += twoA * sum(h) / 6.0
    assert abs(ones.sum() - vol) < 1e-13
