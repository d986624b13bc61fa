"""Pins of the oracle's horizontal-facet loop (Algorithm 3 with d2 = 0:
lambda + 1 facets per column) and its jump form: closed forms per facet with
explicit prism enumeration, symmetry and positivity, and the vanishing of
interior jumps for a vertically continuous field."""
import numpy as np
import pytest

import oracle
from paper_1604_05937_amd import meshgen
from tests import bruteforce

# stencil position -> (horizontal node a, vertical node b) for the spaces
# that are discontinuous across levels (per entity: bottom, top, vertical
# DoFs; several DoFs on one entity horizontal-node major)
NODES = {
    "DG0": lambda p: (0, 0),
    "DG1": lambda p: (p // 2, p % 2),
    "DG0xDG1": lambda p: (0, p),
    "DG1xDG0": lambda p: (p, 0),
    "CG1xDG0": lambda p: (p, 0),
    "CG1xDG1": lambda p: (p // 2, p % 2),
}
HORIZONTAL_P1 = {"DG1", "DG1xDG0", "CG1xDG0", "CG1xDG1"}
VERTICAL_DG1 = {"DG1", "DG0xDG1", "CG1xDG1"}


def facet_area(mesh, vc, c, l):
    P = vc[mesh.cell_vertex[c], l, :]
    return 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))


def reference_jump(space, mesh, vc, lam, x):
    """The jump form facet by facet: closed-form facet mass (the facet is a
    flat triangle), prisms and DoFs by brute-force enumeration."""
    pr_space = oracle.SPACES[space]
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, lam, oracle.delta_table(*pr_space))
    y = np.zeros(n)
    nodes = NODES[space]
    vdg1 = space in VERTICAL_DG1

    def psi(b, zeta):   # vertical basis at the bottom (0) / top (1) face of a prism
        return (zeta if b == 1 else 1.0 - zeta) if vdg1 else 1.0

    for c in range(mesh.n_cells):
        for l in range(lam + 1):
            A = facet_area(mesh, vc, c, l)
            Mh = A * (np.eye(3) + 1.0) / 12.0 if space in HORIZONTAL_P1 else np.array([[A]])
            lo = stencils.get((c, l - 1))
            hi = stencils.get((c, l))
            k = len(lo if lo is not None else hi)
            ab = [nodes(p) for p in range(k)]
            # nodal jump on the facet, per horizontal node
            nh = Mh.shape[0]
            j = np.zeros(nh)
            for p, (a, b) in enumerate(ab):
                if lo is not None:
                    j[a] += psi(b, 1.0) * x[lo[p]]
                if hi is not None:
                    j[a] -= psi(b, 0.0) * x[hi[p]]
            r = Mh @ j
            for p, (a, b) in enumerate(ab):
                if lo is not None:
                    y[lo[p]] += psi(b, 1.0) * r[a]
                if hi is not None:
                    y[hi[p]] -= psi(b, 0.0) * r[a]
    return y


@pytest.mark.parametrize("space", list(NODES))
@pytest.mark.parametrize("lam,terrain", [(1, 0.0), (4, 0.0), (5, 0.3)])
def test_facet_jump_matches_closed_form(space, lam, terrain):
    mesh = meshgen.tri_square(3, jitter=0.2)
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=terrain)
    pr = oracle.Problem(mesh, lam, space, vc)
    x = meshgen.uniform_values(pr.n_dofs, seed=31)
    got = pr.facet_jump(x)
    ref = reference_jump(space, mesh, vc, lam, x)
    assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


def test_dg0_is_the_vertical_second_difference_times_the_facet_areas():
    mesh = meshgen.tri_square(4, jitter=0.2)
    lam = 6
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=0.4)
    pr = oracle.Problem(mesh, lam, "DG0", vc)
    x = meshgen.uniform_values(pr.n_dofs, seed=32)
    y = pr.facet_jump(x)
    for c in range(mesh.n_cells):
        col = x[pr.num_v.lmap[c, 0]:pr.num_v.lmap[c, 0] + lam]
        ext = np.concatenate([[0.0], col, [0.0]])
        A = np.array([facet_area(mesh, vc, c, l) for l in range(lam + 1)])
        want = A[:-1] * (ext[1:-1] - ext[:-2]) + A[1:] * (ext[1:-1] - ext[2:])
        np.testing.assert_allclose(y[pr.num_v.lmap[c, 0]:pr.num_v.lmap[c, 0] + lam], want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("space", list(NODES))
def test_facet_form_is_symmetric_and_positive(space):
    mesh = meshgen.tri_square(3)
    vc = meshgen.extruded_vertex_coords(mesh, 4, terrain=0.2)
    pr = oracle.Problem(mesh, 4, space, vc)
    a = meshgen.uniform_values(pr.n_dofs, seed=33)
    b = meshgen.uniform_values(pr.n_dofs, seed=34)
    assert abs(a @ pr.facet_jump(b) - b @ pr.facet_jump(a)) < 1e-14
    assert a @ pr.facet_jump(a) > 0.0
    assert (pr.facet_jump_abs(a) >= np.abs(pr.facet_jump(a)) - 1e-16).all()


def test_continuous_field_has_only_boundary_terms():
    # DG1 x DG1 values sampled from a P1 x P1 field: the interior jumps vanish,
    # and the bottom and top facets give the facet mass of the field
    mesh = meshgen.tri_square(3)
    lam = 5
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=0.3)
    pr = oracle.Problem(mesh, lam, "DG1", vc)
    g = meshgen.uniform_values(mesh.n_vertices * (lam + 1), seed=35).reshape(mesh.n_vertices, lam + 1)
    x = np.zeros(pr.n_dofs)
    for c in range(mesh.n_cells):
        for l in range(lam):
            for p in range(6):
                a, b = p // 2, p % 2
                x[pr.num_v.lmap[c, p] + 6 * l] = g[mesh.cell_vertex[c, a], l + b]
    y = pr.facet_jump(x)
    for c in range(mesh.n_cells):
        for l in range(lam):
            for p in range(6):
                a, b = p // 2, p % 2
                i = pr.num_v.lmap[c, p] + 6 * l
                if (l == 0 and b == 0) or (l == lam - 1 and b == 1):
                    lev = 0 if l == 0 else lam
                    A = facet_area(mesh, vc, c, lev)
                    gv = g[mesh.cell_vertex[c], lev]
                    want = A * (gv.sum() + gv[a]) / 12.0
                    assert abs(y[i] - want) < 1e-15
                else:
                    assert abs(y[i]) < 1e-15
