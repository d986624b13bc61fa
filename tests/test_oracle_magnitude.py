"""Pins of the oracle's magnitude forms, which scale every componentwise
parity bound: the same integrals as the mass action, the cubic residual and
its adjoint (Section 4.1.1 and the derivative of the cubic form) with every
factor replaced by its absolute value.

Where every basis function is non-negative (P1, DG0, DG1 and the six mixed
{CG1, DG0, DG1} products), |phi| = phi, so a magnitude form is the plain form
of the absolute values and has an exact value: it is checked against exact
rational integration of tiny meshes (tests/bruteforce.py, no quadrature, no
oracle code).  P2 basis functions change sign, so |phi| is not a polynomial
and its magnitude form is a quadrature of |phi|; it is checked by the bounds
that make it a valid error scale."""
import numpy as np
import pytest

import oracle
from paper_1604_05937_amd import meshgen
from tests import bruteforce

NONNEG = ["P1", "DG0", "DG1", ("CG1", "DG0"), ("DG0", "CG1"), ("DG1", "CG1"), ("CG1", "DG1"), ("DG0", "DG1"),
          ("DG1", "DG0")]
ALL = NONNEG + ["P2"]


def _close_exact(got, exact, tol=1e-13):
    exact = np.array([float(x) for x in exact])
    assert got.shape == exact.shape
    err = np.abs(got - exact).max() / max(1e-300, np.abs(exact).max())
    assert err <= tol, err


def _problem(space, n=2, lam=2, terrain=0.3, seed=0):
    mesh = meshgen.tri_square(n, jitter=0.2, seed=seed)
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=terrain)
    return mesh, lam, vc, oracle.Problem(mesh, lam, space, vc)


@pytest.mark.parametrize("space", NONNEG)
@pytest.mark.parametrize("terrain", [0.0, 0.3])
def test_mass_abs_is_exact_mass_of_magnitudes(space, terrain):
    mesh, lam, vc, pr = _problem(space, n=3, terrain=terrain)
    x = meshgen.uniform_values(pr.n_dofs, seed=41)
    got = pr.mass_abs(x)
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, lam, oracle.delta_table(*pr.space))
    _close_exact(got, bruteforce.exact_mass(mesh, vc, lam, pr.space, stencils, n, np.abs(x)))


@pytest.mark.parametrize("space", ALL)
def test_mass_abs_bounds_every_term(space):
    # |sum of terms| <= sum of |terms|, componentwise, for any field; equality
    # for a field of one sign on the non-negative bases
    mesh, lam, vc, pr = _problem(space, n=4, lam=3)
    for seed in (42, 43):
        x = meshgen.uniform_values(pr.n_dofs, seed=seed)
        a = pr.mass_abs(x)
        assert np.all(a >= np.abs(pr.mass(x)) * (1 - 1e-14))
        assert np.all(a >= 0.0)
        # the magnitude form sees only |x|
        np.testing.assert_array_equal(a, pr.mass_abs(np.abs(x)))
        np.testing.assert_array_equal(a, pr.mass_abs(-x))


def test_p2_mass_abs_lebesgue_bounds():
    # sum_i |phi_i| lies in [1, 5/3 * 5/4] pointwise on P2 x P2 (the Lebesgue
    # constants of equispaced quadratic interpolation on the triangle and the
    # interval), so the magnitude form of x = 1 sums to between the volume and
    # (25/12)^2 times it; P1 (all phi >= 0, partition of unity) gives exactly
    # the volume
    for space, lo, hi in (("P2", 1.0, (25.0 / 12.0) ** 2), ("P1", 1.0, 1.0)):
        mesh, lam, vc, pr = _problem(space, n=4, lam=3, terrain=0.0)
        total = pr.mass_abs(np.ones(pr.n_dofs)).sum()
        assert lo * (1 - 1e-13) <= total <= hi * (1 + 1e-13), (space, total)
    # P2 basis functions change sign: the magnitude form is strictly larger
    mesh, lam, vc, pr = _problem("P2", n=4, lam=3, terrain=0.0)
    one = np.ones(pr.n_dofs)
    assert pr.mass_abs(one).sum() > pr.mass(one).sum() * (1 + 1e-3)


@pytest.mark.parametrize("terrain", [0.0, 0.3])
def test_cubic_abs_is_exact(terrain):
    # integral (|u|_h^3 + |f|_h) v_i = the cubic residual of (|u|, -|f|), exactly
    mesh, lam, vc, pr = _problem("P1", terrain=terrain)
    u = meshgen.uniform_values(pr.n_dofs, seed=44)
    f = meshgen.uniform_values(pr.n_dofs, seed=45)
    got = pr.cubic_abs(u, f)
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, lam, oracle.delta_table("CG1", "CG1"))
    _close_exact(got, bruteforce.exact_cubic(mesh, vc, lam, stencils, n, np.abs(u), -np.abs(f)))
    assert np.all(got >= np.abs(pr.cubic(u, f)) * (1 - 1e-14))


@pytest.mark.parametrize("terrain", [0.0, 0.3])
def test_vjp_and_vjp_abs_are_exact(terrain):
    mesh, lam, vc, pr = _problem("P1", terrain=terrain)
    u = meshgen.uniform_values(pr.n_dofs, seed=46)
    w = meshgen.uniform_values(pr.n_dofs, seed=47)
    n, _, stencils, _ = bruteforce.bruteforce_numbering(mesh, lam, oracle.delta_table("CG1", "CG1"))
    # the adjoint itself: g_u = integral 3 u^2 w v_i, g_f = -integral w v_i
    gu, gf = pr.cubic_vjp(u, w)
    _close_exact(gu, bruteforce.exact_cubic_vjp(mesh, vc, lam, stencils, n, u, w))
    _close_exact(gf, [-x for x in bruteforce.exact_mass(mesh, vc, lam, ("CG1", "CG1"), stencils, n, w)])
    # its magnitude form: the same integrals of |u| and |w|
    au, af = pr.vjp_abs(u, w)
    _close_exact(au, bruteforce.exact_cubic_vjp(mesh, vc, lam, stencils, n, np.abs(u), np.abs(w)))
    _close_exact(af, bruteforce.exact_mass(mesh, vc, lam, ("CG1", "CG1"), stencils, n, np.abs(w)))
    assert np.all(au >= np.abs(gu) * (1 - 1e-14))
    assert np.all(af >= np.abs(gf) * (1 - 1e-14))


def test_mixed_dg_mass_abs_is_mass_of_magnitudes():
    mesh = meshgen.tri_square(3, jitter=0.2)
    lam = 3
    vc = meshgen.extruded_vertex_coords(mesh, lam, terrain=0.2)
    nd = meshgen.cell_degrees(mesh, frac_dg1=0.5)
    x = meshgen.uniform_values(int(nd.sum()) * lam, seed=48)   # DG columns only: n_dofs = lambda * sum of cell counts
    a, _ = oracle.mixed_dg_mass(mesh, lam, vc, nd, x, absf=True)
    m, _ = oracle.mixed_dg_mass(mesh, lam, vc, nd, np.abs(x))
    np.testing.assert_allclose(a, m, rtol=1e-14, atol=0)
    assert np.all(a >= np.abs(oracle.mixed_dg_mass(mesh, lam, vc, nd, x)[0]) * (1 - 1e-14))
