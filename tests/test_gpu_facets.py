"""Parity of the horizontal-facet loop (Algorithm 3 with d2 = 0, lambda + 1
facets per column) and its jump form with the oracle."""
import numpy as np
import pytest

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import Case, assert_close, say

pytestmark = pytest.mark.gpu

FACET_SPACES = ["DG0", "DG1", "DG0xDG1", "DG1xDG0", "CG1xDG0", "CG1xDG1"]
SHAPES = [(4, 3), (5, 1), (3, 70), (6, 63), (2, 64)]


def _facets(c, x, y0=None, **opts):
    xd = c.dev(x)
    y = c.V.zeros() if y0 is None else c.dev(y0)
    acc = c.out_access() if y0 is None else exm.EXM_INC
    exm.par_loop(exm.EXM_K_FACET_JUMP, c.mesh, c.X, c.Vx, [(xd, c.V, exm.EXM_READ), (y, c.V, acc)], **opts)
    return c.host(y)


@pytest.mark.parametrize("space", FACET_SPACES)
@pytest.mark.parametrize("n,lam", SHAPES)
@pytest.mark.parametrize("race", [exm.EXM_RACE_ATOMIC, exm.EXM_RACE_COLOUR])
@pytest.mark.parametrize("cpw", [0, 1, 3, 16])
def test_facet_jump_matches_oracle(space, n, lam, race, cpw):
    say(f"facets {space} n={n} lam={lam} race={race} cpw={cpw}")
    c = Case(meshgen.tri_square(n), lam, space, terrain=0.3)
    x = meshgen.uniform_values(c.n, seed=41)
    got = _facets(c, x, race=race, cols_per_wave=cpw)
    assert_close(got, c.ref.facet_jump(x), c.ref.facet_jump_abs(x), what=f"facet jump {space}")


@pytest.mark.parametrize("space", FACET_SPACES)
def test_facet_jump_inc_accumulates(space):
    c = Case(meshgen.tri_square(5), 7, space, terrain=0.1)
    x = meshgen.uniform_values(c.n, seed=42)
    y0 = meshgen.uniform_values(c.n, seed=43)
    got = _facets(c, x, y0=y0)
    assert_close(got, c.ref.facet_jump(x) + y0, c.ref.facet_jump_abs(x) + np.abs(y0), what=f"INC {space}")


def test_facet_jump_autotuned_and_refusals():
    c = Case(meshgen.tri_square(6), 10, "DG1", terrain=0.2)
    x = c.dev(meshgen.uniform_values(c.n, seed=44))
    y = c.V.zeros()
    args = [(x, c.V, exm.EXM_READ), (y, c.V, exm.EXM_WRITE)]
    cfg = exm.autotune(exm.EXM_K_FACET_JUMP, c.mesh, c.X, c.Vx, args)
    assert cfg["schedule"] == exm.EXM_SCHED_DIRECT
    exm.par_loop(exm.EXM_K_FACET_JUMP, c.mesh, c.X, c.Vx, args, **cfg)
    xh = c.host(x)
    assert_close(c.host(y), c.ref.facet_jump(xh), c.ref.facet_jump_abs(xh), what="autotuned facets")
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_FACET_JUMP, c.mesh, c.X, c.Vx, args, race=exm.EXM_RACE_OWNER)
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED
    p1 = Case(meshgen.tri_square(4), 3, "P1", with_oracle=False)
    z = p1.V.zeros()
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_FACET_JUMP, p1.mesh, p1.X, p1.Vx, [(p1.V.zeros(), p1.V, exm.EXM_READ),
                                                                  (z, p1.V, exm.EXM_INC)])
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED
    base = meshgen.tri_square(4)
    v = Case(base, 5, "DG0", layers=meshgen.layer_ranges(base, 5, "random"), with_oracle=False)
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_FACET_JUMP, v.mesh, v.X, v.Vx, [(v.V.zeros(), v.V, exm.EXM_READ),
                                                               (v.V.zeros(), v.V, exm.EXM_WRITE)])
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED
