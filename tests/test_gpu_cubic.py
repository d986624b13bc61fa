"""Parity of the cubic residual, its vector-Jacobian product and the fused
forward+adjoint kernel with the oracle."""
import numpy as np
import pytest

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import Case, assert_close, say

pytestmark = pytest.mark.gpu

OPTS = [dict(schedule=exm.EXM_SCHED_DIRECT, race=exm.EXM_RACE_ATOMIC),
        dict(schedule=exm.EXM_SCHED_DIRECT, race=exm.EXM_RACE_COLOUR, cols_per_wave=3),
        dict(schedule=exm.EXM_SCHED_TILED, race=exm.EXM_RACE_ATOMIC),
        dict(schedule=exm.EXM_SCHED_TILED, race=exm.EXM_RACE_COLOUR, tile_cells=24, cols_per_wave=3),
        dict(schedule=exm.EXM_SCHED_STAGED, race=exm.EXM_RACE_ATOMIC, tile_cells=40, chunk_layers=16),
        dict(schedule=exm.EXM_SCHED_STAGED, race=exm.EXM_RACE_COLOUR, tile_cells=16, chunk_layers=8),
        dict(schedule=exm.EXM_SCHED_PIPELINED, race=exm.EXM_RACE_ATOMIC),
        dict(schedule=exm.EXM_SCHED_PIPELINED, race=exm.EXM_RACE_COLOUR, tile_cells=16, chunk_layers=16),
        dict(schedule=exm.EXM_SCHED_PIPELINED, race=exm.EXM_RACE_ATOMIC, tile_cells=8, chunk_layers=8)]


def _run(c, kernel, ins, nout, **opts):
    dev_in = [c.dev(x) for x in ins]
    outs = [c.V.zeros() for _ in range(nout)]
    fields = [(d, c.V, exm.EXM_READ) for d in dev_in] + [(o, c.V, exm.EXM_INC) for o in outs]
    exm.par_loop(kernel, c.mesh, c.X, c.Vx, fields, **opts)
    return [c.host(o) for o in outs]


@pytest.mark.parametrize("opts", OPTS)
# heights with a last chunk shorter than the chunk length (its top level
# written by the chunk's own items) and one that fills it (16 layers)
@pytest.mark.parametrize("n,lam,terrain", [(8, 10, 0.0), (6, 33, 0.3), (3, 1, 0.0), (5, 70, 0.1), (4, 16, 0.2)])
def test_cubic_forward_vjp_fused(opts, n, lam, terrain):
    say(f"cubic n={n} lam={lam} opts={opts}")
    base = meshgen.tri_square(n)
    c = Case(base, lam, "P1", terrain=terrain)
    u = meshgen.uniform_values(c.n, seed=31)
    f = meshgen.uniform_values(c.n, seed=32)
    w = meshgen.uniform_values(c.n, seed=meshgen.SEED_COTAN)
    F_ref = c.ref.cubic(u, f)
    F_scale = c.ref.cubic_abs(u, f)
    gu_ref, gf_ref = c.ref.cubic_vjp(u, w)
    gu_scale, gf_scale = c.ref.vjp_abs(u, w)
    (F,) = _run(c, exm.EXM_K_CUBIC, [u, f], 1, **opts)
    assert_close(F, F_ref, F_scale, what="cubic F")
    gu, gf = _run(c, exm.EXM_K_CUBIC_VJP, [u, w], 2, **opts)
    assert_close(gu, gu_ref, gu_scale, what="vjp g_u")
    assert_close(gf, gf_ref, gf_scale, what="vjp g_f")
    F2, gu2, gf2 = _run(c, exm.EXM_K_CUBIC_FUSED, [u, f, w], 3, **opts)
    assert_close(F2, F_ref, F_scale, what="fused F")
    assert_close(gu2, gu_ref, gu_scale, what="fused g_u")
    assert_close(gf2, gf_ref, gf_scale, what="fused g_f")


@pytest.mark.parametrize("race", [exm.EXM_RACE_ATOMIC, exm.EXM_RACE_COLOUR])
@pytest.mark.parametrize("chunk", [8, 16])
@pytest.mark.parametrize("extra", [5, 0])
def test_cubic_pipelined_inc_into_nonzero(race, chunk, extra):
    # INC: the pipelined write-back adds the old output values it loaded one
    # chunk ahead; outputs start from random values here (a ragged last chunk,
    # whose top level the chunk's items write, and a full one)
    say(f"cubic pipelined INC race={race} chunk={chunk} extra={extra}")
    base = meshgen.tri_square(9, order="random")
    c = Case(base, 2 * chunk + extra, "P1", terrain=0.2)
    u = meshgen.uniform_values(c.n, seed=41)
    f = meshgen.uniform_values(c.n, seed=42)
    w = meshgen.uniform_values(c.n, seed=43)
    y0 = [meshgen.uniform_values(c.n, seed=50 + i) for i in range(3)]
    outs = [c.dev(y) for y in y0]
    fields = [(c.dev(x), c.V, exm.EXM_READ) for x in (u, f, w)] + [(o, c.V, exm.EXM_INC) for o in outs]
    exm.par_loop(exm.EXM_K_CUBIC_FUSED, c.mesh, c.X, c.Vx, fields, schedule=exm.EXM_SCHED_PIPELINED, race=race,
                 chunk_layers=chunk, tile_cells=256 // chunk)
    F_ref, gu_ref, gf_ref = c.ref.cubic(u, f), *c.ref.cubic_vjp(u, w)
    F_scale, (gu_scale, gf_scale) = c.ref.cubic_abs(u, f), c.ref.vjp_abs(u, w)
    for got, ref, scale, y, what in ((outs[0], F_ref, F_scale, y0[0], "F"), (outs[1], gu_ref, gu_scale, y0[1], "g_u"),
                                     (outs[2], gf_ref, gf_scale, y0[2], "g_f")):
        assert_close(c.host(got), ref + y, scale + np.abs(y), what=f"pipelined INC {what}")


def test_cubic_pipelined_refuses_owner_and_bad_chunks():
    c = Case(meshgen.tri_square(5), 9, "P1", with_oracle=False)
    x = c.dev(meshgen.uniform_values(c.n, seed=1))
    fields = [(x, c.V, exm.EXM_READ), (x, c.V, exm.EXM_READ), (c.V.zeros(), c.V, exm.EXM_INC)]
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_CUBIC, c.mesh, c.X, c.Vx, fields, race=exm.EXM_RACE_OWNER)
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_CUBIC, c.mesh, c.X, c.Vx, fields, schedule=exm.EXM_SCHED_PIPELINED, chunk_layers=32)
    assert e.value.status == exm._abi.EXM_ERANGE
