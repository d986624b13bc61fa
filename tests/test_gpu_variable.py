"""Parity of meshes whose cell columns carry different layer ranges (the
constant layer count is only a simplification of the exposition, Section 3.1
and Section 5): Algorithm 1's numbering over every entity's own range, the
explicit lists of the bottom prisms and Algorithm 3's loop with a layer count
per column, against the oracle on the same seeded inputs."""
import numpy as np
import pytest

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import Case, assert_close, say

pytestmark = pytest.mark.gpu

ALL_SPACES = ["P1", "DG0", "DG1", "P2", "CG1xDG0", "CG1xDG1", "DG0xCG1", "DG0xDG1", "DG1xCG1", "DG1xDG0"]
# (n, lambda, kind): lambda = 1 (every range is [0, 1)), ranges that end
# inside one 64-lane step, and columns longer than one step
SHAPES = [(6, 1, "random"), (8, 10, "bathymetry"), (7, 10, "random"), (5, 70, "bathymetry"), (4, 130, "random")]
RACES = [exm.EXM_RACE_ATOMIC, exm.EXM_RACE_COLOUR]


def _case(n, lam, kind, space, terrain=0.25, order="rcm"):
    base = meshgen.tri_square(n, order=order)
    layers = meshgen.layer_ranges(base, lam, kind)
    return Case(base, lam, space, terrain=terrain, layers=layers)


@pytest.mark.parametrize("space", ALL_SPACES)
@pytest.mark.parametrize("n,lam,kind", SHAPES)
@pytest.mark.parametrize("order", ["rcm", "random"])
def test_variable_numbering_bit_exact(space, n, lam, kind, order):
    say(f"variable numbering {space} n={n} lam={lam} {kind} {order}")
    c = _case(n, lam, kind, space, order=order)
    ref = c.ref.num_v
    assert c.V.n_dofs == ref.n_dofs
    np.testing.assert_array_equal(c.V.offsets(), ref.offsets)
    np.testing.assert_array_equal(c.V.bottom_map().cpu().numpy(), ref.lmap.astype(np.int32))
    for d1 in range(3):
        lo, hi = c.mesh.entity_layers(d1)
        np.testing.assert_array_equal(lo, ref.lo[d1])
        np.testing.assert_array_equal(hi, ref.hi[d1])
        starts = c.V.column_starts(d1).cpu().numpy()
        if ref.first[d1] is None:
            assert np.all(starts == -1)
        else:
            np.testing.assert_array_equal(starts, ref.column_starts(d1).astype(np.int32))


@pytest.mark.parametrize("space", ALL_SPACES)
@pytest.mark.parametrize("n,lam,kind", SHAPES)
@pytest.mark.parametrize("race", RACES)
@pytest.mark.parametrize("cpw", [0, 1, 3, 8])
def test_variable_mass_parity(space, n, lam, kind, race, cpw):
    say(f"variable mass {space} n={n} lam={lam} {kind} race={race} cpw={cpw}")
    c = _case(n, lam, kind, space)
    x = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    got = c.mass(x, race=race, cols_per_wave=cpw)
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"variable mass {space}")


def test_variable_mass_integrates_the_present_prisms():
    # f = 1: the sum of the residual is the volume of the prisms the ranges keep
    c = _case(9, 12, "bathymetry", "P1", terrain=0.0)
    got = c.mass(np.ones(c.n))
    xy = c.base.xy
    vol = 0.0
    for cell, (b, t) in enumerate(c.layers):
        p, q, r = xy[c.base.cell_vertex[cell]]
        vol += 0.5 * abs((q[0] - p[0]) * (r[1] - p[1]) - (r[0] - p[0]) * (q[1] - p[1])) * (t - b) / 12.0
    assert abs(got.sum() - vol) < 1e-13


@pytest.mark.parametrize("n,lam,kind", [(8, 10, "bathymetry"), (5, 70, "random"), (6, 1, "random")])
@pytest.mark.parametrize("race", RACES)
def test_variable_cubic_forward_vjp_fused(n, lam, kind, race):
    say(f"variable cubic n={n} lam={lam} {kind} race={race}")
    c = _case(n, lam, kind, "P1", terrain=0.1)
    u = meshgen.uniform_values(c.n, seed=31)
    f = meshgen.uniform_values(c.n, seed=32)
    w = meshgen.uniform_values(c.n, seed=meshgen.SEED_COTAN)

    def run(kernel, ins, nout):
        dev_in = [c.dev(a) for a in ins]
        outs = [c.V.zeros() for _ in range(nout)]
        fields = [(d, c.V, exm.EXM_READ) for d in dev_in] + [(o, c.V, exm.EXM_INC) for o in outs]
        exm.par_loop(kernel, c.mesh, c.X, c.Vx, fields, race=race)
        return [c.host(o) for o in outs]

    (F,) = run(exm.EXM_K_CUBIC, [u, f], 1)
    assert_close(F, c.ref.cubic(u, f), c.ref.cubic_abs(u, f), what="variable cubic F")
    gu_ref, gf_ref = c.ref.cubic_vjp(u, w)
    gu_s, gf_s = c.ref.vjp_abs(u, w)
    F2, gu, gf = run(exm.EXM_K_CUBIC_FUSED, [u, f, w], 3)
    assert_close(F2, c.ref.cubic(u, f), c.ref.cubic_abs(u, f), what="variable fused F")
    assert_close(gu, gu_ref, gu_s, what="variable fused g_u")
    assert_close(gf, gf_ref, gf_s, what="variable fused g_f")


@pytest.mark.parametrize("space", ["P1", "DG0", "P2", "DG1xCG1"])
def test_full_ranges_match_the_uniform_mesh(space):
    # every cell over [0, lambda): same numbering and the same values as the
    # mesh built without ranges
    base = meshgen.tri_square(7)
    lam = 9
    layers = np.tile(np.array([0, lam], np.int32), (base.n_cells, 1))
    a = Case(base, lam, space, terrain=0.2, with_oracle=False)
    b = Case(base, lam, space, terrain=0.2, layers=layers)
    assert a.V.n_dofs == b.V.n_dofs
    np.testing.assert_array_equal(a.V.bottom_map().cpu().numpy(), b.V.bottom_map().cpu().numpy())
    x = meshgen.uniform_values(a.n, seed=5)
    ya = a.mass(x, race=exm.EXM_RACE_COLOUR)
    yb = b.mass(x, race=exm.EXM_RACE_COLOUR)
    assert_close(yb, ya, b.ref.mass_abs(x), what=f"full ranges {space}")


@pytest.mark.parametrize("schedule", [exm.EXM_SCHED_TILED, exm.EXM_SCHED_STAGED, exm.EXM_SCHED_PIPELINED])
def test_variable_mesh_any_schedule(schedule):
    # TILED and STAGED fall back to DIRECT; PIPELINED has a kernel of its own for P1
    c = _case(8, 10, "bathymetry", "P1")
    x = meshgen.uniform_values(c.n, seed=6)
    got = c.mass(x, schedule=schedule, tile_cells=64, chunk_layers=16)
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"variable P1, schedule {schedule}")


@pytest.mark.parametrize("n,lam,kind", SHAPES + [(6, 62, "random"), (5, 33, "bathymetry"), (9, 16, "random")])
@pytest.mark.parametrize("race", RACES)
@pytest.mark.parametrize("tile,chunk", [(64, 16), (29, 8), (8, 32), (32, 12)])
def test_variable_pipelined_p1(n, lam, kind, race, tile, chunk):
    # the tile pipeline on absolute levels: a window per tile, copies inside
    # each vertex's column, prisms only inside each cell's range; INC into
    # non-zero outputs exercises the old values loaded one chunk ahead
    say(f"variable pipelined P1 n={n} lam={lam} {kind} race={race} tile={tile} chunk={chunk}")
    c = _case(n, lam, kind, "P1", order="random" if tile == 29 else "rcm")
    x = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    y0 = meshgen.uniform_values(c.n, seed=71)
    xd, y = c.dev(x), c.dev(y0)
    fields = [(xd, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)]
    opts = dict(schedule=exm.EXM_SCHED_PIPELINED, race=race, tile_cells=tile, chunk_layers=chunk)
    try:
        cfg = exm.par_loop_config(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, fields, **opts)
        exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, fields, **opts)
    except exm.ExmError as e:
        # tiles too large for the chunk length are refused before any launch
        assert e.status == exm._abi.EXM_EUNSUPPORTED and "PIPELINED" in str(e), str(e)
        return
    assert cfg["schedule"] == exm.EXM_SCHED_PIPELINED
    assert_close(c.host(y), c.ref.mass(x) + y0, c.ref.mass_abs(x) + np.abs(y0), what="variable pipelined P1")


@pytest.mark.parametrize("n,lam,kind", SHAPES + [(6, 62, "random"), (5, 33, "bathymetry")])
@pytest.mark.parametrize("acc", ["write", "inc"])
@pytest.mark.parametrize("tile,chunk", [(32, 32), (64, 16), (29, 8), (8, 32)])
def test_variable_pipelined_dg0(n, lam, kind, acc, tile, chunk):
    # the DG0 tile pipeline on absolute levels: z copies inside each vertex's
    # column, each cell's layers loaded, evaluated and stored only inside its
    # range; outputs start non-zero, so WRITE must overwrite and INC add
    say(f"variable pipelined DG0 n={n} lam={lam} {kind} {acc} tile={tile} chunk={chunk}")
    c = _case(n, lam, kind, "DG0", order="random" if tile == 29 else "rcm")
    x = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    y0 = meshgen.uniform_values(c.n, seed=71)
    xd, y = c.dev(x), c.dev(y0)
    mode = exm.EXM_WRITE if acc == "write" else exm.EXM_INC
    fields = [(xd, c.V, exm.EXM_READ), (y, c.V, mode)]
    opts = dict(schedule=exm.EXM_SCHED_PIPELINED, race=exm.EXM_RACE_ATOMIC, tile_cells=tile, chunk_layers=chunk)
    try:
        cfg = exm.par_loop_config(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, fields, **opts)
        exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, fields, **opts)
    except exm.ExmError as e:
        # tiles too large for the chunk length are refused before any launch
        assert e.status == exm._abi.EXM_EUNSUPPORTED and "PIPELINED" in str(e), str(e)
        return
    assert cfg["schedule"] == exm.EXM_SCHED_PIPELINED
    want = c.ref.mass(x) + (y0 if acc == "inc" else 0.0)
    assert_close(c.host(y), want, c.ref.mass_abs(x) + np.abs(y0), what=f"variable pipelined DG0 {acc}")


@pytest.mark.parametrize("lam,expect", [(2000, "pipelined"), (2001, "direct")])
def test_variable_pipelined_layer_limit(lam, expect):
    # the pipelined kernel keeps chunk indices in 8 bits: up to 2000 layers it
    # runs, above that the loop falls back to DIRECT; both match the oracle
    say(f"variable pipelined P1 layer limit lam={lam}")
    c = _case(2, lam, "bathymetry", "P1")
    x = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    xd, y = c.dev(x), c.V.zeros()
    fields = [(xd, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)]
    opts = dict(schedule=exm.EXM_SCHED_PIPELINED, race=exm.EXM_RACE_ATOMIC, tile_cells=8, chunk_layers=8)
    cfg = exm.par_loop_config(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, fields, **opts)
    want = exm.EXM_SCHED_PIPELINED if expect == "pipelined" else exm.EXM_SCHED_DIRECT
    assert cfg["schedule"] == want
    exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, fields, **opts)
    assert_close(c.host(y), c.ref.mass(x), c.ref.mass_abs(x), what=f"variable P1, {lam} layers")


def test_variable_mesh_refuses_owner_computes():
    c = _case(6, 10, "random", "P1", terrain=0.0)
    x = c.dev(np.ones(c.n))
    y = c.V.zeros()
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(x, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)],
                     race=exm.EXM_RACE_OWNER)
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED


@pytest.mark.parametrize("space", ["P1", "CG1xDG0", "CG1xDG1"])
@pytest.mark.parametrize("n,lam,kind", SHAPES + [(6, 62, "random"), (5, 125, "bathymetry")])
@pytest.mark.parametrize("wpb", [1, 4])
def test_variable_gather(space, n, lam, kind, wpb):
    # the vertex-column schedule on columns of different heights: every
    # neighbour read at the same absolute level, prisms only inside the cell's range
    say(f"variable gather {space} n={n} lam={lam} {kind} wpb={wpb}")
    c = _case(n, lam, kind, space)
    x = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    cfg = exm.par_loop_config(exm.EXM_K_MASS, c.mesh, c.X, c.Vx,
                              [(c.dev(x), c.V, exm.EXM_READ), (c.V.zeros(), c.V, exm.EXM_INC)],
                              schedule=exm.EXM_SCHED_GATHER, waves_per_block=wpb)
    assert cfg["schedule"] == exm.EXM_SCHED_GATHER
    got = c.mass(x, schedule=exm.EXM_SCHED_GATHER, waves_per_block=wpb)
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"variable gather {space}")


@pytest.mark.parametrize("space", ["P1", "CG1xDG1"])
def test_variable_gather_checkerboard(space):
    base = meshgen.tri_checkerboard(5)
    lam = 9
    layers = meshgen.layer_ranges(base, lam, "random")
    c = Case(base, lam, space, terrain=0.2, layers=layers)
    x = meshgen.uniform_values(c.n, seed=63)
    got = c.mass(x, schedule=exm.EXM_SCHED_GATHER)
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"variable gather checkerboard {space}")
