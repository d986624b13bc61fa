"""Parity of the HIP path (through the C ABI) with the CPU oracle on seeded
inputs: numbering and lists bit-exact, FP64 values to the componentwise
tolerance of tests/gpu_common.py."""
import numpy as np
import pytest
import torch

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import RTOL, Case, assert_close, say

pytestmark = pytest.mark.gpu

# configs: (n, layers) -- 16x16 base x 10 layers is the tiny workload; the
# others cover lambda = 1, lambda not a multiple of any lane group, and more
# layers than one 64-lane step.
SHAPES = [(16, 10), (5, 1), (7, 63), (6, 65), (3, 130)]


ALL_SPACES = ["P1", "DG0", "DG1", "P2", "CG1xDG0", "CG1xDG1", "DG0xCG1", "DG0xDG1", "DG1xCG1", "DG1xDG0"]


@pytest.mark.parametrize("space", ALL_SPACES)
@pytest.mark.parametrize("n,lam", SHAPES)
@pytest.mark.parametrize("order", ["rcm", "random"])
def test_numbering_bit_exact(space, n, lam, order):
    say(f"numbering {space} n={n} lam={lam} {order}")
    base = meshgen.tri_square(n, order=order)
    c = Case(base, lam, space)
    ref = c.ref.num_v
    assert c.V.n_dofs == ref.n_dofs
    assert c.V.arity == ref.k
    np.testing.assert_array_equal(c.V.offsets(), ref.offsets)
    np.testing.assert_array_equal(c.V.bottom_map().cpu().numpy(), ref.lmap.astype(np.int32))
    for d1 in range(3):
        starts = c.V.column_starts(d1).cpu().numpy()
        if ref.first[d1] is None:
            assert np.all(starts == -1)
        else:
            np.testing.assert_array_equal(starts, ref.column_starts(d1).astype(np.int32))


SCHEDULES = [exm.EXM_SCHED_DIRECT, exm.EXM_SCHED_TILED, exm.EXM_SCHED_STAGED, exm.EXM_SCHED_PIPELINED,
             exm.EXM_SCHED_CHUNKED, exm.EXM_SCHED_GATHER]
RACES = [exm.EXM_RACE_ATOMIC, exm.EXM_RACE_COLOUR]


@pytest.mark.parametrize("space", ALL_SPACES)
@pytest.mark.parametrize("n,lam", SHAPES)
@pytest.mark.parametrize("race", RACES)
@pytest.mark.parametrize("schedule", SCHEDULES)
def test_mass_parity(space, n, lam, race, schedule):
    say(f"mass {space} n={n} lam={lam} race={race} schedule={schedule}")
    base = meshgen.tri_square(n)
    c = Case(base, lam, space, terrain=0.25)
    x = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    got = c.mass(x, race=race, schedule=schedule)
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"mass {space}")


@pytest.mark.parametrize("space", ["P1", "P2", "DG1", "DG0"])
@pytest.mark.parametrize("cpw", [1, 2, 3, 4, 5, 7, 8, 16])
@pytest.mark.parametrize("wpb", [1, 4])
def test_mass_direct_shapes(space, cpw, wpb):
    say(f"direct shape {space} cpw={cpw} wpb={wpb}")
    base = meshgen.tri_square(9)
    c = Case(base, 23, space)
    x = meshgen.uniform_values(c.n, seed=5)
    got = c.mass(x, schedule=exm.EXM_SCHED_DIRECT, cols_per_wave=cpw, waves_per_block=wpb)
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"mass {space} cpw={cpw}")


@pytest.mark.parametrize("space", ["P1", "P2", "DG1", "DG0"])
@pytest.mark.parametrize("tile", [8, 17, 64, 300])
@pytest.mark.parametrize("cpw", [0, 1, 3, 8])
@pytest.mark.parametrize("race", RACES)
def test_mass_tiled_shapes(space, tile, cpw, race):
    say(f"tiled shape {space} tile={tile} cpw={cpw} race={race}")
    base = meshgen.tri_square(11, order="random" if tile == 17 else "rcm")
    c = Case(base, 23, space, terrain=0.2)
    x = meshgen.uniform_values(c.n, seed=6)
    try:
        got = c.mass(x, schedule=exm.EXM_SCHED_TILED, tile_cells=tile, cols_per_wave=cpw, race=race,
                     waves_per_block=2 if cpw == 3 else 0)
    except exm.ExmError as e:
        # a tile whose per-level sums exceed LDS is refused before any launch
        assert e.status == exm._abi.EXM_EUNSUPPORTED and "LDS" in str(e) and cpw in (1, 3), str(e)
        return
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"tiled mass {space} tile={tile} cpw={cpw}")


@pytest.mark.parametrize("space", ["P1", "DG1", "DG0"])
@pytest.mark.parametrize("tile", [8, 29, 128])
@pytest.mark.parametrize("chunk", [8, 16, 32, 64])
@pytest.mark.parametrize("race", RACES)
def test_mass_staged_shapes(space, tile, chunk, race):
    say(f"staged shape {space} tile={tile} chunk={chunk} race={race}")
    base = meshgen.tri_square(10, order="random" if tile == 29 else "rcm")
    for lam in (chunk - 1, chunk, 2 * chunk + 3):
        c = Case(base, lam, space, terrain=0.2)
        x = meshgen.uniform_values(c.n, seed=7)
        try:
            got = c.mass(x, schedule=exm.EXM_SCHED_STAGED, tile_cells=tile, chunk_layers=chunk, race=race)
        except exm.ExmError as e:
            # tiles too large for the chunk length are refused before any launch
            assert e.status == exm._abi.EXM_EUNSUPPORTED and tile * chunk > 1024, str(e)
            return
        assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"staged mass {space} tile={tile} S={chunk} lam={lam}")


@pytest.mark.parametrize("schedule", [exm.EXM_SCHED_PIPELINED, exm.EXM_SCHED_CHUNKED])
@pytest.mark.parametrize("space", ["P1", "P2", "DG0", "DG1", "DG0xDG1", "DG1xDG0", "DG0xCG1", "DG1xCG1", "CG1xDG0",
                                   "CG1xDG1"])
@pytest.mark.parametrize("tile", [8, 29, 64, 128])
@pytest.mark.parametrize("chunk", [8, 12, 16, 20, 24, 32])
@pytest.mark.parametrize("race", RACES + [exm.EXM_RACE_OWNER])
def test_mass_pipelined_shapes(schedule, space, tile, chunk, race):
    say(f"pipelined shape {space} schedule={schedule} tile={tile} chunk={chunk} race={race}")
    base = meshgen.tri_square(10, order="random" if tile == 29 else "rcm")
    for lam in (1, chunk - 1, chunk, 2 * chunk + 3):
        c = Case(base, lam, space, terrain=0.2)
        x = meshgen.uniform_values(c.n, seed=7)
        y0 = meshgen.uniform_values(c.n, seed=8)
        xd, y = c.dev(x), c.dev(y0)
        try:
            exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(xd, c.V, exm.EXM_READ), (y, c.V, c.out_access())],
                         schedule=schedule, tile_cells=tile, chunk_layers=chunk, race=race)
        except exm.ExmError as e:
            # tiles too large for the chunk length, and chunk lengths a schedule or
            # space does not take, are refused before any launch
            big = e.status == exm._abi.EXM_EUNSUPPORTED and ("PIPELINED" in str(e) or "CHUNKED" in str(e))
            odd = e.status == exm._abi.EXM_ERANGE and (
                (chunk in (12, 20, 24) and (space != "P1" or schedule != 4)) or (chunk == 32 and space in ("P2", "CG1xDG0", "CG1xDG1")))
            assert big or odd, str(e)
            return
        if c.out_access() == exm.EXM_INC:
            # INC into a non-zero output: the old values pass through the staged copy
            want, scale = c.ref.mass(x) + y0, c.ref.mass_abs(x) + np.abs(y0)
        else:   # WRITE overwrites
            want, scale = c.ref.mass(x), c.ref.mass_abs(x)
        assert_close(c.host(y), want, scale, what=f"pipelined mass {space} tile={tile} S={chunk} lam={lam}")


@pytest.mark.parametrize("tile,chunk", [(8, 16), (32, 16), (48, 16), (96, 16), (128, 16), (192, 16), (256, 8),
                                        (96, 8), (64, 32), (48, 32)])
@pytest.mark.parametrize("race", RACES + [exm.EXM_RACE_OWNER])
def test_p1_pipelined_workgroup_widths(tile, chunk, race):
    # the fixed-height P1 tile walk in workgroups of 128 to 512 threads (one
    # pass over the tile's cells) and two passes of 512
    say(f"P1 pipelined width tile={tile} chunk={chunk} race={race}")
    base = meshgen.tri_square(14)
    for lam in (1, chunk - 1, 2 * chunk + 3):
        c = Case(base, lam, "P1", terrain=0.2)
        x = meshgen.uniform_values(c.n, seed=17)
        y0 = meshgen.uniform_values(c.n, seed=18)
        xd, y = c.dev(x), c.dev(y0)
        try:
            exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(xd, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)],
                         schedule=exm.EXM_SCHED_PIPELINED, tile_cells=tile, chunk_layers=chunk, race=race)
        except exm.ExmError as e:
            # more vertices than the widest workgroup's items take: refused before any launch
            assert e.status == exm._abi.EXM_EUNSUPPORTED and "PIPELINED" in str(e), str(e)
            assert tile * chunk >= 2048, str(e)
            return
        assert_close(c.host(y), c.ref.mass(x) + y0, c.ref.mass_abs(x) + np.abs(y0),
                     what=f"P1 pipelined tile={tile} S={chunk} lam={lam}")


@pytest.mark.parametrize("space", ["DG0", "DG1", "DG0xDG1", "DG1xDG0", "DG0xCG1", "DG1xCG1"])
def test_pipelined_dg_inc(space):
    base = meshgen.tri_square(7)
    c = Case(base, 19, space)
    x = meshgen.uniform_values(c.n, seed=9)
    y0 = meshgen.uniform_values(c.n, seed=10)
    xd, y = c.dev(x), c.dev(y0)
    exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(xd, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)],
                 schedule=exm.EXM_SCHED_PIPELINED, chunk_layers=8)
    assert_close(c.host(y), c.ref.mass(x) + y0, c.ref.mass_abs(x) + np.abs(y0), what=f"pipelined {space} INC")


@pytest.mark.parametrize("chunk,tile", [(20, 16), (20, 32), (20, 50), (26, 24), (26, 38), (34, 16), (34, 24),
                                        (34, 30)])
def test_pipelined_dg0_long_chunks(chunk, tile):
    # DG0xDG0 on columns of one height takes chunks of 20, 26 or 34 layers
    # (20, 50 and 100 layers in one, two and three steps); a single layer, one
    # short of a chunk, one chunk, one over, a ragged height and 100 layers
    say(f"DG0 pipelined {chunk}-layer chunks tile={tile}")
    base = meshgen.tri_square(9)
    for lam in (1, chunk - 1, chunk, chunk + 1, 2 * chunk + 3, 100):
        c = Case(base, lam, "DG0", terrain=0.2)
        x = meshgen.uniform_values(c.n, seed=23)
        y0 = meshgen.uniform_values(c.n, seed=24)
        xd, y = c.dev(x), c.dev(y0)
        exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(xd, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)],
                     schedule=exm.EXM_SCHED_PIPELINED, tile_cells=tile, chunk_layers=chunk)
        assert_close(c.host(y), c.ref.mass(x) + y0, c.ref.mass_abs(x) + np.abs(y0),
                     what=f"DG0 pipelined tile={tile} S={chunk} lam={lam}")
        got = c.mass(x, schedule=exm.EXM_SCHED_PIPELINED, tile_cells=tile, chunk_layers=chunk)
        assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"DG0 pipelined WRITE tile={tile} S={chunk} lam={lam}")


@pytest.mark.parametrize("chunk", [20, 26, 34])
def test_pipelined_long_chunks_only_on_dg0(chunk):
    # other spaces, and DG0 on columns of different heights, refuse them
    # before any launch
    c = Case(meshgen.tri_square(4), 10, "DG1")
    x = meshgen.uniform_values(c.n, seed=25)
    with pytest.raises(exm.ExmError) as e:
        c.mass(x, schedule=exm.EXM_SCHED_PIPELINED, tile_cells=16, chunk_layers=chunk)
    assert e.value.status == exm._abi.EXM_ERANGE, str(e.value)
    base = meshgen.tri_square(4)
    v = Case(base, 10, "DG0", layers=meshgen.layer_ranges(base, 10, "random"))
    with pytest.raises(exm.ExmError) as e:
        v.mass(meshgen.uniform_values(v.n, seed=26), schedule=exm.EXM_SCHED_PIPELINED, tile_cells=16,
               chunk_layers=chunk)
    assert e.value.status == exm._abi.EXM_ERANGE and "one height" in str(e.value), str(e.value)


@pytest.mark.parametrize("n,lam", SHAPES)
def test_owner_computes_matches_oracle(n, lam):
    say(f"owner computes n={n} lam={lam}")
    c = Case(meshgen.tri_square(n, order="random"), lam, "P1", terrain=0.3)
    x = meshgen.uniform_values(c.n, seed=11)
    got = c.mass(x, race=exm.EXM_RACE_OWNER)
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what="owner-computes P1")
    cfg = exm.par_loop_config(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(c.dev(x), c.V, exm.EXM_READ),
                                                                 (c.V.zeros(), c.V, exm.EXM_INC)],
                              race=exm.EXM_RACE_OWNER)
    assert cfg["schedule"] == exm.EXM_SCHED_PIPELINED and cfg["race"] == exm.EXM_RACE_OWNER


@pytest.mark.parametrize("space", ["CG1xDG0", "CG1xDG1", "DG0xCG1", "DG1xCG1"])
def test_shared_spaces_refuse_write(space):
    c = Case(meshgen.tri_square(4), 3, space, with_oracle=False)
    x = c.dev(meshgen.uniform_values(c.n, seed=1))
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(x, c.V, exm.EXM_READ), (c.V.zeros(), c.V, exm.EXM_WRITE)])
    assert e.value.status == exm._abi.EXM_EINVAL


@pytest.mark.parametrize("space", ["CG1xDG0", "DG1xCG1"])
def test_tensor_spaces_direct_shapes(space):
    c = Case(meshgen.tri_square(9), 23, space, terrain=0.3)
    x = meshgen.uniform_values(c.n, seed=12)
    for cpw in (1, 2, 3, 5, 16):
        got = c.mass(x, schedule=exm.EXM_SCHED_DIRECT, cols_per_wave=cpw)
        assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"{space} cpw={cpw}")


def test_owner_computes_unsupported_on_p2():
    c = Case(meshgen.tri_square(4), 3, "P2", with_oracle=False)
    x = c.dev(meshgen.uniform_values(c.n, seed=1))
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(x, c.V, exm.EXM_READ), (c.V.zeros(), c.V, exm.EXM_INC)],
                     race=exm.EXM_RACE_OWNER)
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED


def test_pipelined_needs_aligned_pointers():
    base = meshgen.tri_square(6)
    c = Case(base, 9, "P1", with_oracle=False)
    buf = c.torch.zeros(c.n + 1, dtype=c.torch.float64, device="cuda")
    x = buf[1:]   # 8-byte aligned only
    y = c.V.zeros()
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(x, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)],
                     schedule=exm.EXM_SCHED_PIPELINED)
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED


@pytest.mark.parametrize("space", ["P1", "CG1xDG0", "CG1xDG1"])
@pytest.mark.parametrize("lam", [1, 2, 10, 60, 61, 62, 63, 64, 65, 123, 124, 125, 130])
@pytest.mark.parametrize("order", ["rcm", "random"])
@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_gather_schedule_shapes(space, lam, order, wpb):
    # the vertex-column schedule: steps of 62 owned levels (P1), of 64 layers
    # (CG1 x DG*), so lambda around multiples of 62 and 64 exercises the ends
    say(f"gather {space} lam={lam} order={order} wpb={wpb}")
    c = Case(meshgen.tri_square(7, order=order), lam, space, terrain=0.3)
    x = meshgen.uniform_values(c.n, seed=51)
    cfg = exm.par_loop_config(exm.EXM_K_MASS, c.mesh, c.X, c.Vx,
                              [(c.dev(x), c.V, exm.EXM_READ), (c.V.zeros(), c.V, exm.EXM_INC)],
                              schedule=exm.EXM_SCHED_GATHER, waves_per_block=wpb)
    assert cfg["schedule"] == exm.EXM_SCHED_GATHER and cfg["race"] == exm.EXM_RACE_OWNER
    got = c.mass(x, schedule=exm.EXM_SCHED_GATHER, waves_per_block=wpb)
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"gather {space}")


@pytest.mark.parametrize("space", ["P1", "CG1xDG0", "CG1xDG1"])
@pytest.mark.parametrize("n", [4, 5, 7])
@pytest.mark.parametrize("schedule", [exm.EXM_SCHED_GATHER, exm.EXM_SCHED_PIPELINED, exm.EXM_SCHED_DIRECT])
def test_checkerboard_mesh(space, n, schedule):
    # every other quad removed: interior vertices carry two fans that touch only
    # at the vertex, and (n even) some vertices belong to no cell
    c = Case(meshgen.tri_checkerboard(n), 9, space, terrain=0.2)
    x = meshgen.uniform_values(c.n, seed=52)
    y0 = meshgen.uniform_values(c.n, seed=53)
    xd = c.dev(x)
    y = c.dev(y0)
    exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(xd, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)],
                 schedule=schedule)
    assert_close(c.host(y), c.ref.mass(x) + y0, c.ref.mass_abs(x) + np.abs(y0), what=f"checkerboard {space}")


def test_tiny_config_p1_rhs():
    # 16x16 triangulated square, 10 layers of height 0.1, P1 x P1, f ~ U[-1, 1]
    base = meshgen.tri_square(16)
    c = Case(base, 10, "P1")
    f = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    for race in (exm.EXM_RACE_ATOMIC, exm.EXM_RACE_COLOUR):
        got = c.mass(f, race=race)
        assert_close(got, c.ref.mass(f), c.ref.mass_abs(f), what="tiny P1 rhs")
    # partition of unity on the device result: sum_i b_i = integral of f
    one = c.mass(np.ones(c.n))
    assert abs(one.sum() - 1.0) < 1e-13


def test_single_cell_mesh():
    base = meshgen.tri_rectangle(1, 1, 1.0, jitter=0.0)
    for space in ("P1", "DG0", "DG1", "P2"):
        c = Case(base, 3, space)
        x = meshgen.uniform_values(c.n, seed=2)
        assert_close(c.mass(x), c.ref.mass(x), c.ref.mass_abs(x), what=f"single quad {space}")


def test_inc_accumulates():
    base = meshgen.tri_square(6)
    c = Case(base, 5, "P1")
    x = meshgen.uniform_values(c.n, seed=3)
    xd = c.dev(x)
    y = c.dev(np.full(c.n, 2.0))
    exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(xd, c.V, exm.EXM_READ), (y, c.V, exm.EXM_INC)])
    ref = c.ref.mass(x) + 2.0
    assert_close(c.host(y), ref, c.ref.mass_abs(x) + 2.0, what="INC into non-zero output")


def test_colour_counts():
    base = meshgen.tri_square(16)
    mesh = exm.Mesh(base, 4)
    n = mesh.colours()
    # a vertex of the triangulated square touches at most 6 cells
    assert 6 <= n <= 13


@pytest.mark.parametrize("case", ["same_buffer", "output_inside_input", "input_inside_output", "output_in_coords",
                                  "two_outputs_overlap"])
def test_par_loop_refuses_overlapping_arguments(case):
    # an output may share no byte with any other argument (refused on the
    # host, before any launch); disjoint views of one allocation are fine
    c = Case(meshgen.tri_square(4), 5, "P1")
    n = c.n
    big = torch.zeros(3 * n + 8, dtype=torch.float64, device="cuda")
    x = big[:n]
    R, I = exm.EXM_READ, exm.EXM_INC
    if case == "same_buffer":
        fields = [(x, c.V, R), (x, c.V, I)]
    elif case == "output_inside_input":
        fields = [(x, c.V, R), (big[n - 1:2 * n - 1], c.V, I)]
    elif case == "input_inside_output":
        fields = [(big[1:n + 1], c.V, R), (x, c.V, I)]
    elif case == "output_in_coords":
        fields = [(x, c.V, R), (c.X.view(-1)[2 * n:3 * n], c.V, I)]
    else:
        u = big[n:2 * n]
        fields = [(x, c.V, R), (u, c.V, R), (big[2 * n:3 * n], c.V, I), (big[2 * n + 4:3 * n + 4], c.V, I)]
    kernel = exm.EXM_K_CUBIC_VJP if case == "two_outputs_overlap" else exm.EXM_K_MASS
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(kernel, c.mesh, c.X, c.Vx, fields)
    assert e.value.status == exm._abi.EXM_EINVAL and "overlaps" in str(e.value), str(e.value)
    # back to back views of one allocation are accepted
    exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, [(x, c.V, R), (big[n:2 * n], c.V, I)])
    torch.cuda.synchronize()
