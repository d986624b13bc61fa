"""Degenerate and extreme shapes: numberings past the int32 range are refused
before anything is allocated; very tall columns on a tiny base (many chunk
steps, a ragged last chunk) match the oracle on every schedule that takes
them; one layer and one cell."""
import numpy as np
import pytest

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import Case, assert_close, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("space,lam", [("DG1", 200_000_000), ("P1", 2**31 - 2), ("P1", 240_000_000),
                                       ("P2", 120_000_000)])
def test_numbering_past_int32_is_refused(space, lam):
    # a 2 x 2 base (9 vertices, 16 edges, 8 cells): every count is past 2^31
    base = meshgen.tri_square(2)
    mesh = exm.Mesh(base, lam)
    with pytest.raises(exm.ExmError) as e:
        exm.Space(mesh, space)
    assert e.value.status == exm._abi.EXM_EOVERFLOW


def test_mixed_counts_past_int32_are_refused():
    base = meshgen.tri_square(3)
    mesh = exm.Mesh(base, 40_000_000)
    dofs = [np.full((base.n_vertices, 2), 0, np.int32), None, np.full((base.n_cells, 2), 64, np.int32)]
    with pytest.raises(exm.ExmError) as e:
        exm.Space.mixed(mesh, dofs)
    assert e.value.status == exm._abi.EXM_EOVERFLOW


TALL = [(exm.EXM_SCHED_DIRECT, {}), (exm.EXM_SCHED_PIPELINED, dict(tile_cells=32, chunk_layers=16)),
        (exm.EXM_SCHED_PIPELINED, dict(tile_cells=8, chunk_layers=8)), (exm.EXM_SCHED_STAGED, dict(chunk_layers=64)),
        (exm.EXM_SCHED_GATHER, {}), (exm.EXM_SCHED_AUTO, {})]


@pytest.mark.parametrize("space", ["P1", "DG0", "DG1", "P2", "CG1xDG0", "DG0xCG1"])
@pytest.mark.parametrize("schedule,extra", TALL)
def test_tall_columns_on_a_tiny_base(space, schedule, extra):
    say(f"tall columns {space} schedule={schedule} {extra}")
    base = meshgen.tri_square(2)
    lam = 2999   # many chunk steps and 64-lane steps, a ragged last one
    c = Case(base, lam, space, terrain=0.2)
    x = meshgen.uniform_values(c.n, seed=21)
    try:
        got = c.mass(x, schedule=schedule, **extra)
    except exm.ExmError as e:
        # a schedule that does not take this space says so before any launch
        assert e.status in (exm._abi.EXM_EUNSUPPORTED, exm._abi.EXM_ERANGE), str(e)
        return
    assert_close(got, c.ref.mass(x), c.ref.mass_abs(x), what=f"tall {space}")


@pytest.mark.parametrize("space", ["P1", "DG0", "DG1", "P2", "CG1xDG1", "DG1xCG1"])
def test_one_layer_one_cell(space):
    # a single right triangle extruded once: every entity on the boundary
    base = meshgen._assemble(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 2]]), "natural", 0, {})
    c = Case(base, 1, space)
    x = meshgen.uniform_values(c.n, seed=22)
    for schedule in (exm.EXM_SCHED_DIRECT, exm.EXM_SCHED_AUTO):
        assert_close(c.mass(x, schedule=schedule), c.ref.mass(x), c.ref.mass_abs(x), what=f"one prism {space}")
    # the volume of the one prism, from the residual of 1
    assert abs(c.mass(np.ones(c.n)).sum() - 0.5) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 1001, 4096])
@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("grid", [0, 3])
def test_stream_triad(n, offset, grid):
    # 16-byte pairs (aligned arrays, odd n ends in a single element) and one
    # element per lane (arrays 8 bytes off), one element or pair per thread
    # or a grid-stride loop over few workgroups
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    # three allocations (each 16-byte aligned), viewed from element `offset`
    a, b, c = (torch.rand(n + 1, dtype=torch.float64, device="cuda", generator=g)[offset:offset + n]
               for _ in range(3))
    assert all((t.data_ptr() % 16 == 0) == (offset == 0) for t in (a, b, c))
    want = b.cpu().numpy() + 3.0 * c.cpu().numpy()
    exm.stream_triad(a, b, c, 3.0, block=256, grid=grid)
    torch.cuda.synchronize()
    # within one rounding of the fused or separate multiply-add
    np.testing.assert_allclose(a.cpu().numpy(), want, rtol=4.5e-16, atol=0)
