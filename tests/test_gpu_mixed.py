"""Parity of spaces with a DoF count per entity (the per-type constant of the
exposition relaxed, Section 5): Algorithm 1's numbering and the per-entity
lists bit-exact, and the mixed-degree DG mass action, against the oracle."""
import numpy as np
import pytest

import oracle
import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import assert_close, say

pytestmark = pytest.mark.gpu


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,lam", [(3, 1), (5, 4), (4, 70)])
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("order", ["rcm", "random"])
def test_entity_dofs_numbering_bit_exact(n, lam, seed, order):
    say(f"entity dofs n={n} lam={lam} seed={seed} {order}")
    base = meshgen.tri_square(n, order=order)
    dofs = meshgen.entity_dofs(base, hi=3, seed=seed)
    mesh = exm.Mesh(base, lam)
    V = exm.Space.mixed(mesh, dofs)
    ref = oracle.number_mixed(base.counts, lam, dofs, base.cell_vertex, base.cell_edge)
    assert V.n_dofs == ref.n_dofs
    for d in range(3):
        np.testing.assert_array_equal(_host(V.column_starts(d)), ref.column_starts(d).astype(np.int32))
    off, lst, eo = V.lists()
    np.testing.assert_array_equal(_host(off), ref.list_off.astype(np.int32))
    np.testing.assert_array_equal(_host(lst), ref.lmap.astype(np.int32))
    np.testing.assert_array_equal(_host(eo), ref.offsets)


@pytest.mark.parametrize("space", ["P1", "P2", "DG1", "CG1xDG1", "DG1xCG1"])
def test_type_table_as_entity_dofs_matches_the_uniform_space(space):
    base = meshgen.tri_square(4)
    mesh = exm.Mesh(base, 6)
    U = exm.Space(mesh, space)
    delta = np.asarray(exm.DELTA[exm.ELEMENTS[space]]).reshape(3, 2)
    M = exm.Space.mixed(mesh, [np.tile(delta[d], (base.counts[d], 1)) for d in range(3)])
    assert M.n_dofs == U.n_dofs and M.arity == U.arity
    for a, b in zip(U.lists(), M.lists()):
        np.testing.assert_array_equal(_host(a), _host(b))
    np.testing.assert_array_equal(_host(U.bottom_map()).ravel(), _host(M.lists()[1]))


@pytest.mark.parametrize("n,lam", [(4, 3), (5, 1), (3, 70), (6, 64)])
@pytest.mark.parametrize("frac", [0.0, 0.3, 1.0])
@pytest.mark.parametrize("access", ["write", "inc"])
@pytest.mark.parametrize("cpw", [0, 1, 3])
def test_mixed_degree_dg_mass(n, lam, frac, access, cpw):
    say(f"dgmix n={n} lam={lam} frac={frac} {access} cpw={cpw}")
    import torch
    base = meshgen.tri_square(n)
    vc = meshgen.extruded_vertex_coords(base, lam, terrain=0.3)
    nd = meshgen.cell_degrees(base, frac_dg1=frac)
    mesh = exm.Mesh(base, lam)
    Vx = exm.Space(mesh, "P1")
    X = exm.coordinate_field(Vx, vc)
    dofs = [np.zeros((base.n_vertices, 2), np.int32), None, np.stack([np.zeros_like(nd), nd], 1)]
    V = exm.Space.mixed(mesh, dofs, element=exm.EXM_ELEMENT_DGMIX)
    x = meshgen.uniform_values(V.n_dofs, seed=61)
    ref, num = oracle.mixed_dg_mass(base, lam, vc, nd, x)
    scale, _ = oracle.mixed_dg_mass(base, lam, vc, nd, x, absf=True)
    assert num.n_dofs == V.n_dofs
    y0 = meshgen.uniform_values(V.n_dofs, seed=62) if access == "inc" else np.zeros(V.n_dofs)
    y = torch.from_numpy(y0).to("cuda")
    acc = exm.EXM_INC if access == "inc" else exm.EXM_WRITE
    exm.par_loop(exm.EXM_K_MASS, mesh, X, Vx, [(torch.from_numpy(x).to("cuda"), V, exm.EXM_READ), (y, V, acc)],
                 cols_per_wave=cpw)
    assert_close(_host(y), ref + y0, scale + np.abs(y0), what="mixed-degree DG mass")


def test_mixed_space_refusals():
    base = meshgen.tri_square(4)
    mesh = exm.Mesh(base, 3)
    nd = meshgen.cell_degrees(base)
    bad = np.stack([np.zeros_like(nd), np.where(nd == 6, 2, 1)], 1)   # 2 DoFs per layer: neither DG0 nor DG1
    with pytest.raises(exm.ExmError) as e:
        exm.Space.mixed(mesh, [np.zeros((base.n_vertices, 2)), None, bad], element=exm.EXM_ELEMENT_DGMIX)
    assert e.value.status == exm._abi.EXM_EINVAL
    with pytest.raises(exm.ExmError) as e:
        exm.Space.mixed(mesh, [np.full((base.n_vertices, 2), 65), None, np.zeros((base.n_cells, 2))])
    assert e.value.status == exm._abi.EXM_ERANGE
    V = exm.Space.mixed(mesh, meshgen.entity_dofs(base))
    with pytest.raises(exm.ExmError) as e:
        V.offsets()
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED
    with pytest.raises(exm.ExmError) as e:
        V.bottom_map()
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED
    D = exm.Space.mixed(mesh, [np.zeros((base.n_vertices, 2)), None, np.stack([np.zeros_like(nd), nd], 1)],
                        element=exm.EXM_ELEMENT_DGMIX)
    with pytest.raises(exm.ExmError) as e:
        exm.Matrix(D)
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED
    vmesh = exm.Mesh(base, 5, layers=meshgen.layer_ranges(base, 5, "random"))
    with pytest.raises(exm.ExmError) as e:
        exm.Space.mixed(vmesh, meshgen.entity_dofs(base))
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED
