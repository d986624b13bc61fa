"""The coordinate field at the boundary: placement by the library from
per-(vertex, level) coordinates, refusal of columns that lean (the element
kernels need the x, y of a vertex to be the same at every level), and meshes
built from device-resident adjacency."""
import numpy as np
import pytest
import torch

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import Case, assert_close, say

pytestmark = pytest.mark.gpu


def _lean(vc, vertex, level, dx=1e-3):
    bad = vc.copy()
    bad[vertex, level, 0] += dx
    return bad


@pytest.mark.parametrize("layers", [None, "bathymetry"])
def test_coordinate_field_matches_the_numbering(layers):
    say(f"coordinate placement layers={layers}")
    base = meshgen.tri_square(9)
    lam = 7
    rng = None if layers is None else meshgen.layer_ranges(base, lam, kind=layers)
    mesh = exm.Mesh(base, lam, layers=rng)
    V = exm.Space(mesh, "P1")
    vc = meshgen.extruded_vertex_coords(base, lam, terrain=0.2)
    for src in (vc, torch.from_numpy(vc).cuda()):
        X = exm.coordinate_field(V, src).cpu().numpy()
        starts = V.column_starts(0).cpu().numpy()
        lo, hi = mesh.entity_layers(0)
        for v in range(base.n_vertices):
            for lev in range(lo[v], hi[v] + 1):
                np.testing.assert_array_equal(X[:, starts[v] + lev - lo[v]], vc[v, lev])


@pytest.mark.parametrize("on_device", [False, True])
def test_leaning_column_is_refused_at_placement(on_device):
    base = meshgen.tri_square(6)
    lam = 5
    mesh = exm.Mesh(base, lam)
    V = exm.Space(mesh, "P1")
    bad = _lean(meshgen.extruded_vertex_coords(base, lam), vertex=17, level=3)
    src = torch.from_numpy(bad).cuda() if on_device else bad
    with pytest.raises(exm.ExmError) as e:
        exm.coordinate_field(V, src)
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED and "17" in str(e.value)
    # a change of z alone (terrain) is allowed
    ok = meshgen.extruded_vertex_coords(base, lam)
    ok[17, 3, 2] += 1e-3
    exm.coordinate_field(V, torch.from_numpy(ok).cuda() if on_device else ok)


def test_leaning_field_is_refused_by_the_loop():
    c = Case(meshgen.tri_square(6), 5, "P1")
    f = c.dev(meshgen.uniform_values(c.n, seed=1))
    # a field built outside the library whose vertex 9 leans at level 2
    starts = c.Vx.column_starts(0).cpu().numpy()
    Xbad = c.X.clone()
    Xbad[0, int(starts[9]) + 2] += 1e-3
    b = c.V.zeros()
    with pytest.raises(exm.ExmError) as e:
        exm.par_loop(exm.EXM_K_MASS, c.mesh, Xbad, c.Vx, [(f, c.V, exm.EXM_READ), (b, c.V, exm.EXM_INC)])
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED and "9" in str(e.value)
    with pytest.raises(exm.ExmError):
        exm.verify_coordinates(c.Vx, Xbad)
    # the same field made vertical again passes the explicit check and the loop
    Xbad[0, int(starts[9]) + 2] -= 1e-3
    exm.verify_coordinates(c.Vx, Xbad)
    exm.par_loop(exm.EXM_K_MASS, c.mesh, Xbad, c.Vx, [(f, c.V, exm.EXM_READ), (b, c.V, exm.EXM_INC)])
    assert_close(c.host(b), c.ref.mass(c.host(f)), c.ref.mass_abs(c.host(f)), what="loop after re-check")


def test_unchecked_field_is_refused_under_capture():
    c = Case(meshgen.tri_square(4), 3, "P1")
    f = c.dev(meshgen.uniform_values(c.n, seed=1))
    b = c.V.zeros()
    X2 = c.X.clone()    # a new address the library has not checked
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(exm.ExmError) as e:
        with torch.cuda.graph(g, stream=s):
            exm.par_loop(exm.EXM_K_MASS, c.mesh, X2, c.Vx, [(f, c.V, exm.EXM_READ), (b, c.V, exm.EXM_INC)])
    assert e.value.status == exm._abi.EXM_EINVAL and "captur" in str(e.value)
    torch.cuda.synchronize()


@pytest.mark.parametrize("layers", [None, "random"])
def test_mesh_from_device_adjacency(layers):
    base = meshgen.tri_square(8)
    lam = 6
    rng = None if layers is None else meshgen.layer_ranges(base, lam, kind=layers)
    host = exm.Mesh(base, lam, layers=rng)
    dev = exm.Mesh.from_device(base, lam, torch.from_numpy(base.cell_vertex.astype(np.int32)).cuda(),
                               torch.from_numpy(base.cell_edge.astype(np.int32)).cuda(),
                               None if rng is None else torch.from_numpy(rng.astype(np.int32)).cuda())
    for name in ("P1", "P2", "DG1"):
        a, b = exm.Space(host, name), exm.Space(dev, name)
        assert a.n_dofs == b.n_dofs
        assert torch.equal(a.bottom_map(), b.bottom_map())
        for d in range(3):
            assert torch.equal(a.column_starts(d), b.column_starts(d))
    for d in range(3):
        for x, y in zip(host.entity_layers(d), dev.entity_layers(d)):
            np.testing.assert_array_equal(x, y)


def test_mesh_from_device_refuses_host_memory():
    base = meshgen.tri_square(3)
    cv = np.ascontiguousarray(base.cell_vertex, dtype=np.int32)
    h = exm.ctypes.c_void_p()
    with pytest.raises(exm.ExmError) as e:
        exm._abi.exm_mesh_create_device(base.n_vertices, base.n_edges, base.n_cells,
                                        cv.ctypes.data_as(exm.ctypes.c_void_p), None, 2, None, exm.ctypes.byref(h))
    assert e.value.status == exm._abi.EXM_EINVAL
