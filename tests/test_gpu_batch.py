"""Batched persistent launch (HIP graph): every output equals its single
par_loop counterpart and the oracle, on every graph replay."""
import numpy as np
import pytest
import torch

import oracle
import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import assert_close, say

pytestmark = pytest.mark.gpu


def _setup(n_meshes, scale, n_fields, adjoint, seed=meshgen.SEED_BATCH):
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    items, refs = [], []
    for it in meshgen.batch_meshes(n_meshes=n_meshes, scale=scale, seed=seed):
        mesh = exm.Mesh(it.mesh, it.n_layers)
        Vx = exm.Space(mesh, "P1")
        V = exm.Space(mesh, it.space) if it.space != "P1" else Vx
        vc = meshgen.extruded_vertex_coords(it.mesh, it.n_layers)
        X = exm.coordinate_field(Vx, vc)
        rnd = lambda: torch.rand(V.n_dofs, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
        d = dict(space=V, coord_space=Vx, coords=X, mesh=mesh, base=it,
                 f=[rnd() for _ in range(n_fields)], b=[V.zeros() for _ in range(n_fields)])
        if adjoint:
            d["w"] = [rnd() for _ in range(n_fields)]
            d["g"] = [V.zeros() for _ in range(n_fields)]
        items.append(d)
        refs.append(vc)
    return items, refs


def _single(d, x):
    y = d["space"].zeros()
    acc = exm.EXM_INC if d["space"].element == exm.EXM_ELEMENT_P1P1 else exm.EXM_WRITE
    exm.par_loop(exm.EXM_K_MASS, d["mesh"], d["coords"], d["coord_space"], [(x, d["space"], exm.EXM_READ),
                                                                             (y, d["space"], acc)])
    return y


# items on tiles (default: timed tile sizes; a fixed unit size takes the
# first tiling that fits; chunk_layers fixes the chunk: 8 and 16 tile both
# kinds, 32 and 34 only DG0) or on work units (GATHER)
@pytest.mark.parametrize("cpw,unit,sched,chunk", [(0, 0, 0, 0), (1, 8, 0, 0), (3, 64, 0, 8), (2, 1000, 0, 16),
                                                  (0, 0, 0, 32), (0, 0, 0, 34), (0, 0, "gather", 0),
                                                  (3, 64, "gather", 0)])
def test_batch_matches_single_launches(cpw, unit, sched, chunk):
    say(f"batch cpw={cpw} unit={unit} sched={sched} chunk={chunk}")
    items, _ = _setup(6, 0.01, 3, True)
    schedule = exm.EXM_SCHED_GATHER if sched == "gather" else 0
    B = exm.Batch(items, cols_per_wave=cpw, unit_cells=unit, schedule=schedule, chunk_layers=chunk)
    n_units, n_blocks = B.info()
    t1, t0 = B.tiles("P1"), B.tiles("DG0")
    if sched == "gather":
        assert t1 == (0, 0) and t0 == (0, 0)
        assert n_units >= len(items) and n_blocks > 0
    else:
        if chunk in (32, 34):   # P1 tiles take 8 or 16: the P1 items run on vertex units
            assert t1 == (0, 0) and n_units > 0
        else:
            assert t1[0] > 0 and t1[1] == (chunk or t1[1]) and t1[1] in (8, 16)
        assert t0[0] > 0 and t0[1] == (chunk or t0[1]) and t0[1] in (8, 16, 32, 34)
    ref = [([_single(d, f) for f in d["f"]], [_single(d, w) for w in d["w"]]) for d in items]
    torch.cuda.synchronize()
    for replay in range(3):
        # eager work between replays: scribble on the outputs
        for d in items:
            for t in d["b"] + d["g"]:
                t.fill_(123.0)
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for d, (rb, rg) in zip(items, ref):
            for got, want in zip(d["b"] + d["g"], rb + rg):
                g_, w_ = got.cpu().numpy(), want.cpu().numpy()
                assert_close(g_, w_, np.abs(w_) + np.abs(w_).max() * 1e-3, rtol=1e-13, what=f"replay {replay}")


@pytest.mark.parametrize("race", [exm.EXM_RACE_OWNER, exm.EXM_RACE_ATOMIC])
@pytest.mark.parametrize("chunk", [8, 16])
def test_batch_p1_tile_kinds(race, chunk):
    # P1 items on owner tiles, or on shared tiles whose boundary columns are
    # zeroed in the graph and added atomically: every replay equals the single
    # launches and the oracle, whatever the outputs held before
    say(f"batch P1 tiles race={race} chunk={chunk}")
    items, vcs = _setup(6, 0.01, 2, True, seed=13)
    B = exm.Batch(items, chunk_layers=chunk, race=race)
    t1 = B.tiles("P1")
    assert t1[0] > 0 and t1[1] == chunk
    ref = [([_single(d, f) for f in d["f"]], [_single(d, w) for w in d["w"]]) for d in items]
    torch.cuda.synchronize()
    for replay in range(3):
        for d in items:
            for t in d["b"] + d["g"]:
                t.fill_(-7.5 if replay % 2 else 123.0)
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for d, (rb, rg) in zip(items, ref):
            for got, want in zip(d["b"] + d["g"], rb + rg):
                g_, w_ = got.cpu().numpy(), want.cpu().numpy()
                assert_close(g_, w_, np.abs(w_) + np.abs(w_).max() * 1e-3, rtol=1e-13, what=f"replay {replay}")
    for d, vc in zip(items, vcs):
        if d["space"].element != exm.EXM_ELEMENT_P1P1:
            continue
        pr = oracle.Problem(d["base"].mesh, d["base"].n_layers, "P1", vc)
        for x, y in zip(d["f"] + d["w"], d["b"] + d["g"]):
            xn = x.cpu().numpy()
            assert_close(y.cpu().numpy(), pr.mass(xn), pr.mass_abs(xn), what=f"batch P1 race={race} vs oracle")


@pytest.mark.parametrize("sched", [0, "gather"])
def test_batch_matches_oracle(sched):
    items, vcs = _setup(4, 0.004, 2, True, seed=9)
    B = exm.Batch(items, schedule=exm.EXM_SCHED_GATHER if sched == "gather" else 0)
    with pytest.raises(exm.ExmError):
        exm._abi.exm_batch_tiles(B.handle, exm.EXM_ELEMENT_P2P2, None, None)
    B.launch()
    torch.cuda.synchronize()
    for d, vc in zip(items, vcs):
        name = "P1" if d["space"].element == exm.EXM_ELEMENT_P1P1 else "DG0"
        pr = oracle.Problem(d["base"].mesh, d["base"].n_layers, name, vc)
        for src, dst in ((d["f"], d["b"]), (d["w"], d["g"])):
            for x, y in zip(src, dst):
                xn = x.cpu().numpy()
                assert_close(y.cpu().numpy(), pr.mass(xn), pr.mass_abs(xn), what=f"batch vs oracle {name}")


def test_batch_rejects_bad_items():
    items, _ = _setup(2, 0.004, 1, False)
    items[0]["b"] = [items[0]["f"][0]]   # output aliases input
    with pytest.raises(exm.ExmError):
        exm.Batch(items)


@pytest.mark.parametrize("case", ["out_is_other_input", "two_equal_outputs", "out_is_other_cotangent",
                                  "out_is_coords", "out_overlaps_output"])
def test_batch_rejects_aliases_across_items(case):
    items, _ = _setup(2, 0.004, 2, True)
    a, b = items
    if case == "out_is_other_input":
        na, nb = a["space"].n_dofs, b["space"].n_dofs
        big = torch.rand(max(na, nb), dtype=torch.float64, device="cuda")
        b["f"][0] = big[:nb]
        a["b"][1] = big[:na]
    elif case == "two_equal_outputs":
        a["g"][0] = a["b"][1]
    elif case == "out_is_other_cotangent":
        a["g"][1] = a["w"][0]
    elif case == "out_is_coords":
        a["b"][0] = a["coords"].view(-1)[:a["space"].n_dofs]
    else:
        # an output that starts inside another item's output
        big = torch.zeros(a["space"].n_dofs + b["space"].n_dofs, dtype=torch.float64, device="cuda")
        a["b"][0] = big[:a["space"].n_dofs]
        b["b"][0] = big[a["space"].n_dofs - 1:a["space"].n_dofs - 1 + b["space"].n_dofs]
    with pytest.raises(exm.ExmError, match="overlap"):
        exm.Batch(items)
    # the same items with their own outputs are accepted
    items2, _ = _setup(2, 0.004, 2, True)
    exm.Batch(items2)


@pytest.mark.parametrize("sched", [0, "gather"])
def test_batch_short_columns_odd_field_count(sched):
    # P1 columns shorter than one chunk, or than one 62-level step of the
    # vertex units, and 5 fields (a partial group of the vertex units' four
    # fields per walk of the fan); no adjoint
    say(f"batch short columns, 5 fields, sched={sched}")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(21)
    items = []
    for space, n, lam in (("P1", 9, 7), ("DG0", 8, 5), ("P1", 6, 61), ("P1", 5, 1)):
        base = meshgen.tri_square(n)
        mesh = exm.Mesh(base, lam)
        Vx = exm.Space(mesh, "P1")
        V = exm.Space(mesh, space) if space != "P1" else Vx
        X = exm.coordinate_field(Vx, meshgen.extruded_vertex_coords(base, lam))
        rnd = lambda: torch.rand(V.n_dofs, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
        items.append(dict(space=V, coord_space=Vx, coords=X, mesh=mesh,
                          f=[rnd() for _ in range(5)], b=[V.zeros() for _ in range(5)]))
    B = exm.Batch(items, schedule=exm.EXM_SCHED_GATHER if sched == "gather" else 0)
    assert (B.tiles("P1") == (0, 0)) == (sched == "gather")
    assert (B.tiles("DG0") == (0, 0)) == (sched == "gather")
    ref = [[_single(d, f) for f in d["f"]] for d in items]
    for d in items:
        for t in d["b"]:
            t.fill_(-7.0)
    torch.cuda.synchronize()
    B.launch()
    torch.cuda.synchronize()
    for d, rb in zip(items, ref):
        for got, want in zip(d["b"], rb):
            g_, w_ = got.cpu().numpy(), want.cpu().numpy()
            assert_close(g_, w_, np.abs(w_) + np.abs(w_).max() * 1e-3, rtol=1e-13, what="short columns")


def test_batch_misaligned_p1_field_runs_on_units():
    # the tile walk copies P1 fields 16 bytes at a time: a field that starts
    # 8 bytes into its allocation puts the P1 items on vertex units, the DG0
    # items stay on tiles, and every output still matches
    say("batch, misaligned P1 field")
    items, _ = _setup(4, 0.004, 2, True, seed=13)
    p1 = next(d for d in items if d["space"].element == exm.EXM_ELEMENT_P1P1)
    n = p1["space"].n_dofs
    store = torch.empty(n + 1, dtype=torch.float64, device="cuda")
    store[1:] = p1["f"][0]
    p1["f"][0] = store[1:]
    assert p1["f"][0].data_ptr() % 16 == 8
    B = exm.Batch(items)
    assert B.tiles("P1") == (0, 0) and B.tiles("DG0") != (0, 0)
    # references from aligned copies (the single launch may take a tiled schedule)
    ref = [([_single(d, f.clone()) for f in d["f"]], [_single(d, w) for w in d["w"]]) for d in items]
    B.launch()
    torch.cuda.synchronize()
    for d, (rb, rg) in zip(items, ref):
        for got, want in zip(d["b"] + d["g"], rb + rg):
            g_, w_ = got.cpu().numpy(), want.cpu().numpy()
            assert_close(g_, w_, np.abs(w_) + np.abs(w_).max() * 1e-3, rtol=1e-13, what="misaligned P1 field")


@pytest.mark.parametrize("kind", ["P1", "DG0"])
def test_batch_single_kind(kind):
    # a batch of one kind of item: the other branch of the graph is empty
    say(f"batch of {kind} items only")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(31)
    items = []
    for n, lam in ((7, 9), (5, 33)):
        base = meshgen.tri_square(n)
        mesh = exm.Mesh(base, lam)
        Vx = exm.Space(mesh, "P1")
        V = exm.Space(mesh, kind) if kind != "P1" else Vx
        X = exm.coordinate_field(Vx, meshgen.extruded_vertex_coords(base, lam))
        rnd = lambda: torch.rand(V.n_dofs, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
        items.append(dict(space=V, coord_space=Vx, coords=X, mesh=mesh, f=[rnd() for _ in range(3)],
                          b=[V.zeros() for _ in range(3)], w=[rnd() for _ in range(3)], g=[V.zeros() for _ in range(3)]))
    B = exm.Batch(items)
    assert B.tiles(kind) != (0, 0) and B.tiles("DG0" if kind == "P1" else "P1") == (0, 0)
    ref = [([_single(d, f) for f in d["f"]], [_single(d, w) for w in d["w"]]) for d in items]
    for replay in range(2):
        for d in items:
            for t in d["b"] + d["g"]:
                t.fill_(5.0)
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for d, (rb, rg) in zip(items, ref):
            for got, want in zip(d["b"] + d["g"], rb + rg):
                g_, w_ = got.cpu().numpy(), want.cpu().numpy()
                assert_close(g_, w_, np.abs(w_) + np.abs(w_).max() * 1e-3, rtol=1e-13, what=f"{kind} only, replay {replay}")


def test_batch_refuses_columns_of_different_heights():
    # batch items take meshes with one layer count: a mesh with a layer range
    # per column is refused at creation, before any launch
    base = meshgen.tri_square(5)
    layers = meshgen.layer_ranges(base, 12, "bathymetry")
    mesh = exm.Mesh(base, 12, layers=layers)
    Vx = exm.Space(mesh, "P1")
    X = exm.coordinate_field(Vx, meshgen.extruded_vertex_coords(base, 12))
    f = [torch.ones(Vx.n_dofs, dtype=torch.float64, device="cuda")]
    b = [Vx.zeros()]
    with pytest.raises(exm.ExmError) as e:
        exm.Batch([dict(space=Vx, coord_space=Vx, coords=X, mesh=mesh, f=f, b=b)])
    assert e.value.status == exm._abi.EXM_EUNSUPPORTED and "layer count" in str(e.value)


@pytest.mark.parametrize("how", [dict(race=exm.EXM_RACE_ATOMIC), dict(race=exm.EXM_RACE_OWNER),
                                 dict(schedule=exm.EXM_SCHED_GATHER)])
def test_batch_vertices_in_no_cell(how):
    # checkerboard bases of even n hold vertices that belong to no cell: on
    # shared tiles, owner tiles and vertex units alike their output columns
    # come out zero whatever the outputs held, and every other entry matches
    # the oracle
    say(f"batch, vertices in no cell, {how}")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(41)
    items, probs, lone = [], [], []
    for n, lam in ((4, 9), (12, 20)):
        base = meshgen.tri_checkerboard(n)
        mesh = exm.Mesh(base, lam)
        V = exm.Space(mesh, "P1")
        vc = meshgen.extruded_vertex_coords(base, lam, terrain=0.2)
        X = exm.coordinate_field(V, vc)
        rnd = lambda: torch.rand(V.n_dofs, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
        items.append(dict(space=V, coord_space=V, coords=X, mesh=mesh, f=[rnd() for _ in range(2)],
                          b=[V.zeros() for _ in range(2)], w=[rnd() for _ in range(2)], g=[V.zeros() for _ in range(2)]))
        probs.append(oracle.Problem(base, lam, "P1", vc))
        no_cell = np.nonzero(np.bincount(base.cell_vertex.ravel(), minlength=base.n_vertices) == 0)[0]
        assert no_cell.size > 0
        # P1 numbering: vertex v's column holds levels 0 .. lam at v * (lam + 1)
        lone.append((no_cell[:, None] * (lam + 1) + np.arange(lam + 1)).ravel())
    B = exm.Batch(items, **how)
    if "race" in how:
        assert B.tiles("P1")[0] > 0
    for replay in range(2):
        for d in items:
            for t in d["b"] + d["g"]:
                t.fill_(5.0 if replay else -3.0)
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for d, pr, idx in zip(items, probs, lone):
            for x, y in zip(d["f"] + d["w"], d["b"] + d["g"]):
                yn, xn = y.cpu().numpy(), x.cpu().numpy()
                assert np.all(yn[idx] == 0.0), f"replay {replay}: a column of a vertex in no cell holds {yn[idx]}"
                assert_close(yn, pr.mass(xn), pr.mass_abs(xn), what=f"batch {how} replay {replay}")
