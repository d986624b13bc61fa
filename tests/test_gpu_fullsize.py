"""Parity at the benchmark sizes, in the launch configuration bench.py uses
(autotuned, then the library's choice): sampled columns against the oracle,
which assembles just the base cells around each sampled column."""
import numpy as np
import pytest
import torch

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from tests.gpu_common import Case, assert_close, say

pytestmark = pytest.mark.gpu


def _cells_around_vertices(base, verts):
    return np.nonzero(np.isin(base.cell_vertex, verts).any(axis=1))[0]


def _cells_around_edges(base, edges):
    return np.nonzero(np.isin(base.cell_edge, edges).any(axis=1))[0]


def _check_columns(got, ref, scale, starts, ids, length, what):
    idx = (starts[ids][:, None] + np.arange(length)[None, :]).ravel()
    assert_close(got[idx], ref[idx], scale[idx], what=what)


def _tuned_mass(c, x_np):
    xd = c.dev(x_np)
    y = c.V.zeros()
    fields = [(xd, c.V, exm.EXM_READ), (y, c.V, c.out_access())]
    cfg = exm.autotune(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, fields)
    exm.par_loop(exm.EXM_K_MASS, c.mesh, c.X, c.Vx, fields)
    return c.host(y), cfg


@pytest.mark.parametrize("space", ["P1", "DG0"])
def test_config2_sampled(space):
    say(f"full size 512x512x100 {space}")
    base = meshgen.tri_square(512)
    lam = 100
    c = Case(base, lam, space)
    x = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    got, cfg = _tuned_mass(c, x)
    say(f"  launch {cfg}")
    rng = np.random.default_rng(77)
    if space == "P1":
        verts = rng.choice(base.n_vertices, 64, replace=False)
        cells = _cells_around_vertices(base, verts)
        ref = c.ref.mass(x, cells=cells)
        scale = c.ref.mass_abs(x, cells=cells)
        _check_columns(got, ref, scale, c.ref.num_v.column_starts(0), verts, lam + 1, "P1 columns")
    else:
        cells = rng.choice(base.n_cells, 256, replace=False)
        ref = c.ref.mass(x, cells=cells)
        scale = c.ref.mass_abs(x, cells=cells)
        _check_columns(got, ref, scale, c.ref.num_v.column_starts(2), cells, lam, "DG0 columns")
    # invariant over the whole output: sum of the residual of f = 1 is the volume
    one = np.ones(c.n)
    got_one, _ = _tuned_mass(c, one)
    assert abs(got_one.sum() - 1.0) < 1e-11


@pytest.mark.parametrize("space", ["DG1", "P2"])
def test_config3_sampled(space):
    say(f"full size 256x256x64 {space}")
    base = meshgen.tri_square(256)
    lam = 64
    c = Case(base, lam, space)
    x = meshgen.uniform_values(c.n, seed=meshgen.SEED_FIELD)
    got, cfg = _tuned_mass(c, x)
    say(f"  launch {cfg}")
    rng = np.random.default_rng(78)
    if space == "DG1":
        cells = rng.choice(base.n_cells, 256, replace=False)
        ref = c.ref.mass(x, cells=cells)
        scale = c.ref.mass_abs(x, cells=cells)
        _check_columns(got, ref, scale, c.ref.num_v.column_starts(2), cells, 6 * lam, "DG1 columns")
    else:
        verts = rng.choice(base.n_vertices, 48, replace=False)
        edges = rng.choice(base.n_edges, 48, replace=False)
        cells = np.union1d(_cells_around_vertices(base, verts), _cells_around_edges(base, edges))
        ref = c.ref.mass(x, cells=cells)
        scale = c.ref.mass_abs(x, cells=cells)
        _check_columns(got, ref, scale, c.ref.num_v.column_starts(0), verts, 2 * lam + 1, "P2 vertex columns")
        _check_columns(got, ref, scale, c.ref.num_v.column_starts(1), edges, 2 * lam + 1, "P2 edge columns")


def test_config4_sampled():
    say("full size 256x256x50 cubic")
    base = meshgen.tri_square(256)
    lam = 50
    c = Case(base, lam, "P1")
    u = meshgen.uniform_values(c.n, seed=31)
    f = meshgen.uniform_values(c.n, seed=32)
    w = meshgen.uniform_values(c.n, seed=meshgen.SEED_COTAN)
    ud, fd, wd = c.dev(u), c.dev(f), c.dev(w)
    F, gu, gf = c.V.zeros(), c.V.zeros(), c.V.zeros()
    fields = [(ud, c.V, exm.EXM_READ), (fd, c.V, exm.EXM_READ), (wd, c.V, exm.EXM_READ), (F, c.V, exm.EXM_INC),
              (gu, c.V, exm.EXM_INC), (gf, c.V, exm.EXM_INC)]
    exm.autotune(exm.EXM_K_CUBIC_FUSED, c.mesh, c.X, c.Vx, fields)
    exm.par_loop(exm.EXM_K_CUBIC_FUSED, c.mesh, c.X, c.Vx, fields)
    rng = np.random.default_rng(79)
    verts = rng.choice(base.n_vertices, 64, replace=False)
    cells = _cells_around_vertices(base, verts)
    S = c.ref.num_v.column_starts(0)
    Fr, gur, gfr = c.ref.cubic_fused(u, f, w, cells=cells)
    Fs = c.ref.cubic_abs(u, f, cells=cells)
    gus, gfs = c.ref.vjp_abs(u, w, cells=cells)
    _check_columns(c.host(F), Fr, Fs, S, verts, lam + 1, "fused F")
    _check_columns(c.host(gu), gur, gus, S, verts, lam + 1, "fused g_u")
    _check_columns(c.host(gf), gfr, gfs, S, verts, lam + 1, "fused g_f")
