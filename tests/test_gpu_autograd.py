"""The adjoint path: torch.autograd.Function wrappers over the hand-written
VJP kernels, checked against central finite differences (h = 1e-6) and the
oracle gradient, and the fused forward+adjoint kernel."""
import numpy as np
import pytest
import torch

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen
from paper_1604_05937_amd.autograd import (Extruded, cubic_residual, cubic_residual_with_vjp, mass_action)
from tests.gpu_common import Case, assert_close, say

pytestmark = pytest.mark.gpu


def _prob(c, **opts):
    return Extruded(c.mesh, c.Vx, c.X, c.V, **opts)


@pytest.mark.parametrize("opts", [{}, dict(schedule=exm.EXM_SCHED_STAGED, tile_cells=32, chunk_layers=8),
                                  dict(schedule=exm.EXM_SCHED_DIRECT, race=exm.EXM_RACE_COLOUR)])
def test_cubic_vjp_matches_oracle_and_fd(opts):
    say(f"autograd cubic {opts}")
    base = meshgen.tri_square(12)
    c = Case(base, 9, "P1", terrain=0.2)
    prob = _prob(c, **opts)
    u_np = meshgen.uniform_values(c.n, seed=41)
    f_np = meshgen.uniform_values(c.n, seed=42)
    w_np = meshgen.uniform_values(c.n, seed=meshgen.SEED_COTAN)
    u = c.dev(u_np).requires_grad_(True)
    f = c.dev(f_np).requires_grad_(True)
    w = c.dev(w_np)
    F = cubic_residual(u, f, prob)
    F.backward(w)
    gu, gf = c.host(u.grad), c.host(f.grad)
    gu_ref, gf_ref = c.ref.cubic_vjp(u_np, w_np)
    su, sf = c.ref.vjp_abs(u_np, w_np)
    assert_close(gu, gu_ref, su, what="autograd g_u vs oracle")
    assert_close(gf, gf_ref, sf, what="autograd g_f vs oracle")
    # central finite differences along seeded directions (h = 1e-6)
    h = 1e-6
    with torch.no_grad():
        for k in range(4):
            du = c.dev(meshgen.uniform_values(c.n, seed=100 + k))
            df = c.dev(meshgen.uniform_values(c.n, seed=200 + k))
            fd_u = (torch.dot(w, cubic_residual(u + h * du, f, prob)) - torch.dot(w, cubic_residual(u - h * du, f, prob))) / (2 * h)
            fd_f = (torch.dot(w, cubic_residual(u, f + h * df, prob)) - torch.dot(w, cubic_residual(u, f - h * df, prob))) / (2 * h)
            an_u = torch.dot(u.grad, du)
            an_f = torch.dot(f.grad, df)
            assert abs(float(fd_u - an_u)) <= 1e-6 * abs(float(an_u)), (float(fd_u), float(an_u))
            assert abs(float(fd_f - an_f)) <= 1e-6 * abs(float(an_f)), (float(fd_f), float(an_f))
    # the fused sweep gives the same three vectors
    F2, gu2, gf2 = cubic_residual_with_vjp(u, f, w, prob)
    assert_close(c.host(F2), c.ref.cubic(u_np, f_np), c.ref.cubic_abs(u_np, f_np), what="fused F")
    assert_close(c.host(gu2), gu_ref, su, what="fused g_u")
    assert_close(c.host(gf2), gf_ref, sf, what="fused g_f")


def _fd_dot(w, F_plus, F_minus, h):
    # w^T (F(x + h d) - F(x - h d)) / 2h: the difference is taken entry by
    # entry first, so the two large dot products never cancel each other
    return float(torch.dot(w, F_plus - F_minus)) / (2 * h)


def test_full_fd_config1():
    """Every coordinate of g_u and g_f against central differences (h = 1e-6)
    on the 16 x 16 x 10 mesh (3,179 DoFs)."""
    say("autograd per-coordinate FD 16x16x10")
    base = meshgen.tri_square(16)
    c = Case(base, 10, "P1")
    assert c.n == 3179
    prob = _prob(c)
    u = c.dev(meshgen.uniform_values(c.n, seed=51)).requires_grad_(True)
    f = c.dev(meshgen.uniform_values(c.n, seed=52)).requires_grad_(True)
    w = c.dev(meshgen.uniform_values(c.n, seed=53))
    cubic_residual(u, f, prob).backward(w)
    gu = c.host(u.grad)
    gf = c.host(f.grad)
    h = 1e-6
    fd_u = np.zeros(c.n)
    fd_f = np.zeros(c.n)
    with torch.no_grad():
        ud, fd = u.detach(), f.detach()
        for i in range(c.n):
            e = torch.zeros_like(ud)
            e[i] = h
            fd_u[i] = _fd_dot(w, cubic_residual(ud + e, fd, prob), cubic_residual(ud - e, fd, prob), h)
            fd_f[i] = _fd_dot(w, cubic_residual(ud, fd + e, prob), cubic_residual(ud, fd - e, prob), h)
    for name, fdv, g in (("g_u", fd_u, gu), ("g_f", fd_f, gf)):
        err = np.abs(fdv - g)
        bound = 1e-6 * np.abs(g) + 1e-9 * np.abs(g).max()
        worst = int(np.argmax(err / bound))
        assert np.all(err <= bound), (name, worst, fdv[worst], g[worst])


def test_config4_autograd_at_size():
    """The 256 x 256 x 50 differentiation case through the autograd path in
    the autotuned launch: g_u, g_f on sampled columns against the oracle, and
    eight seeded directional central differences (h = 1e-6) for each."""
    say("autograd 256x256x50 cubic")
    base = meshgen.tri_square(256)
    lam = 50
    c = Case(base, lam, "P1")
    u_np = meshgen.uniform_values(c.n, seed=31)
    f_np = meshgen.uniform_values(c.n, seed=32)
    w_np = meshgen.uniform_values(c.n, seed=meshgen.SEED_COTAN)
    u, f, w = c.dev(u_np), c.dev(f_np), c.dev(w_np)
    tmp = [c.V.zeros() for _ in range(2)]
    exm.autotune(exm.EXM_K_CUBIC, c.mesh, c.X, c.Vx,
                 [(u, c.V, exm.EXM_READ), (f, c.V, exm.EXM_READ), (tmp[0], c.V, exm.EXM_INC)])
    exm.autotune(exm.EXM_K_CUBIC_VJP, c.mesh, c.X, c.Vx,
                 [(u, c.V, exm.EXM_READ), (w, c.V, exm.EXM_READ), (tmp[0], c.V, exm.EXM_INC),
                  (tmp[1], c.V, exm.EXM_INC)])
    prob = _prob(c)
    ug = u.clone().requires_grad_(True)
    fg = f.clone().requires_grad_(True)
    cubic_residual(ug, fg, prob).backward(w)
    gu, gf = c.host(ug.grad), c.host(fg.grad)
    rng = np.random.default_rng(80)
    verts = rng.choice(base.n_vertices, 64, replace=False)
    cells = np.nonzero(np.isin(base.cell_vertex, verts).any(axis=1))[0]
    gur, gfr = c.ref.cubic_vjp(u_np, w_np, cells=cells)
    gus, gfs = c.ref.vjp_abs(u_np, w_np, cells=cells)
    S = c.ref.num_v.column_starts(0)
    idx = (S[verts][:, None] + np.arange(lam + 1)[None, :]).ravel()
    assert_close(gu[idx], gur[idx], gus[idx], what="autograd g_u, sampled columns")
    assert_close(gf[idx], gfr[idx], gfs[idx], what="autograd g_f, sampled columns")
    h = 1e-6
    with torch.no_grad():
        for k in range(8):
            du = c.dev(meshgen.uniform_values(c.n, seed=300 + k))
            df = c.dev(meshgen.uniform_values(c.n, seed=400 + k))
            fd_u = _fd_dot(w, cubic_residual(u + h * du, f, prob), cubic_residual(u - h * du, f, prob), h)
            fd_f = _fd_dot(w, cubic_residual(u, f + h * df, prob), cubic_residual(u, f - h * df, prob), h)
            an_u = float(torch.dot(ug.grad, du))
            an_f = float(torch.dot(fg.grad, df))
            say(f"  direction {k}: u {fd_u:.12e} vs {an_u:.12e}, f {fd_f:.12e} vs {an_f:.12e}")
            assert abs(fd_u - an_u) <= 1e-6 * abs(an_u), (k, fd_u, an_u)
            assert abs(fd_f - an_f) <= 1e-6 * abs(an_f), (k, fd_f, an_f)


@pytest.mark.parametrize("space", sorted(exm.ELEMENTS))
def test_mass_action_adjoint(space):
    base = meshgen.tri_square(7)
    c = Case(base, 6, space, terrain=0.1)
    prob = _prob(c)
    x = c.dev(meshgen.uniform_values(c.n, seed=61)).requires_grad_(True)
    w_np = meshgen.uniform_values(c.n, seed=62)
    mass_action(x, prob).backward(c.dev(w_np))
    assert_close(c.host(x.grad), c.ref.mass(w_np), c.ref.mass_abs(w_np), what=f"M^T w {space}")
