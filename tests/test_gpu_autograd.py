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


def test_full_fd_tiny():
    # every coordinate of the gradient against central differences on a tiny mesh
    base = meshgen.tri_square(2)
    c = Case(base, 2, "P1")
    prob = _prob(c)
    u = c.dev(meshgen.uniform_values(c.n, seed=51)).requires_grad_(True)
    f = c.dev(meshgen.uniform_values(c.n, seed=52))
    w = c.dev(meshgen.uniform_values(c.n, seed=53))
    cubic_residual(u, f, prob).backward(w)
    g = u.grad.clone()
    h = 1e-6
    with torch.no_grad():
        for i in range(c.n):
            e = torch.zeros_like(u)
            e[i] = h
            fd = (torch.dot(w, cubic_residual(u + e, f, prob)) - torch.dot(w, cubic_residual(u - e, f, prob))) / (2 * h)
            assert abs(float(fd - g[i])) <= 1e-6 * max(1e-3, abs(float(g[i]))), (i, float(fd), float(g[i]))


@pytest.mark.parametrize("space", ["P1", "DG0", "DG1", "P2"])
def test_mass_action_adjoint(space):
    base = meshgen.tri_square(7)
    c = Case(base, 6, space, terrain=0.1)
    prob = _prob(c)
    x = c.dev(meshgen.uniform_values(c.n, seed=61)).requires_grad_(True)
    w_np = meshgen.uniform_values(c.n, seed=62)
    mass_action(x, prob).backward(c.dev(w_np))
    assert_close(c.host(x.grad), c.ref.mass(w_np), c.ref.mass_abs(w_np), what=f"M^T w {space}")
