"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and driven through every entry point on small meshes:
no out-of-bounds access, use after free or undefined behaviour."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import numpy as np
import oracle
from paper_1604_05937_amd import meshgen

base = meshgen.tri_square(5)
lam = 4
vc = meshgen.extruded_vertex_coords(base, lam, terrain=0.1)
for space in ("P1", "P2", "DG0", "DG1", "CG1xDG0", "CG1xDG1", "DG0xCG1", "DG0xDG1", "DG1xCG1", "DG1xDG0"):
    pr = oracle.Problem(base, lam, space, vc)
    x = meshgen.uniform_values(pr.n_dofs, seed=3)
    pr.mass(x); pr.mass_abs(x); pr.mass(x, cells=np.array([0, 7, 11]))
    pr.mass_matrix(); pr.mass_matrix_abs()
    if not oracle.is_continuous(pr.space) or space.startswith("CG1xDG"):
        if space not in ("DG0xCG1", "DG1xCG1"):
            pr.facet_jump(x); pr.facet_jump_abs(x)
pr = oracle.Problem(base, lam, "P1", vc)
u, f, w = (meshgen.uniform_values(pr.n_dofs, seed=s) for s in (4, 5, 6))
pr.cubic(u, f); pr.cubic_vjp(u, w); pr.cubic_jvp(u, u, f); pr.cubic_fused(u, f, w)
pr.cubic_abs(u, f); pr.vjp_abs(u, w); pr.cubic_jacobian(u); pr.cubic_jacobian_abs(u)
rng = meshgen.layer_ranges(base, lam, kind="random")
for space in ("P1", "DG0", "P2"):
    pv = oracle.Problem(base, lam, space, vc, layers=rng)
    pv.mass(meshgen.uniform_values(pv.n_dofs, seed=7))
dofs = meshgen.entity_dofs(base)
oracle.number_mixed(base.counts, lam, dofs, base.cell_vertex, base.cell_edge)
nd = meshgen.cell_degrees(base, frac_dg1=0.5)
oracle.mixed_dg_mass(base, lam, vc, nd, meshgen.uniform_values(int(base.n_cells * lam * 0 + (nd.sum() * lam)), seed=8))
colour, n = oracle.greedy_colour(base.cell_vertex, base.n_vertices)
out = np.zeros(pr.n_dofs)
oracle.par_loop_threaded(oracle.FORM_MASS, pr.space, pr.num_v, pr.num_x, pr.X, [u], [out], threads=3, colour=colour)
print("sanitized oracle ok", flush=True)
'''


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fPIC", "-shared",
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(lib), "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    env = dict(os.environ, ORACLE_LIB=str(lib), LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", DRIVER], capture_output=True, text=True, env=env, cwd=ROOT,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
