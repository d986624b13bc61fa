"""Shared set-up for the GPU parity tests: the same seeded inputs go to the
HIP path (through the C ABI) and to the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import paper_1604_05937_amd as exm
from paper_1604_05937_amd import meshgen

# FP64 tolerance (componentwise): |gpu - oracle| <= RTOL * s_i, s_i the
# oracle's assembly of the magnitudes of every term of DoF i, which bounds the
# rounding of any summation order.
RTOL = 1e-12


def say(*msg):
    print(*msg, flush=True)
    sys.stdout.flush()


class Case:
    """One extruded mesh with the coordinate space, a field space and the
    oracle problem on the same inputs."""

    def __init__(self, base, n_layers, space, terrain=0.0, with_oracle=True, layers=None):
        import torch
        self.base = base
        self.n_layers = n_layers
        self.space_name = space
        self.vc = meshgen.extruded_vertex_coords(base, n_layers, terrain=terrain)
        self.layers = layers
        self.mesh = exm.Mesh(base, n_layers, layers=layers)
        self.Vx = exm.Space(self.mesh, "P1")
        self.V = exm.Space(self.mesh, space) if space != "P1" else self.Vx
        self.X = exm.coordinate_field(self.Vx, self.vc)
        self.ref = oracle.Problem(base, n_layers, space, self.vc, layers=layers) if with_oracle else None
        self.torch = torch

    @property
    def n(self) -> int:
        return self.V.n_dofs

    def dev(self, a: np.ndarray):
        return self.torch.from_numpy(np.ascontiguousarray(a)).to("cuda")

    def host(self, t) -> np.ndarray:
        self.torch.cuda.synchronize()
        return t.cpu().numpy()

    def out_access(self):
        return exm.EXM_INC if self.space_name in exm.CONTINUOUS else exm.EXM_WRITE

    def mass(self, x: np.ndarray, **opts) -> np.ndarray:
        xd = self.dev(x)
        y = self.V.zeros()
        exm.par_loop(exm.EXM_K_MASS, self.mesh, self.X, self.Vx,
                     [(xd, self.V, exm.EXM_READ), (y, self.V, self.out_access())], **opts)
        return self.host(y)


def assert_close(got, ref, scale, rtol=RTOL, what=""):
    got = np.asarray(got)
    ref = np.asarray(ref)
    err = np.abs(got - ref)
    bound = rtol * np.asarray(scale) + 1e-300
    bad = np.nonzero(err > bound)[0]
    if bad.size:
        i = bad[np.argmax(err[bad] / bound[bad])]
        raise AssertionError(f"{what}: {bad.size} of {got.size} entries off; worst i={i} got={got[i]!r} "
                             f"ref={ref[i]!r} err={err[i]:.3e} bound={bound[i]:.3e}")
    # also the normwise relative error
    nrm = np.abs(ref).max() if ref.size else 0.0
    if nrm > 0:
        assert err.max() <= rtol * nrm, f"{what}: normwise relative error {err.max() / nrm:.3e}"
