"""torch.autograd.Function wrappers over the library's forward and adjoint
column loops.

The adjoint kernels are hand-written: where the forward gathers a field and
scatters (increments) the residual, the vector-Jacobian product gathers the
cotangent and scatters into the gradients.  PyTorch only carries the tensors
and the graph bookkeeping; every arithmetic step runs in libexm.
"""
from __future__ import annotations

import torch

from . import (CONTINUOUS, ELEMENTS, EXM_INC, EXM_K_CUBIC, EXM_K_CUBIC_FUSED, EXM_K_CUBIC_VJP, EXM_K_MASS, EXM_READ,
               EXM_WRITE, Mesh, Space, par_loop)

# elements whose DoFs are shared between cells or layers: their outputs are INC
_SHARED = frozenset(ELEMENTS[name] for name in CONTINUOUS)


class Extruded:
    """A mesh with its coordinate space and field, and a field space."""

    def __init__(self, mesh: Mesh, coord_space: Space, coords, space: Space, **opts):
        self.mesh = mesh
        self.coord_space = coord_space
        self.coords = coords
        self.space = space
        self.opts = opts

    def _out_access(self):
        return EXM_INC if self.space.element in _SHARED else EXM_WRITE

    def mass(self, x):
        y = self.space.zeros()
        par_loop(EXM_K_MASS, self.mesh, self.coords, self.coord_space,
                 [(x, self.space, EXM_READ), (y, self.space, self._out_access())], **self.opts)
        return y

    def cubic(self, u, f):
        F = self.space.zeros()
        par_loop(EXM_K_CUBIC, self.mesh, self.coords, self.coord_space,
                 [(u, self.space, EXM_READ), (f, self.space, EXM_READ), (F, self.space, EXM_INC)], **self.opts)
        return F

    def cubic_vjp(self, u, w):
        gu = self.space.zeros()
        gf = self.space.zeros()
        par_loop(EXM_K_CUBIC_VJP, self.mesh, self.coords, self.coord_space,
                 [(u, self.space, EXM_READ), (w, self.space, EXM_READ), (gu, self.space, EXM_INC),
                  (gf, self.space, EXM_INC)], **self.opts)
        return gu, gf

    def cubic_fused(self, u, f, w):
        F = self.space.zeros()
        gu = self.space.zeros()
        gf = self.space.zeros()
        par_loop(EXM_K_CUBIC_FUSED, self.mesh, self.coords, self.coord_space,
                 [(u, self.space, EXM_READ), (f, self.space, EXM_READ), (w, self.space, EXM_READ),
                  (F, self.space, EXM_INC), (gu, self.space, EXM_INC), (gf, self.space, EXM_INC)], **self.opts)
        return F, gu, gf


def _c(t):
    return t.detach().contiguous()


class CubicResidual(torch.autograd.Function):
    """F(u, f)_i = integral (u^3 - f) v_i dx on P1 x P1; backward = the VJP kernel."""

    @staticmethod
    def forward(ctx, u, f, prob: Extruded):
        ctx.prob = prob
        ctx.save_for_backward(u)
        return prob.cubic(_c(u), _c(f))

    @staticmethod
    def backward(ctx, w):
        (u,) = ctx.saved_tensors
        gu, gf = ctx.prob.cubic_vjp(_c(u), _c(w))
        return gu, gf, None


class MassAction(torch.autograd.Function):
    """y = M x (the residual of the integral of x v); backward g = M^T w = M w."""

    @staticmethod
    def forward(ctx, x, prob: Extruded):
        ctx.prob = prob
        return prob.mass(_c(x))

    @staticmethod
    def backward(ctx, w):
        return ctx.prob.mass(_c(w)), None


def cubic_residual(u, f, prob: Extruded):
    return CubicResidual.apply(u, f, prob)


def mass_action(x, prob: Extruded):
    return MassAction.apply(x, prob)


def cubic_residual_with_vjp(u, f, w, prob: Extruded):
    """F(u, f) and its VJP (g_u, g_f) with cotangent w from one fused sweep."""
    return prob.cubic_fused(_c(u), _c(f), _c(w))
