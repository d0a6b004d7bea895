"""Differentiable Poisson solve: phi = S(4 pi G rho) with an adjoint backward.

The discrete solution operator is linear in rho.  With the Laplacian M
symmetric (7-point stencil with the ghosts of Sec. 2.3) and the boundary data
independent of rho, the gradient of a loss L(phi) is

    dL/drho = 4 pi G * S_0(dL/dphi)

where S_0 is the same solve with homogeneous boundary values (Dirichlet faces
set to zero) and, for periodic boxes, the mean of the source removed and the
zero-mean gauge on the result (the projection P_perp of eq.
source_modification is symmetric too).  So the backward pass costs one more
solve on the GPU, through the same C ABI as the forward.

Both passes run in the library's HIP kernels; this module only arranges the
calls.  ``rho`` may carry leading batch dimensions: (..., nz, ny, nx).
"""
from __future__ import annotations

import dataclasses

import torch

from . import _lib


def _solve_many(src, h, bc, faces, opts):
    """Solve for every trailing 3-D block of ``src`` (float64 CUDA): one
    batched call (one grid class) when there are several blocks and no
    Dirichlet face data, else one solve per block."""
    shape = src.shape
    flat = src.reshape((-1,) + tuple(shape[-3:])).contiguous()
    nb = flat.shape[0]
    if nb > 1 and faces is None:
        phis, _ = _lib.solve_batched([flat[q] for q in range(nb)], [h] * nb, bc, opts=opts)
        return torch.stack(phis).reshape(shape)
    outs = []
    for q in range(nb):
        phi, _ = _lib.solve(flat[q], h, bc, faces=faces, opts=opts)
        outs.append(phi)
    return torch.stack(outs).reshape(shape)


class PoissonSolve(torch.autograd.Function):
    """``PoissonSolve.apply(rho, h, bc, faces, opts)`` -> phi."""

    @staticmethod
    def forward(ctx, rho, h, bc="periodic", faces=None, opts=None):
        opts = opts or _lib.Options()
        ctx.h, ctx.bc, ctx.opts = h, bc, opts
        return _solve_many(rho.detach(), h, bc, faces, opts)

    @staticmethod
    def backward(ctx, gphi):
        o = dataclasses.replace(ctx.opts, four_pi_G=1.0)
        lam = _solve_many(gphi.detach().contiguous(), ctx.h, ctx.bc, None, o)
        return ctx.opts.four_pi_G * lam, None, None, None, None


def poisson_solve(rho, h, bc="periodic", faces=None, opts=None):
    """Differentiable phi(rho); see :class:`PoissonSolve`."""
    return PoissonSolve.apply(rho, h, bc, faces, opts)
