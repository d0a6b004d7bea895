"""Differentiable Poisson solve: phi = S(4 pi G rho) with an adjoint backward.

The discrete solution operator is linear in rho.  With the Laplacian M
symmetric (7-point stencil with the ghosts of Sec. 2.3) and the boundary data
independent of rho, the gradient of a loss L(phi) is

    dL/drho = 4 pi G * S_0(dL/dphi)

where S_0 is the same solve with homogeneous boundary values (Dirichlet faces
set to zero) and, for periodic boxes, the mean of the source removed and the
zero-mean gauge on the result (the projection P_perp of eq.
source_modification is symmetric too).  The library's solve forms
four_pi_G * (source) itself, so dL/drho is exactly the solve of
M lambda = 4 pi G dL/dphi with homogeneous faces: the backward pass is one more
call of the same C ABI as the forward, with dL/dphi in place of rho and the
same options, and its result is returned as it comes.

Both passes run in the library's HIP kernels; this module only arranges the
calls and does no arithmetic on the tensors.  ``rho`` may carry leading batch
dimensions: (..., nz, ny, nx).
"""
from __future__ import annotations

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
        # S is linear: solving with source dL/dphi and the forward's four_pi_G
        # gives 4 pi G S_0(dL/dphi) directly (homogeneous faces: None)
        grad = _solve_many(gphi.detach().contiguous(), ctx.h, ctx.bc, None, ctx.opts)
        return grad, None, None, None, None


def poisson_solve(rho, h, bc="periodic", faces=None, opts=None):
    """Differentiable phi(rho); see :class:`PoissonSolve`."""
    return PoissonSolve.apply(rho, h, bc, faces, opts)
