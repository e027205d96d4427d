"""The forward operator as a differentiable torch function.

`ProjectFn.apply(vol, grid, optics, rot, defocus, shift)` returns C_i T_i P_i v
for every image (eq. (fwd model) without noise; shift None: T = I) through
csg_project; its backward is the hand-written adjoint (csg_backproject with
the CTF to the first power).  The operator is complex-linear, so for a real
loss L the vector-Jacobian product in torch's convention (dL/dRe + i dL/dIm)
is the adjoint P^T T^* C applied to the incoming image gradient.  Hessian-vector products of a
quadratic loss built from it therefore use the same two kernels, which is how
the paper obtains its HVPs by automatic differentiation (Sec. 3.2).
"""
from __future__ import annotations

import torch

from . import binding as B


class ProjectFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vol, grid: B.Grid, optics: B.Optics, rot, defocus, shift=None):
        ctx.grid, ctx.optics = grid, optics
        ctx.shift = shift
        ctx.save_for_backward(rot, defocus)
        return B.project(grid, optics, rot, defocus, vol.contiguous(), shift=shift)

    @staticmethod
    def backward(ctx, grad_out):
        rot, defocus = ctx.saved_tensors
        g = B.backproject(ctx.grid, ctx.optics, rot, defocus, grad_out.contiguous(), ctf_power=1, scale=1.0,
                          shift=ctx.shift)
        return g, None, None, None, None, None


def project(vol, grid: B.Grid, optics: B.Optics, rot, defocus, shift=None):
    """Differentiable C T P v (see ProjectFn)."""
    return ProjectFn.apply(vol, grid, optics, rot, defocus, shift)


def hvp_autograd(z, grid: B.Grid, optics: B.Optics, rot, defocus, scale: float = 1.0, lam: float = 0.0,
                 shift=None):
    """H z of f(v) = scale/2 sum_i ||C_i P_i v||^2 + lam/2 ||v||^2 obtained by
    differentiating the gradient of f through ProjectFn (the gradient is
    linear in v, so one backward pass of the gradient at z is H z)."""
    v = z.detach().clone().requires_grad_(True)
    y = project(v, grid, optics, rot, defocus, shift)
    f = 0.5 * scale * torch.sum(torch.abs(y) ** 2) + 0.5 * lam * torch.sum(torch.abs(v) ** 2)
    (g,) = torch.autograd.grad(f, v)
    return g
