"""torch.autograd.Function whose backward is the library's exact gradient (Section 6.2).

``P1Energy.apply(vhat, mesh, prec)`` returns the 0-d energy J(vhat) on the device.

When ``vhat`` requires grad, the forward pass computes the energy and the exact gradient in
one pass over the mesh (``p1e_energy_forces``, which keeps the gradient on the device), and
the backward pass scales the kept gradient by the incoming gradient, a device-side scalar
(``p1e_grad_gather``). If another call rewrote the kept gradient between the two passes,
backward recomputes it at the saved input. The bad-element count of the forward pass is kept
on ``mesh.last_flag``.
"""

import torch


class P1Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vhat, mesh, prec="mixed"):
        if vhat.requires_grad:
            out3, flag, gen = mesh.energy_forces(vhat.detach(), prec)
            ctx.save_for_backward(vhat)
            ctx.gen = gen
        else:
            out3, flag = mesh.energy(vhat, prec)
        ctx.mesh, ctx.prec = mesh, prec
        mesh.last_flag = flag
        return out3[0]

    @staticmethod
    def backward(ctx, grad_j):
        (vhat,) = ctx.saved_tensors
        mesh = ctx.mesh
        scale = grad_j.reshape(1).to(torch.float64).contiguous()
        if mesh.forces_gen == ctx.gen:
            g = mesh.grad_gather(ctx.prec, scale=scale)
        else:
            mesh.energy_forces(vhat, ctx.prec)
            g = mesh.grad_gather(ctx.prec, scale=scale)
        return g, None, None


def p1_energy(vhat, mesh, prec="mixed"):
    """J(vhat) as a differentiable 0-d tensor."""
    return P1Energy.apply(vhat, mesh, prec)
