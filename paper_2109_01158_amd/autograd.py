"""torch.autograd.Function whose backward is the library's exact gradient (Section 6.2).

``P1Energy.apply(vhat, mesh, prec)`` returns the 0-d energy J(vhat) on the device.

When ``vhat`` requires grad, the forward pass computes the energy and the exact gradient in
one pass over the mesh (``p1e_grad_exact``) into a fresh device buffer held by the autograd
context, and the backward pass hands that buffer back scaled in place by the incoming
gradient, a device-side scalar (``p1e_grad_scale``, which writes nothing when the scale is 1).
A second backward through the same graph (``retain_graph=True``) recomputes the gradient at
the saved input. The bad-element count of the forward pass is kept on ``mesh.last_flag``.
"""

import torch


class P1Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vhat, mesh, prec="mixed"):
        if vhat.requires_grad:
            g, out3, flag = mesh.grad_exact(vhat.detach(), prec)
            ctx.save_for_backward(vhat)
            ctx.g = g
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
        g, ctx.g = ctx.g, None  # handed over: autograd may keep it as vhat.grad
        if g is None:
            g, _, _ = mesh.grad_exact(vhat.detach(), ctx.prec)
        return mesh.grad_scale(g, scale), None, None


def p1_energy(vhat, mesh, prec="mixed"):
    """J(vhat) as a differentiable 0-d tensor."""
    return P1Energy.apply(vhat, mesh, prec)
