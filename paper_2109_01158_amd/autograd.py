"""torch.autograd.Function whose backward is the library's exact gradient (Section 6.2).

``P1Energy.apply(vhat, mesh, prec)`` returns the 0-d energy J(vhat) on the device. When
``vhat`` requires grad, the forward pass runs the fused J + grad J call once and keeps the
gradient, so backward is only ``grad_output * g`` (no second pass over the mesh).
"""

import torch


class P1Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vhat, mesh, prec="mixed"):
        if vhat.requires_grad:
            g, out3, flag = mesh.grad_exact(vhat.detach(), prec)
            ctx.save_for_backward(g)
        else:
            out3, flag = mesh.energy(vhat, prec)
        ctx.mark_non_differentiable(flag)
        return out3[0], flag

    @staticmethod
    def backward(ctx, grad_j, grad_flag):
        (g,) = ctx.saved_tensors
        return grad_j * g, None, None


def p1_energy(vhat, mesh, prec="mixed"):
    """J(vhat) as a differentiable 0-d tensor (the bad-element count is dropped)."""
    J, _ = P1Energy.apply(vhat, mesh, prec)
    return J
