"""torch.autograd.Function whose backward is the library's exact gradient (Section 6.2).

``P1Energy.apply(vhat, mesh, prec)`` returns the 0-d energy J(vhat) on the device.

When ``vhat`` requires grad, the forward pass computes the energy and the exact gradient in
one pass over the mesh (``p1e_grad_exact``) into a fresh device buffer held by the autograd
context, and the backward pass hands that buffer back scaled in place by the incoming
gradient, a device-side scalar (``p1e_grad_scale``, which writes nothing when the scale is 1).
A second backward through the same graph (``retain_graph=True``) recomputes the gradient at
the saved input. The bad-element count of the forward pass is kept on ``mesh.last_flag``.

``GraphedStep`` captures one such step (forward and backward) in a HIP graph and replays it.
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


class GraphedStep:
    """One J + exact grad J step through the autograd hook, captured once in a HIP graph
    (``torch.cuda.CUDAGraph``) and replayed: the step's kernels (element tiles, halo rows, the
    in-place scaling of the backward pass) for one graph launch on the host.

    Every replay reads ``vhat``'s memory as it is then (change it in place, e.g.
    ``vhat.data.copy_(...)``) and rewrites ``J`` (0-d) and ``grad`` in place. The step runs on
    a leaf of its own that shares ``vhat``'s memory, so that its gradient accumulator is made
    on the capture's stream: one that earlier eager backward passes made for ``vhat`` would sit
    on another stream, and the captured step would have to synchronise with it, which a
    capture cannot hold. The capture runs ``warmup`` eager steps on a side stream first, as
    torch requires; ``replay`` launches on the current stream. The mesh's scratch arrays are
    shared with eager calls on the same mesh, so replays and eager calls must not overlap
    (issue them on one stream)."""

    def __init__(self, vhat, mesh, prec="mixed", warmup=3):
        dev = vhat.device
        x = vhat.detach().requires_grad_(True)  # a new leaf on vhat's memory
        seed = torch.ones((), dtype=torch.float64, device=dev)

        def step():
            x.grad = None
            J = p1_energy(x, mesh, prec)
            torch.autograd.backward(J, seed)
            return J

        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            for _ in range(warmup):
                step()
        torch.cuda.current_stream(dev).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.J = step()
        # the graph's kernels read the mesh's device arrays: keep the mesh alive with it
        self.vhat, self.mesh, self.grad, self._leaf, self._seed = vhat, mesh, x.grad, x, seed

    def replay(self):
        """Runs the step; returns (J, grad), the tensors it rewrites."""
        self.graph.replay()
        return self.J, self.grad
