"""Amplitudes as a differentiable function of the u3 angles.

Forward: rebuild the u3 leaves from the angles on the GPU and contract the
requested slices. Backward: libltn's adjoint contraction, which pulls the
incoming gradient back to the leaves and through the u3 chain rule to the
angles (FP64 accumulation). It recomputes every slice's intermediates,
except when the forward ran as one batch on a plan bound for gradients:
those intermediates are still in the gradient workspace, so the backward
leaves the parameters as they are (same angles) and libltn reuses them.
"""
import torch

from .plan import Plan


class Amplitudes(torch.autograd.Function):
    @staticmethod
    def forward(ctx, angles: torch.Tensor, plan: Plan, slice_ids, mode: str = "c64"):
        plan.set_params(angles.detach().to(torch.float64))
        out = plan.new_output(angles.device)
        plan.execute(slice_ids, out, mode)
        ctx.plan = plan
        ctx.slice_ids = slice_ids
        ctx.mode = mode
        ctx.params_token = plan.params_token
        ctx.save_for_backward(angles)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (angles,) = ctx.saved_tensors
        plan = ctx.plan
        if plan.params_token != ctx.params_token:  # parameters set again since the forward
            plan.set_params(angles.detach().to(torch.float64))
        g = plan.execute_grad(ctx.slice_ids, grad_out.to(torch.complex128).contiguous(), None,
                              None, ctx.mode)
        return g.to(angles.dtype), None, None, None
