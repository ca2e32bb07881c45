"""torch.autograd.Function over the HIP forward / adjoint pair.

forward: fwi_forward_keep — modelled traces; what the backward needs (the
whole pressure history when it fits the plan's budget, else checkpoints every
k steps and the last segment's history) and the prepared model stay in a
workspace held by the autograd context.  backward: fwi_adjoint_kept with the
incoming gradient of the traces as adjoint source — a checkpointed plan
recomputes its segments, so memory is O(sqrt(nt) N) instead of O(nt N).

Any loss written in torch on the traces differentiates through to the model
parameters of the chosen parameterization (Table 1 of the paper).
"""
import torch

from . import _lib as L


class FWIFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m1, m2, wavelet, plan, param):
        ws = plan.new_workspace(L.FWI_OP_GRADIENT)
        traces = plan.forward_keep(param, m1, m2, wavelet, ws)
        ctx.plan, ctx.param, ctx.ws = plan, param, ws
        ctx.save_for_backward(m1, m2, wavelet)
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        m1, m2, wavelet = ctx.saved_tensors
        if ctx.ws is None:
            raise RuntimeError("FWIFunction.backward called twice: the kept state is consumed")
        g1, g2 = ctx.plan.adjoint_kept(ctx.param, m1, m2, wavelet, grad_traces.contiguous(),
                                       ctx.ws)
        ctx.ws = None
        return g1, g2, None, None, None


def model_traces(plan, param, m1, m2, wavelet):
    """Differentiable traces [S][nrec][nt] of the model (m1, m2) in `param`."""
    return FWIFunction.apply(m1, m2, wavelet, plan, param)
