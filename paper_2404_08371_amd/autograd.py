"""torch.autograd binding of the operator apply y = A(k) x.

The forward map on the macro-local layout is y = S L(k) x: macro-local
applies L followed by the interface sum S over the copies of shared DoFs.
Its transpose is L(k)^T S = L(k) S (L is symmetric, boundary masking
included), so the backward pass first sums dL/dy over copies and then runs
the library's hand-written reverse-mode kernels: for the div(k grad) and
epsilon operators dL/dx = L(k) (S dL/dy) and dL/dk_m = (S dL/dy) . (dL/dk_m) x
per coefficient copy (P1: one fused launch; P2 and epsilon: the local apply
plus a coefficient-gradient launch); for the Laplacians dL/dx is a
macro-local apply (they have no coefficient).
"""
import torch

from .operators import P1_DIVKGRAD, P2_DIVKGRAD, P2V_EPSILON


class TmfApply(torch.autograd.Function):
    """y = TmfApply.apply(x, k, op) with gradients for x and (div(k grad), epsilon) k."""

    @staticmethod
    def forward(ctx, x, k, op):
        y = op.apply(x, k)
        ctx.op = op
        ctx.save_for_backward(x, k)
        return y

    @staticmethod
    def backward(ctx, gy):
        op = ctx.op
        x, k = ctx.saved_tensors
        gys = op.interface_sum_(gy.contiguous().clone())
        need_x, need_k = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if op.kind in (P1_DIVKGRAD, P2_DIVKGRAD, P2V_EPSILON):
            gx, gk = op.adjoint(k, x, gys, want_gk=need_k)
            return (gx if need_x else None), (gk if need_k else None), None
        if need_k:
            raise NotImplementedError("the coefficient gradient is implemented for the div(k grad) and epsilon operators")
        return op.apply_local(gys, k), None, None


def apply(x, k, op):
    """Differentiable y = A(k) x."""
    return TmfApply.apply(x, k, op)
