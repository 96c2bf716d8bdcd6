"""Differentiable contraction: a torch.autograd.Function whose backward is the
library's hand-written block-sparse backward (sym_contract_backward).

For L = <C, G> with C = A . B, the gradients per sector are
dA_s = G_s B_s^T and dB_s = A_s^T G_s (the adjoint of the block-wise
multiply eq:blockmult), split back into A's and B's layouts.
"""
from __future__ import annotations

import torch

from .tensor import Context, SymTensor


class SymContract(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a_data, b_data, A: SymTensor, B: SymTensor, axes_a, axes_b, compute, sctx: Context):
        A.set_data(a_data.detach())
        B.set_data(b_data.detach())
        C = sctx.contract(A, B, axes_a, axes_b, compute)
        ctx.meta = (A, B, C, tuple(axes_a), tuple(axes_b), compute, sctx)
        ctx.save_for_backward(a_data, b_data)
        return C.data

    @staticmethod
    def backward(ctx, grad_c):
        A, B, C, axes_a, axes_b, compute, sctx = ctx.meta
        a_data, b_data = ctx.saved_tensors
        A.set_data(a_data.detach())
        B.set_data(b_data.detach())
        dC = sctx.tensor(C.spec, C.n_row, "f32", data=grad_c.detach().contiguous().float())
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dA, dB = sctx.contract_backward(A, B, dC, axes_a, axes_b, compute, need_a=need_a, need_b=need_b)
        return (dA.data if need_a else None, dB.data if need_b else None, None, None, None, None, None, None)


def contract(sctx: Context, A: SymTensor, B: SymTensor, axes_a, axes_b, compute="f32") -> torch.Tensor:
    """C's data buffer (flat, in C's layout) with autograd through A.data and B.data."""
    return SymContract.apply(A.data, B.data, A, B, tuple(axes_a), tuple(axes_b), compute, sctx)
