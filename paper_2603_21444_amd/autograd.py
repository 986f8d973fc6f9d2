"""torch.autograd.Function around the HIP product and its backward.

C = A B at fixed sparsity: the patterns of A and B are constants, their
values are the differentiable inputs, and the pattern of C is computed once
(symbolic pass) and reused.  backward() runs spgemm_backward:
dA = (dC B^T) on S(A), dB = (A^T dC) on S(B), or, for a pattern made with
deterministic=True, spgemm_backward_deterministic (dB the same bits on
every run).  Every step runs in the HIP library; torch only holds memory
and the autograd graph.
"""
from __future__ import annotations

import torch

from . import binding


class SpGEMMFunction(torch.autograd.Function):
    """C_vals = SpGEMMFunction.apply(A_vals, B_vals, A_pat, B_pat, ctx_plan)

    A_pat / B_pat are DeviceCSR patterns (row_ptr, col_idx; their vals are
    ignored); ctx_plan is a SpGEMMPattern holding the plan and C's pattern.
    """

    @staticmethod
    def forward(ctx, a_vals, b_vals, A_pat, B_pat, pat):
        A = binding.DeviceCSR(A_pat.shape, A_pat.row_ptr, A_pat.col_idx, a_vals.detach())
        B = binding.DeviceCSR(B_pat.shape, B_pat.row_ptr, B_pat.col_idx, b_vals.detach())
        col, vals = pat.plan.numeric([A], [B], pat.row_ptr, pat.nnz, col=pat.col_tmp)
        ctx.save_for_backward(a_vals, b_vals)
        ctx.A_pat, ctx.B_pat, ctx.pat = A_pat, B_pat, pat
        return vals

    @staticmethod
    def backward(ctx, dc):
        a_vals, b_vals = ctx.saved_tensors
        A = binding.DeviceCSR(ctx.A_pat.shape, ctx.A_pat.row_ptr, ctx.A_pat.col_idx, a_vals.detach())
        B = binding.DeviceCSR(ctx.B_pat.shape, ctx.B_pat.row_ptr, ctx.B_pat.col_idx, b_vals.detach())
        pat = ctx.pat
        dC = binding.DeviceCSR((A.shape[0], B.shape[1]), pat.row_ptr, pat.col_idx,
                               dc.contiguous().to(a_vals.dtype))
        dA, dB = pat.plan.backward(A, B, dC, ctx.needs_input_grad[0], ctx.needs_input_grad[1],
                                   deterministic=pat.deterministic)
        return dA, dB, None, None, None


class SpGEMMPattern:
    """Symbolic pass of C = A B, done once for fixed patterns."""

    def __init__(self, A_pat: binding.DeviceCSR, B_pat: binding.DeviceCSR, plan=None,
                 deterministic: bool = False):
        self.plan = plan or binding.Plan()
        self.deterministic = deterministic
        self.row_ptr, self.nnz = self.plan.symbolic([A_pat], [B_pat])
        dev = A_pat.row_ptr.device
        self.col_tmp = torch.empty(max(self.nnz, 0), dtype=torch.int32, device=dev)
        # one numeric pass fixes C's column order
        self.col_idx, _ = self.plan.numeric([A_pat], [B_pat], self.row_ptr, self.nnz)
        self.shape = (A_pat.shape[0], B_pat.shape[1])


def spgemm_values(a_vals, b_vals, A_pat, B_pat, pattern: SpGEMMPattern):
    """Differentiable C values (aligned with pattern.col_idx)."""
    return SpGEMMFunction.apply(a_vals, b_vals, A_pat, B_pat, pattern)
