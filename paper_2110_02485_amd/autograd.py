"""torch.autograd.Function over the fixed-k truncated R-tSVD restoration.

Forward: X_k = V_k * S_k^{-1} * U_k^T * B (R-tSVD factor with a fixed Gaussian tensor, q = 0,
fixed k) through librtsvd.  Backward: the library's hand-written adjoint (rtsvd_solve_vjp) gives
dL/dB and, for an operator A(s) whose derivative dA/ds is supplied, dL/ds; the factor is
recomputed in the backward pass rather than stored.
"""
from __future__ import annotations

import torch

from . import rtsvd as rt


class RtsvdRestore(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B, s, A, dA_ds, omega, k, oversample):
        precision = "fp64" if A.dtype == torch.float64 else "fp32"
        f = rt.factor(A, k, oversample, 0, precision, omega)
        res = f.solve(B, 1e300, 1.01, k)        # k_start = k_max = k: the truncation index is fixed
        f.close()
        ctx.save_for_backward(A, dA_ds, B, omega)
        ctx.k, ctx.oversample = k, oversample
        return res.X

    @staticmethod
    def backward(ctx, gX):
        A, dA_ds, B, omega = ctx.saved_tensors
        gB, gdot = rt.solve_vjp(A, dA_ds, B, omega, gX.contiguous(), ctx.k, ctx.oversample)
        gs = gdot.to(A.dtype).reshape(()) if gdot is not None else None
        return gB, gs, None, None, None, None, None


def restore(B, s, A, dA_ds, omega, k, oversample):
    """Differentiable fixed-k restoration: returns X; gradients flow to B and to the scalar s."""
    return RtsvdRestore.apply(B, s, A, dA_ds, omega, k, oversample)
