"""Squared-error CP loss as a torch.autograd.Function with a hand-written backward.

    L(A_1..A_N) = || T - [[A_1, ..., A_N]] ||_F^2

(the objective of the paper's eq. objFun without its 1/2). Forward: the float64 Gram
trick of Sec. 3.1.3 from the last mode's MTTKRP and Gram product (`ntf_cp_loss`).
Backward (Sec. 2, eq. def:grad): dL/dA_n = 2 (A_n G_n - P_n) with G_n the Hadamard product
of the other factors' Grams and P_n the mode-n MTTKRP, scaled by the incoming gradient on
the device (`ntf_cp_grad`). The last mode's MTTKRP is the forward's; the others come from
one `ntf_mttkrp_multi` call (for a 3-way tensor one more pass over T, through
Y = T x_3 A_3), so a forward and backward stream a 3-way T twice. Every step runs in libntf's kernels; this module only
sequences the calls.
"""
from __future__ import annotations

import torch


class NTFLoss(torch.autograd.Function):
    """L = ||T - [[A_1..A_N]]||_F^2; T (float32 or bfloat16) is data, factors are float32."""

    @staticmethod
    def forward(ctx, T: torch.Tensor, normT2: torch.Tensor, *factors: torch.Tensor):
        from . import ntf_cp_loss, ntf_gram, ntf_mttkrp
        n = T.dim() - 1
        factors = tuple(f.detach() for f in factors)
        P = ntf_mttkrp(T, factors, n)
        _, G64 = ntf_gram(factors, exclude=n, want32=False)
        loss = ntf_cp_loss(normT2, P, factors[n], G64)
        ctx.save_for_backward(T, *factors)
        ctx.last = (P, G64)
        return loss

    @staticmethod
    def backward(ctx, grad_loss: torch.Tensor):
        from . import ntf_cp_grad, ntf_gram, ntf_mttkrp_multi
        T, *factors = ctx.saved_tensors
        N = T.dim()
        scale = grad_loss.detach()
        if scale.dtype != torch.float64 or not scale.is_contiguous():
            raise TypeError("NTFLoss expects a float64 scalar incoming gradient")
        # the other modes' MTTKRPs in one call (a 3-way tensor's first two share a pass; both
        # are formed whenever one is asked for, so a factor's gradient has the same bits
        # whichever other factors require gradients)
        need = [n for n in range(N - 1) if ctx.needs_input_grad[2 + n]]
        if N == 3 and need:
            need = [0, 1]
        Ps = ntf_mttkrp_multi(T, factors, need) if need else {}
        grads = []
        for n in range(N):
            if not ctx.needs_input_grad[2 + n]:
                grads.append(None)
                continue
            if n == N - 1:
                P, G64 = ctx.last
            else:
                P = Ps[n]
                _, G64 = ntf_gram(factors, exclude=n, want32=False)
            grads.append(ntf_cp_grad(factors[n], P, G64, scale=scale, alpha=2.0))
        ctx.last = None
        return (None, None, *grads)


def ntf_loss(T: torch.Tensor, factors, normT2: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable ||T - [[factors]]||_F^2 (float64 scalar on T's device)."""
    from . import ntf_norm2
    if normT2 is None:
        normT2 = ntf_norm2(T)
    return NTFLoss.apply(T, normT2, *factors)
