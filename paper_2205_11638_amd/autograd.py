"""torch.autograd.Function around the unrolled solver (forward and backward run in libdd.so).

DualLowerBound.apply(inst, c, omega, alpha_hat, T, ckpt_every) returns the dual lower bound (D)
after T iterations of Alg. 1 started from lambda = c/|J_i|, M = 0, with alpha = softmax over J_i
of alpha_hat (Alg. 3).  Its backward is the library's hand-written reverse mode (Alg. 2 through
every pass, checkpointed); gradients flow to c, omega and alpha_hat.  The paper maximizes this
loss (Sec. "Loss"), so a torch optimizer should minimize its negative.
"""
from __future__ import annotations

import torch


class DualLowerBound(torch.autograd.Function):
    @staticmethod
    def forward(ctx, inst, c, omega, alpha_hat, T, ckpt_every=0):
        c32 = c.detach().to(torch.float32).contiguous()
        om = omega.detach().to(torch.float32).contiguous()
        ah = alpha_hat.detach().to(torch.float32).contiguous()
        inst.set_costs(c32)
        alpha = inst.seg_softmax(ah)
        inst.set_params(om, alpha)
        lb = inst.forward_unrolled(int(T), int(ckpt_every))
        ctx.inst = inst
        ctx.save_for_backward(alpha)
        ctx.dtypes = (c.dtype, omega.dtype, alpha_hat.dtype)
        return torch.tensor(lb, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, grad):
        (alpha,) = ctx.saved_tensors
        inst = ctx.inst
        d_omega, d_alpha, d_c = inst.backward(float(grad.item()))
        d_alpha_hat = inst.seg_softmax_vjp(alpha, d_alpha)
        tc, tw, ta = ctx.dtypes
        return None, d_c.to(tc), d_omega.to(tw), d_alpha_hat.to(ta), None, None


def dual_lower_bound(inst, c, omega, alpha_hat, T, ckpt_every=0):
    return DualLowerBound.apply(inst, c, omega, alpha_hat, T, ckpt_every)
