"""torch.autograd.Function around the unrolled solver (forward and backward run in libdd.so).

DualLowerBound.apply(inst, c, omega, alpha_hat, T, ckpt_every) returns the dual lower bound (D)
after T iterations of Alg. 1 started from lambda = c/|J_i|, M = 0, with alpha = softmax over J_i
of alpha_hat (Alg. 3).  Its backward is the library's hand-written reverse mode (Alg. 2 through
every pass, checkpointed); gradients flow to c, omega and alpha_hat.  The paper maximizes this
loss (Sec. "Loss"), so a torch optimizer should minimize its negative.

DualRound.apply(inst, omega_hat, alpha_hat, theta_hat, T, ckpt_every) is one round of the
pipeline: output transforms, non-parametric update of the current state, T iterations, bound.
"""
from __future__ import annotations

import torch

from .binding import DD_E_STATE, DDError


def _check_record(ctx):
    """The instance's recorded forward must still be this node's: a later forward on the same
    instance (another node of the graph) replaces it, and its backward would differentiate that one."""
    now = ctx.inst.record_serial()
    if now != ctx.serial:
        raise DDError(DD_E_STATE, f"this node's unrolled forward (record {ctx.serial}) is no longer the "
                                  f"instance's record ({now}): run its backward before another forward "
                                  "on the same instance, or use one instance per node")


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
        ctx.serial = inst.record_serial()
        ctx.save_for_backward(alpha)
        ctx.dtypes = (c.dtype, omega.dtype, alpha_hat.dtype)
        return torch.tensor(lb, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, grad):
        (alpha,) = ctx.saved_tensors
        inst = ctx.inst
        _check_record(ctx)
        d_omega, d_alpha, d_c = inst.backward(float(grad.item()))
        d_alpha_hat = inst.seg_softmax_vjp(alpha, d_alpha)
        tc, tw, ta = ctx.dtypes
        return None, d_c.to(tc), d_omega.to(tw), d_alpha_hat.to(ta), None, None


def dual_lower_bound(inst, c, omega, alpha_hat, T, ckpt_every=0):
    return DualLowerBound.apply(inst, c, omega, alpha_hat, T, ckpt_every)


class DualRound(torch.autograd.Function):
    """One round of the paper's pipeline without the predictor network (Sec. "Overall pipeline"):
    the raw predictions (omega_hat, alpha_hat, theta_hat) go through Alg. 3's output transforms,
    the non-parametric update (eq. 2) moves the instance's current multipliers by theta, then T
    iterations of Alg. 1 run from there and the bound (D) is returned.  The state the round starts
    from is a constant (earlier rounds run without gradients); the instance is left at the end of
    the round, ready for the next one.  Gradients flow to all three predictions."""

    @staticmethod
    def forward(ctx, inst, omega_hat, alpha_hat, theta_hat, T, ckpt_every=0):
        wh, ah, th = (x.detach().to(torch.float32).contiguous() for x in (omega_hat, alpha_hat, theta_hat))
        omega, alpha, _ = inst.param_transform(wh, ah)
        inst.set_params(omega, alpha)
        inst.nonparam_update(th)
        lb = inst.forward_unrolled_from_state(int(T), int(ckpt_every))
        ctx.inst = inst
        ctx.serial = inst.record_serial()
        ctx.save_for_backward(omega, alpha)
        ctx.dtypes = (omega_hat.dtype, alpha_hat.dtype, theta_hat.dtype)
        return torch.tensor(lb, dtype=torch.float64, device=omega_hat.device)

    @staticmethod
    def backward(ctx, grad):
        omega, alpha = ctx.saved_tensors
        inst = ctx.inst
        _check_record(ctx)
        d_omega, d_alpha, d_lam0, _ = inst.backward_state(float(grad.item()))
        # lambda_0 = lambda_prev + theta_hat - mean over J_i: its adjoint is the centring of d_lam0
        dwh, dah, dth = inst.param_transform_vjp(omega, alpha, d_omega, d_alpha, d_lam0)
        tw, ta, tt = ctx.dtypes
        return None, dwh.to(tw), dah.to(ta), dth.to(tt), None, None


def dual_round(inst, omega_hat, alpha_hat, theta_hat, T, ckpt_every=0):
    return DualRound.apply(inst, omega_hat, alpha_hat, theta_hat, T, ckpt_every)
