"""Helpers shared by the GPU parity tests (the oracle side stays in oracle/)."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_instance(prob, omega=None, alpha_hat=None, **opts):
    """Instance on cuda:0 with omega / alpha = softmax(alpha_hat) set on the device."""
    import torch

    import paper_2205_11638_amd as dd
    inst = dd.Instance(prob, **opts)
    if omega is not None:
        om = torch.tensor(np.asarray(omega, dtype=np.float32), device="cuda")
        ah = torch.tensor(np.asarray(alpha_hat, dtype=np.float32), device="cuda")
        al = inst.seg_softmax(ah)
        inst.set_params(om, al)
        inst.reset()
        return inst, om, al
    return inst, None, None


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def row_scale(prob, lam):
    """Per-edge scale: sum of |lambda| over the edge's row (the size of path costs in that row)."""
    a = np.abs(lam)
    s = np.add.reduceat(a, prob.row_ptr[:-1]) if prob.m else np.zeros(0)
    s = np.where(np.diff(prob.row_ptr) > 0, s, 0.0)
    return np.repeat(s, np.diff(prob.row_ptr))


def assert_close_scaled(got, ref, scale, rtol, what=""):
    err = np.abs(got - ref)
    bound = rtol * np.maximum(np.maximum(np.abs(ref), scale), 1e-6)
    bad = err > bound
    if bad.any():
        k = int(np.argmax(err / bound))
        raise AssertionError(f"{what}: {int(bad.sum())}/{bad.size} entries off; worst at {k}: got {got[k]!r} "
                             f"ref {ref[k]!r} scale {scale[k]!r} (bound {bound[k]:.3g})")
