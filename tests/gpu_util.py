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


def _row_of_width(rng, n, lo, hi, k, amax):
    """A knapsack row (k variables, a ~ U{1..amax}) whose diagram width lies in (lo, hi]: capacities are
    tried on one-row programs until the library reports such a width."""
    import synth
    import paper_2205_11638_amd as dd
    cols = rng.choice(n, size=k, replace=False)
    a = rng.integers(1, amax + 1, size=k)
    for frac in np.linspace(0.05, 0.5, 46):
        rhs = int(frac * a.sum())
        one = synth.generators._from_rows(n, -np.ones(n), [(cols, a, -1, rhs)], "probe")
        w = dd.Instance(one).stats["max_width"]
        if lo < w <= hi:
            return (cols, a, -1, rhs), w
    raise AssertionError(f"no capacity gives a width in ({lo}, {hi}]")


def wide_class_problem(rmax):
    """A program whose one-wave diagrams fall in the register-tile class RMAX (the widest row sets the
    class of all of them): one row of width in that class's range, narrower knapsack rows, and
    2-variable rows (another tile class).  Returns (problem, width of the widest row)."""
    import synth
    lo = {4: 128, 8: 256, 12: 512, 16: 768, 24: 1024, 32: 1536, 64: 3072}[rmax]
    rng = np.random.default_rng(100 + rmax)
    n = 3000
    shape = (320, 60) if rmax > 32 else (200, 40) if rmax > 16 else (140, 24)
    wide, w = _row_of_width(rng, n, lo, rmax * 64, *shape)
    rows = [wide]
    k = synth.knapsack(n=n, m=6, kmin=20, kmax=60, amax=10, frac=0.3, seed=200 + rmax)
    rows += [k.row(j) for j in range(k.m)]
    s = synth.independent_set(n=n, M=50, seed=300 + rmax)
    rows += [s.row(j) for j in range(s.m)]
    return synth.generators._from_rows(n, -rng.uniform(0, 1, size=n), rows, f"class-{rmax}"), w


def coded_and_raw_problem(seed=31):
    """One-wave diagrams whose passes read some levels in byte codes (child-code steps of 0..15) and
    some in 4-byte codes: >= rows (their small partial sums lead to the 0-terminal first, so child
    codes are not monotone), <= rows with coefficients up to 400 (steps beyond a nibble), knapsack
    rows (every level coded), next to = rows and 2-variable rows of narrower classes."""
    import synth
    rng = np.random.default_rng(seed)
    n = 3000
    rows = []
    for _ in range(3):
        cols = rng.choice(n, 60, replace=False)
        a = rng.integers(1, 21, 60)
        rows.append((cols, a, 1, int(0.6 * a.sum())))
    for _ in range(3):
        cols = rng.choice(n, 40, replace=False)
        a = rng.integers(1, 9, 40)
        rows.append((cols, a, 0, int(0.5 * a.sum())))
    for _ in range(2):
        cols = rng.choice(n, 24, replace=False)
        a = rng.integers(1, 400, 24)
        rows.append((cols, a, -1, int(0.4 * a.sum())))
    k = synth.knapsack(n=n, m=4, kmin=40, kmax=80, amax=20, frac=0.4, seed=seed)
    rows += [k.row(j) for j in range(k.m)]
    s = synth.independent_set(n=n, M=40, seed=seed + 1)
    rows += [s.row(j) for j in range(s.m)]
    # normal costs (of both signs) from a stream of their own: the dual is still moving after a few
    # iterations, so the gradients with respect to omega are not rounding residue
    c = np.random.default_rng(seed + 68).normal(size=n)
    return synth.generators._from_rows(n, c, rows, "coded-and-raw")
