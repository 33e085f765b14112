"""The deferred sums S_i = sum over the subproblems k of M_ik (the coupling term of the multiplier
update, Alg. 1) are formed in one fixed order, so a program gets the same bits alone and packed into a
batch. A team of lanes per variable takes the variable's edges (rows ascending) in strided order.
Each lane loads up to four terms ahead, then adds them in list order, and a fixed butterfly (partner
lane half the team away first, lane 1 last) adds the partial sums. The flushed multipliers
lambda + alpha * S, read back through the C ABI, must equal a float32 host model of that order bit
for bit, for variables in 1 to 45 rows (every tail of the strided loads)."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.gpu_util import make_instance, say

pytestmark = pytest.mark.gpu

TEAM = 4  # lanes per variable in the library's per-variable sums


def degree_problem():
    """Covering rows sum x >= 1 in which variable i sits in 1 + (i mod 45) rows."""
    rng, n, m = np.random.default_rng(5), 270, 60
    members = [[] for _ in range(m)]
    for i in range(n):
        for j in rng.choice(m, size=1 + i % 45, replace=False):
            members[j].append(i)
    rows = [(np.array(mem), np.ones(len(mem), np.int64), 1, 1) for mem in members if mem]
    return synth.generators._from_rows(n, rng.uniform(-1, 1, size=n), rows, "degrees")


def team_sum(vals):
    """float32 model of one variable's sum: strided lane sums from 0, then the butterfly (partner
    lane TEAM/2 first, lane 1 last)."""
    part = []
    for u in range(TEAM):
        s = np.float32(0.0)
        for v in vals[u::TEAM]:
            s = np.float32(s + v)
        part.append(s)
    w = TEAM // 2
    while w:
        part = [np.float32(part[u] + part[u ^ w]) for u in range(TEAM)]
        w //= 2
    return part[0]


def test_flushed_multipliers_follow_the_fixed_sum_order():
    import torch

    prob = degree_problem()
    say(f"[deferred] {prob.name}: n={prob.n} m={prob.m} edges={int(prob.row_ptr[-1])}")
    inst, _, _ = make_instance(prob)
    var, _ = inst.edge_map()
    E = inst.E
    deg = np.bincount(var, minlength=prob.n)
    assert deg.min() == 1 and deg.max() == 45
    rng = np.random.default_rng(7)
    lam = rng.standard_normal(E).astype(np.float32)
    # magnitudes over six decades, so a different order of the adds changes the rounded sums
    M = (rng.standard_normal(E) * 10.0 ** rng.integers(-3, 3, size=E)).astype(np.float32)
    alpha = rng.uniform(0.05, 1.0, size=E).astype(np.float32)
    omega = np.full(E, 0.5, np.float32)
    dev = lambda a: torch.tensor(a, device="cuda")
    inst.set_params(dev(omega), dev(alpha))
    inst.set_state(dev(lam), dev(M))
    lam_bar, M_back = inst.get_state(flushed=True)
    torch.cuda.synchronize()
    S = np.zeros(prob.n, np.float32)
    for i in range(prob.n):
        S[i] = team_sum(M[np.nonzero(var == i)[0]])  # canonical order within a variable: rows ascending
    want = lam + (alpha * S[var]).astype(np.float32)
    assert want.dtype == np.float32
    np.testing.assert_array_equal(M_back.cpu().numpy(), M)
    got = lam_bar.cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (f"{bad.size} of {E} flushed multipliers differ; first at edge {bad[0]} "
                           f"(variable {var[bad[0]]} in {deg[var[bad[0]]]} rows): {got[bad[0]]!r} vs {want[bad[0]]!r}")
    # the model is sensitive to the order: a plain left-to-right sum differs somewhere
    plain = np.array([np.float32(sum(np.float32(x) for x in M[np.nonzero(var == i)[0]])) if deg[i] else 0
                      for i in range(prob.n)], np.float32)
    assert (plain != S).any()
