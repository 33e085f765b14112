"""GPU: solver features of the appendix's feature table -- smoothed subproblems (soft-min energies
E_tau and their gradients, the Gibbs marginals) and the minimizing assignment -- against the FP64
oracle.

Tolerances (fp32 derivation): a soft-min path cost carries rounding of order 2^-24 times the row's
cost scale s_j per operation, and E_tau itself grows like tau log |X_j|, so energies are compared
to 1e-4 of max(|E|, s_j, tau); marginals are probabilities formed from exp(-(cost difference)/tau)
and are compared to 1e-4 absolute.  The minimizing assignment is an integer decision: bit-exact on
rows whose decisions are unique -- every decision's two options further apart than the rounding of
the fp32 path costs compared, 2 (L_j + 2) 2^-24 s_j (flip_tol) -- and on the others a feasible
assignment whose cost is the row minimum to fp32 precision.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, make_instance, row_scale, say
from tests.test_gpu_adjoint import CASES, f32, flip_tol

pytestmark = pytest.mark.gpu
TAUS = (1.0, 10.0, 100.0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.build(force=False)
    return oracle


def check_smoothed(orc, p, lam, E, pm, tau, what):
    Eo, po = orc.smoothed(p, lam, tau)
    sj = np.add.reduceat(np.abs(lam), p.row_ptr[:-1]) if p.nnz else np.zeros(p.m)
    sj = np.where(np.diff(p.row_ptr) > 0, sj, 0.0)
    tolE = 1e-4 * np.maximum(np.maximum(np.abs(Eo), sj), tau)
    bad = np.abs(E - Eo) > tolE
    assert not bad.any(), (what, tau, int(bad.sum()), float(np.max(np.abs(E - Eo) / tolE)))
    assert np.abs(pm - po).max() <= 1e-4, (what, tau, float(np.abs(pm - po).max()))


def check_argmin(orc, p, lam, x, what):
    xo, _, gap = orc.argmin(p, lam, row_gaps=True)
    tie = gap <= flip_tol(p, [(lam, lam)])  # the GPU's multipliers are the oracle's input
    rowid = np.repeat(np.arange(p.m), np.diff(p.row_ptr))
    uniq = ~tie[rowid]
    say(f"  {what}: rows with a near-tie {int(tie.sum())}/{p.m}")
    np.testing.assert_array_equal(x[uniq], xo[uniq], err_msg=what)
    assert set(np.unique(x)) <= {0.0, 1.0}
    # rows with near-ties: a feasible minimizer
    Ej = orc.energies(p, lam)
    for j in np.flatnonzero(tie):
        a, b = int(p.row_ptr[j]), int(p.row_ptr[j + 1])
        s = int(np.asarray(p.coef[a:b], np.int64) @ x[a:b].astype(np.int64))
        sense, rhs = int(p.sense[j]), int(p.rhs[j])
        assert (s <= rhs) if sense < 0 else (s >= rhs) if sense > 0 else (s == rhs), (what, j)
        assert x[a:b] @ lam[a:b] == pytest.approx(Ej[j], rel=1e-5, abs=1e-5 * np.abs(lam[a:b]).sum())


@pytest.mark.parametrize("case", ["setcover", "gm-small", "knapsack-small", "team-sizes", "mixed0"])
@pytest.mark.parametrize("flushed", [False, True])
def test_smoothed_and_argmin_match_oracle(orc, case, flushed):
    p = CASES[case]()
    rng = np.random.default_rng(1)
    inst, _, _ = make_instance(p, f32(synth.sigmoid(rng.normal(size=p.nnz))), f32(rng.normal(0, 0.3, size=p.nnz)))
    inst.run(3)
    lam = host(inst.get_state(flushed=flushed)[0])
    for tau in TAUS:
        E, pm = (host(x) for x in inst.smoothed(tau, flushed=flushed))
        check_smoothed(orc, p, lam, E, pm, tau, case)
    check_argmin(orc, p, lam, host(inst.argmin_assignment(flushed=flushed)), case)
    # features leave the solver state alone
    lam2 = host(inst.get_state(flushed=flushed)[0])
    np.testing.assert_array_equal(lam2, lam)
    assert inst.lower_bound()[0] == pytest.approx(inst.lower_bound()[0])


def test_small_temperature_from_a_random_state(orc):
    """Small tau on a state with well-separated minimizers (random multipliers): the marginals match
    the oracle and concentrate on the minimizing assignment.  (After a few iterations of averaging
    many min-marginal differences are ~0, so there the marginals legitimately stay near 1/2.)"""
    import torch
    p = CASES["gm-small"]()
    inst, _, _ = make_instance(p)
    lam = f32(np.random.default_rng(9).normal(size=p.nnz))
    inst.set_state(torch.tensor(lam, dtype=torch.float32, device="cuda"),
                   torch.zeros(p.nnz, dtype=torch.float32, device="cuda"))
    tau = 0.01
    E, pm = (host(x) for x in inst.smoothed(tau))
    check_smoothed(orc, p, lam, E, pm, tau, "random state")
    x = host(inst.argmin_assignment())
    check_argmin(orc, p, lam, x, "random state")
    _, po = orc.smoothed(p, lam, tau)
    sure = (po < 1e-3) | (po > 1 - 1e-3)
    assert sure.mean() > 0.9
    np.testing.assert_array_equal(np.round(pm[sure]), x[sure])
    with pytest.raises(Exception):
        inst.smoothed(0.0)


def test_knapsack_full_sampled_rows_features(orc):
    """The full 2M-variable knapsack program: features of 200 seeded rows against the oracle."""
    w = synth.workload("knapsack")
    p = w["problem"]
    say("knapsack full features: compiling")
    inst, _, _ = make_instance(p, f32(w["omega"]), f32(w["alpha_hat"]))
    inst.run(2)
    rows = np.sort(np.random.default_rng(4005).choice(p.m, size=200, replace=False))
    sub = p.subset_rows(rows)
    eidx = np.concatenate([np.arange(p.row_ptr[r], p.row_ptr[r + 1]) for r in rows])
    lbar = host(inst.get_state(flushed=True)[0])
    E, pm = (host(x) for x in inst.smoothed(10.0, flushed=True))
    check_smoothed(orc, sub, lbar[eidx], E[rows], pm[eidx], 10.0, "knapsack")
    check_argmin(orc, sub, lbar[eidx], host(inst.argmin_assignment(flushed=True))[eidx], "knapsack")
