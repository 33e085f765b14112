"""GPU: the test-time driver (rounds of T iterations, the paper's relative-improvement stop) and
the relative dual gap g(t) / g_I of Sec. "Evaluation", against the FP64 oracle's trajectory and the
LP optimum (scipy HiGHS; the rows of set cover and independent set are integral polytopes, so the LP
optimum is the optimum d* of the dual)."""
import numpy as np
import pytest

import synth
from tests import brute
from tests.gpu_util import host, make_instance, say

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("wl,T,rounds", [("setcover", 20, 40), ("indset", 50, 12)])
def test_driver_trace_and_gap(orc, wl, T, rounds):
    import paper_2205_11638_amd as dd
    w = synth.workload(wl, small=(wl == "indset"))
    p = w["problem"]
    inst, _, alt = make_instance(p, np.asarray(w["omega"], np.float32), np.asarray(w["alpha_hat"], np.float32))
    lbs, ms = inst.solve(T, rounds, 1e-6)
    k = len(lbs) - 1
    say(f"  {wl}: {k} rounds, bound {lbs[0]:.4f} -> {lbs[-1]:.4f} in {ms[-1]:.1f} ms")
    assert 1 <= k <= rounds and np.all(np.diff(ms) >= 0)
    # stopping rule, decided on the GPU's own trace
    rel = np.diff(lbs) / np.maximum(np.abs(lbs[:-1]), 1e-300)
    assert np.all(rel[:-1] >= 1e-6)
    assert k == rounds or rel[-1] < 1e-6
    # the trace is the oracle's trajectory
    al = host(alt)
    om = np.asarray(w["omega"], np.float32).astype(np.float64)
    lam, M = orc.init_lambda(p), np.zeros(p.nnz)
    for r in range(k + 1):
        if r:
            lam, M = orc.run(p, om, al, T, lam=lam, M=M)
        lb_o = orc.lower_bound(p, al, lam, M)[0]
        assert lbs[r] == pytest.approx(lb_o, rel=1e-5, abs=1e-6), r
    # relative dual gap against d* = LP optimum
    d_star = brute.lp_optimum(p)
    assert lbs[-1] <= d_star + 1e-5 * abs(d_star)
    g, gi = dd.gap_integral(lbs, ms, d_star)
    assert g[0] == 1.0 and np.all((g >= 0) & (g <= 1)) and g[-1] < g[0]
    assert 0 < gi <= ms[-1] / 1000.0
    say(f"  {wl}: d* {d_star:.4f}, final g {g[-1]:.3g}, g_I {gi:.3g} s")
