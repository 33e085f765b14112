"""GPU: dd_smoothed_noalloc (the entry point that allocates nothing, for callers that cannot
allocate) through the C ABI against dd_smoothed on the same instances: two calls in a row, the
second on a smaller instance, so the static scratch holds the first call's leftovers when the
second one runs.  Same kernels on the same inputs: the outputs must be equal bit for bit."""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, make_instance, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _params(p, seed):
    rng = np.random.default_rng(seed)
    return synth.sigmoid(rng.normal(size=p.nnz)), rng.normal(0, 0.3, size=p.nnz)


def _both(inst, tau, flushed):
    import torch
    E_ref, p_ref = (host(t) for t in inst.smoothed(tau, flushed=flushed))
    E_out = torch.full((inst.m,), float("nan"), device="cuda")
    p_out = torch.full((inst.E,), float("nan"), device="cuda")
    inst.smoothed_noalloc(tau, E_out, p_out, flushed=flushed)
    return (host(E_out), host(p_out)), (E_ref, p_ref)


def test_noalloc_matches_smoothed_twice_in_a_row():
    big = synth.workload("gm", small=True)["problem"]
    small = synth.set_cover(n=300, m=120, seed=5)
    out = []
    for p, seed, tau, flushed in ((big, 1, 10.0, False), (small, 2, 1.0, True)):
        inst, _, _ = make_instance(p, *_params(p, seed))
        inst.run(3)
        assert inst.stats["node_slots"] + 64 <= 1 << 22
        say(f"noalloc smoothed: {p.name} node slots {inst.stats['node_slots']} tau {tau} flushed {flushed}")
        (E, pm), (E_ref, p_ref) = _both(inst, tau, flushed)
        np.testing.assert_array_equal(E, E_ref)
        np.testing.assert_array_equal(pm, p_ref)
        assert np.isfinite(E).all() and np.isfinite(pm).all()
        out.append(inst.stats["node_slots"])
    assert out[1] < out[0]


def test_noalloc_rejects_an_instance_beyond_its_scratch():
    import torch

    import paper_2205_11638_amd as dd
    p = synth.knapsack(n=20000, m=400, seed=1004)
    inst, _, _ = make_instance(p)
    assert inst.stats["node_slots"] + 64 > 1 << 22
    with pytest.raises(dd.DDError) as e:
        inst.smoothed_noalloc(1.0, torch.empty(inst.m, device="cuda"), torch.empty(inst.E, device="cuda"))
    assert e.value.code == dd.binding.DD_E_ARG and "node scratch" in str(e.value)
