"""GPU: boundary behaviour of the C ABI -- the device-memory cap (DD_E_OOM), checkpoint
verification (DD_E_CHECKPOINT, forced from the host through the test hook), the device-side bound
trace, and sizes."""
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


def _gm():
    w = synth.workload("gm", small=True)
    return w["problem"], w["omega"], w["alpha_hat"]


def test_device_memory_cap():
    """An allocation that would pass max_device_bytes fails with DD_E_OOM: at create when the cap is
    below what the instance needs, and later when reverse mode first needs its buffers; the instance
    stays usable after such a refusal."""
    import paper_2205_11638_amd as dd
    p, om, ah = _gm()
    need = make_instance(p)[0].stats["device_bytes"]
    with pytest.raises(dd.DDError) as e:
        make_instance(p, max_device_bytes=need - 1)
    assert e.value.code == dd.binding.DD_E_OOM and "cap" in str(e.value)
    inst, _, _ = make_instance(p, om, ah, max_device_bytes=need)
    assert inst.stats["device_bytes"] == need
    with pytest.raises(dd.DDError) as e:
        inst.forward_unrolled(3, 1)
    assert e.value.code == dd.binding.DD_E_OOM
    inst.run(2)  # still usable
    lb = inst.lower_bound()[0]
    ref, _, _ = make_instance(p, om, ah)
    ref.run(2)
    assert lb == ref.lower_bound()[0]
    # a cap with room for reverse mode but not for a stored trajectory
    big, _, _ = make_instance(p, om, ah, max_device_bytes=need * 4)
    big.forward_unrolled(3, 1)
    big.backward(1.0)
    with pytest.raises(dd.DDError) as e:
        big.forward_unrolled(200, -1)
    assert e.value.code == dd.binding.DD_E_OOM


@pytest.mark.parametrize("replay", [False, True])
def test_checkpoint_verification(replay):
    """The backward sweep checks every checkpoint it reads against the fingerprint taken when it was
    saved, and the state each recomputed segment ends in against the next checkpoint's: a checkpoint
    changed after the forward (the test hook adds 1 to one slot) fails with DD_E_CHECKPOINT; an intact
    record passes and gives the gradients of a fresh instance."""
    import paper_2205_11638_amd as dd
    p, om, ah = _gm()
    inst, _, _ = make_instance(p, om, ah, adj_replay=replay)
    ref, _, _ = make_instance(p, om, ah, adj_replay=replay)
    ref.forward_unrolled(6, 2)
    g_ref = [host(t) for t in ref.backward(1.0)]
    for index in (0, 1, 3):  # the start state, an inner checkpoint, the final state
        inst.forward_unrolled(6, 2)
        inst.corrupt_checkpoint(index)
        with pytest.raises(dd.DDError) as e:
            inst.backward(1.0)
        assert e.value.code == dd.binding.DD_E_CHECKPOINT, index
    # the last segment's start: without replays the forward keeps that segment's records, so the
    # first backward sweep does not read the checkpoint and the second one (which recomputes it) does
    inst.forward_unrolled(6, 2)
    inst.corrupt_checkpoint(2)
    if not replay:
        g = [host(t) for t in inst.backward(1.0)]
        for a, b in zip(g, g_ref):
            np.testing.assert_array_equal(a, b)
    with pytest.raises(dd.DDError) as e:
        inst.backward(1.0)
    assert e.value.code == dd.binding.DD_E_CHECKPOINT
    inst.forward_unrolled(6, 2)
    g = [host(t) for t in inst.backward(1.0)]
    for a, b in zip(g, g_ref):
        np.testing.assert_array_equal(a, b)
    with pytest.raises(dd.DDError) as e:
        inst.corrupt_checkpoint(4)
    assert e.value.code == dd.binding.DD_E_ARG
    inst.forward_unrolled(2, -1)  # a stored trajectory has no checkpoints
    with pytest.raises(dd.DDError) as e:
        inst.corrupt_checkpoint(0)
    assert e.value.code == dd.binding.DD_E_STATE


def test_run_trace_equals_bounds_between_runs():
    p, om, ah = _gm()
    a, _, _ = make_instance(p, om, ah, lb_every=3)
    b, _, _ = make_instance(p, om, ah)
    tr = host(a.run_trace(20))  # 6 bounds; the last 2 iterations run without one
    assert tr.shape == (6,)
    ref = []
    for _ in range(6):
        b.run(3)
        ref.append(b.lower_bound()[0])
    np.testing.assert_array_equal(tr, np.array(ref))
    b.run(2)
    assert a.lower_bound()[0] == b.lower_bound()[0]
    tr7 = host(a.run_trace(7, lb_every=7))
    b.run(7)
    assert tr7[0] == b.lower_bound()[0]
    say("trace", tr)


def test_set_costs_equals_a_fresh_instance():
    """Replacing the costs (device array in the caller's variable order; the library keeps its own
    order) gives the state and cost gradient of an instance created with those costs bit for bit, and
    its bound -- uncovered variables included (the independent-set workload leaves some in no row)."""
    import torch
    for name in ("gm", "indset"):
        w = synth.workload(name, small=True) if name == "gm" else {"problem": synth.independent_set(n=3000, M=4000, seed=5)}
        p = w["problem"]
        rng = np.random.default_rng(3)
        c2 = rng.normal(size=p.n)
        p2 = synth.Problem(p.n, c2, p.row_ptr, p.col, p.coef, p.sense, p.rhs)
        a, _, _ = make_instance(p)
        b, _, _ = make_instance(p2)
        a.set_costs(torch.tensor(c2, dtype=torch.float32, device="cuda"))
        a.run(3)
        b.run(3)
        for x, y in zip(a.get_state(), b.get_state()):
            np.testing.assert_array_equal(host(x), host(y))
        # the constant of the uncovered variables: a device sum of the f32 costs against a host sum of
        # the f64 ones at create
        assert a.lower_bound()[0] == pytest.approx(b.lower_bound()[0], rel=1e-9, abs=1e-9)
        a.forward_unrolled(2, 1)
        b.forward_unrolled(2, 1)
        ga, gb = a.backward(1.0)[2], b.backward(1.0)[2]
        np.testing.assert_array_equal(host(ga), host(gb))
        say(f"set_costs {name}: n={p.n}, uncovered {a.stats['uncovered']}")


def test_sizes():
    p, _, _ = _gm()
    inst, _, _ = make_instance(p)
    assert inst.num_edges() == p.nnz == inst.E


@pytest.mark.parametrize("case,T,K,replay", [("gm", 6, 2, False), ("gm", 5, 2, True), ("gm", 4, -1, False),
                                             ("knapsack", 3, 2, False), ("knapsack", 3, -1, False)])
def test_captured_sequences_equal_eager_launches(case, T, K, replay):
    """The unrolled forward and the backward sweep run as launch sequences captured into graphs the
    first time (T, K, mode) is seen and replayed afterwards; an instance created without graphs
    launches every kernel itself.  Replays take the seed of the moment (it is read from device
    memory), so over several rounds with different seeds, with eager work in between, bound,
    gradients and the state left behind agree bit for bit; a checkpoint changed before a replayed
    backward is still caught."""
    import paper_2205_11638_amd as dd
    if case == "gm":
        p, om, ah = _gm()
    else:
        w = synth.workload("knapsack", small=True)
        p, om, ah = w["problem"], w["omega"], w["alpha_hat"]
    say(f"captured vs eager {case} T={T} K={K} replay={replay}")
    g, _, _ = make_instance(p, om, ah, adj_replay=replay)
    e, _, _ = make_instance(p, om, ah, adj_replay=replay, graphs=False)
    for rnd, seed in enumerate((1.0, -2.5, 0.75)):
        lbg, lbe = g.forward_unrolled(T, K), e.forward_unrolled(T, K)
        assert lbg == lbe, rnd
        gg = [host(t) for t in g.backward(seed)]
        ge = [host(t) for t in e.backward(seed)]
        for a, b, name in zip(gg, ge, ("d_omega", "d_alpha", "d_c")):
            assert np.isfinite(a).all()
            np.testing.assert_array_equal(a, b, err_msg=f"{name} round {rnd}")
        for a, b in zip(g.get_state(), e.get_state()):
            np.testing.assert_array_equal(host(a), host(b))
        g.run(1)  # eager work between the replays
        e.run(1)
        assert g.lower_bound()[0] == e.lower_bound()[0]
    if K > 0:
        # the first segment's start (the last segment's start is read only when that segment is
        # recomputed, which the forward's kept records make unnecessary the first time)
        g.forward_unrolled(T, K)
        g.corrupt_checkpoint(0)
        with pytest.raises(dd.DDError) as err:
            g.backward(1.0)
        assert err.value.code == dd.binding.DD_E_CHECKPOINT


@pytest.mark.parametrize("K,dense", [(5, False), (-1, False), (2, True)])
def test_captured_sequences_from_a_state(K, dense):
    """The same equality for rounds that start from a given state (the training round's form: the
    start state is set, the unrolled forward runs from it, the backward returns the start state's
    adjoints too), alternating with eager calls that move the state; and with the reverse sweeps of
    one-wave diagrams routed node by node (adj_route_dense)."""
    import torch
    if dense:
        w = synth.workload("knapsack", small=True)
        p, om, ah = w["problem"], w["omega"], w["alpha_hat"]
    else:
        p, om, ah = _gm()
    say(f"captured vs eager from a state K={K} dense={dense}")
    g, _, _ = make_instance(p, om, ah, adj_route_dense=dense)
    e, _, _ = make_instance(p, om, ah, adj_route_dense=dense, graphs=False)
    g.run(3)
    lam, M = g.get_state()
    for rnd, (T, seed) in enumerate(((6, 1.0), (6, -0.5), (4, 2.0), (6, 1.0))):
        for inst in (g, e):
            inst.set_state(lam, M)
        lbg, lbe = g.forward_unrolled_from_state(T, K), e.forward_unrolled_from_state(T, K)
        assert lbg == lbe, rnd
        og = [host(t) for t in g.backward_state(seed)]
        oe = [host(t) for t in e.backward_state(seed)]
        for a, b, name in zip(og, oe, ("d_omega", "d_alpha", "d_lam0", "d_M0")):
            assert np.isfinite(a).all()
            np.testing.assert_array_equal(a, b, err_msg=f"{name} round {rnd}")
        g.run(2)
        e.run(2)
        lam, M = (t.clone() for t in g.get_state())
        for a, b in zip(g.get_state(), e.get_state()):
            np.testing.assert_array_equal(host(a), host(b))
        torch.cuda.synchronize()
