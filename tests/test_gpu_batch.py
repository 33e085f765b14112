"""GPU: graph-replayed iterations, resident-grid launches, packed batches and the autotuner.

None of these may change the arithmetic: graph replays issue the same launches as eager
calls, a launch shape only changes which wave takes which tile, and a batch is a disjoint
union whose programs share no variable.  So their states are compared bit for bit with the
plain single-instance path, and the bounds with the FP64 oracle.
"""
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


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.build(force=False)
    return oracle


def mixed():
    return synth.random_tiny(4, n=60, m=90, kmin=1, kmax=14, amin=-7, amax=7)


def learned(p, seed):
    rng = np.random.default_rng(seed)
    om = synth.sigmoid(rng.normal(size=p.nnz)).astype(np.float32)
    ah = rng.normal(0, 0.3, size=p.nnz).astype(np.float32)
    return om, ah


def state(inst):
    return tuple(host(t) for t in inst.get_state())


@pytest.mark.parametrize("case", ["setcover", "gm-small", "mixed", "knapsack-small"])
def test_graph_replays_equal_eager_launches(case):
    p = {"setcover": lambda: synth.workload("setcover")["problem"],
         "gm-small": lambda: synth.workload("gm", small=True)["problem"],
         "mixed": mixed,
         "knapsack-small": lambda: synth.knapsack(n=3000, m=30, seed=9)}[case]()
    om, ah = learned(p, 1)
    say(f"graphs vs eager {case} E={p.nnz}")
    a, _, _ = make_instance(p, om, ah)
    b, _, _ = make_instance(p, om, ah, graphs=False)
    for T in (11, 2, 8):  # both graphs (8 iterations and 1), several replays
        a.run(T)
        b.run(T)
        la, Ma = state(a)
        lb_, Mb = state(b)
        np.testing.assert_array_equal(la, lb_)
        np.testing.assert_array_equal(Ma, Mb)
        # eager work between replays
        assert a.lower_bound() == b.lower_bound()


def test_resident_grid_launch_shapes_are_bitwise_neutral():
    p = mixed()
    om, ah = learned(p, 2)
    ref, _, _ = make_instance(p, om, ah, graphs=False)
    alt, _, _ = make_instance(p, om, ah)
    shapes = alt.launch_shapes()
    say(f"classes {shapes}")
    assert len(shapes) >= 3
    for c, sh in enumerate(shapes):
        # few resident workgroups: every wave walks many tiles
        alt.set_launch(c, 1 if c % 2 else 2, 2 if c % 2 else 1, 1 + c % 3, 2 + c % 2)
    assert alt.launch_shapes()[0]["grid_f"] == 1
    ref.run(5)
    alt.run(5)
    for x, y in zip(state(ref), state(alt)):
        np.testing.assert_array_equal(x, y)
    assert ref.lower_bound() == alt.lower_bound()


def test_set_launch_rejects_bad_shapes():
    import paper_2205_11638_amd as dd
    inst, _, _ = make_instance(mixed())
    n = len(inst.launch_shapes())
    for args in ((n, 1, 1), (-1, 1, 1), (0, 0, 1), (0, 1, 8), (0, 8, 1), (0, 1, 17), (0, 1, 1, -1, 0)):
        with pytest.raises(dd.DDError):
            inst.set_launch(*args)


def batch_programs():
    ps = synth.workload("batch", small=True)["problems"][:6]
    return ps + [synth.knapsack(n=3000, m=30, seed=9), mixed()]


def test_batch_equals_separate_instances(orc):
    import torch

    import paper_2205_11638_amd as dd
    ps = batch_programs()
    params = [learned(p, 10 + q) for q, p in enumerate(ps)]
    say(f"batch of {len(ps)}: n={[p.n for p in ps]}")
    bt = dd.Batch(ps)
    inst = bt.instance
    assert inst.E == sum(p.nnz for p in ps) and inst.n == sum(p.n for p in ps)
    np.testing.assert_array_equal(np.diff(bt.edge_off), [p.nnz for p in ps])
    om = torch.tensor(np.concatenate([q[0] for q in params]), device="cuda")
    ah = torch.tensor(np.concatenate([q[1] for q in params]), device="cuda")
    inst.set_params(om, inst.seg_softmax(ah))
    inst.reset()
    T = 12
    bt.run(T)
    lbs, dls = bt.lower_bounds()
    lam, M = state(inst)
    for q, p in enumerate(ps):
        e0, e1 = bt.edge_off[q], bt.edge_off[q + 1]
        one, _, alt = make_instance(p, *params[q])
        one.run(T)
        l1, M1 = state(one)
        np.testing.assert_array_equal(lam[e0:e1], l1, err_msg=f"program {q}")
        np.testing.assert_array_equal(M[e0:e1], M1, err_msg=f"program {q}")
        lb1, dl1 = one.lower_bound()
        assert lbs[q] == pytest.approx(lb1, rel=1e-12, abs=1e-9)
        assert dls[q] == pytest.approx(dl1, rel=1e-12, abs=1e-9)
        assert dls[q] <= lbs[q] + 1e-6 * max(1.0, abs(lbs[q]))
        # and the FP64 oracle on the same parameters
        lo, Mo = orc.run(p, params[q][0].astype(np.float64), host(alt), T)
        lbo = orc.lower_bound(p, host(alt), lo, Mo)
        lbo = lbo[0] if isinstance(lbo, tuple) else lbo
        assert lbs[q] == pytest.approx(lbo, rel=1e-5, abs=1e-6), q


def test_autotune_cache_roundtrip(tmp_path):
    p = synth.workload("gm", small=True)["problem"]
    om, ah = learned(p, 3)
    cache = tmp_path / "shapes.txt"
    a, _, _ = make_instance(p, om, ah)
    a.run(2)
    before = state(a)
    assert a.autotune(str(cache)) is False
    # the solver state is restored
    for x, y in zip(before, state(a)):
        np.testing.assert_array_equal(x, y)
    tuned = a.launch_shapes()
    say(f"tuned {tuned}")
    assert cache.read_text().count("\n") == 1
    b, _, _ = make_instance(p, om, ah)
    assert b.autotune(str(cache)) is True
    assert b.launch_shapes() == tuned
    ref, _, _ = make_instance(p, om, ah, graphs=False)
    ref.run(2)
    for inst in (a, ref):
        inst.run(4)
    b.run(6)
    for x, y, z in zip(state(ref), state(a), state(b)):
        np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(x, z)


def test_batch_gradients_equal_separate_instances():
    """Reverse mode over a packed batch (the paper trains on mini-batches of instances): the
    gradient of the summed bound, sliced per program, is each program's own gradient."""
    import torch

    import paper_2205_11638_amd as dd
    ps = batch_programs()[2:7]
    params = [learned(p, 20 + q) for q, p in enumerate(ps)]
    bt = dd.Batch(ps)
    inst = bt.instance
    om = torch.tensor(np.concatenate([q[0] for q in params]), device="cuda")
    ah = torch.tensor(np.concatenate([q[1] for q in params]), device="cuda")
    inst.set_params(om, inst.seg_softmax(ah))
    T, K = 4, 2
    inst.forward_unrolled(T, K)
    lbs, _ = bt.lower_bounds()
    dw, da, dc = (host(t) for t in inst.backward(1.0))
    for q, p in enumerate(ps):
        e0, e1 = bt.edge_off[q], bt.edge_off[q + 1]
        v0, v1 = bt.var_off[q], bt.var_off[q + 1]
        one, _, _ = make_instance(p, *params[q])
        lb1 = one.forward_unrolled(T, K)
        assert lbs[q] == pytest.approx(lb1, rel=1e-12, abs=1e-9)
        g1 = [host(t) for t in one.backward(1.0)]
        np.testing.assert_array_equal(dw[e0:e1], g1[0], err_msg=f"program {q}")
        np.testing.assert_array_equal(da[e0:e1], g1[1], err_msg=f"program {q}")
        np.testing.assert_array_equal(dc[v0:v1], g1[2], err_msg=f"program {q}")


def test_alpha_s_formed_in_the_pass_gives_the_separate_launchs_bits():
    """The narrow update passes form alpha * S themselves while S fits in 4 MB (one XCD's L2); a
    larger instance forms it with a separate launch before each pass. Two independent-set programs
    of 540,000 variables each: alone, each forms it in its passes; packed (1,080,000 variables), the
    batch uses the separate launch. The states must agree bit for bit."""
    import torch

    import paper_2205_11638_amd as dd
    ps = [synth.independent_set(n=540_000, M=540_000, seed=31 + q) for q in range(2)]
    params = [learned(p, 40 + q) for q, p in enumerate(ps)]
    say(f"[alpha*S] packed n={sum(p.n for p in ps)}, edges={sum(p.nnz for p in ps)}")
    bt = dd.Batch(ps)
    inst = bt.instance
    om = torch.tensor(np.concatenate([q[0] for q in params]), device="cuda")
    ah = torch.tensor(np.concatenate([q[1] for q in params]), device="cuda")
    inst.set_params(om, inst.seg_softmax(ah))
    inst.reset()
    inst.profile_begin()
    inst.run_pass(0)
    assert "k_edge_alpha_s" in inst.profile_end()
    inst.run_pass(1)
    T = 5
    bt.run(T)
    lam, M = state(inst)
    for q, p in enumerate(ps):
        e0, e1 = bt.edge_off[q], bt.edge_off[q + 1]
        one, _, _ = make_instance(p, *params[q])
        one.profile_begin()
        one.run_pass(0)
        assert "k_edge_alpha_s" not in one.profile_end()
        one.run_pass(1)
        one.run(T)
        l1, M1 = state(one)
        np.testing.assert_array_equal(lam[e0:e1], l1, err_msg=f"program {q}")
        np.testing.assert_array_equal(M[e0:e1], M1, err_msg=f"program {q}")
