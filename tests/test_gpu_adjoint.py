"""GPU reverse mode (Alg. 2 through unrolled passes) against the FP64 oracle's literal Alg. 2.

The oracle traces the minimizers s^j(i, beta) of every block explicitly on the partial-sum
diagram; the GPU routes adjoints through argmins of its BDD sweeps.  Where a minimizer is
unique the two must agree: gradients to 1e-4 relative, norm-wise per parameter vector and
entry-wise with a floor of 1e-4 * max |reference|.  Where two options of a decision are within
GAP_MIN (relative) of each other, fp32 and fp64 may legitimately take different sides, and
both results are valid subgradients.  There the tests compare what is unique (the rows, and
the variables, that no near-tie touches) and check the rest through Euler's identity for
positively homogeneous maps, which every linear piece meeting at the point satisfies.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, make_instance, say, wide_class_problem

pytestmark = pytest.mark.gpu
GRAD_RTOL = 1e-4
GAP_MIN = 1e-5


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


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def close_grad(got, ref, what):
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    nr = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= GRAD_RTOL * max(nr, 1e-6), (what, np.linalg.norm(got - ref), nr)
    floor = GRAD_RTOL * max(np.abs(ref).max(), 1e-6)
    bad = np.abs(got - ref) > np.maximum(GRAD_RTOL * np.abs(ref), floor)
    assert not bad.any(), (what, int(bad.sum()), int(np.argmax(np.abs(got - ref))))


def euler_close(lhs, rhs, scale, what):
    assert abs(lhs - rhs) <= GRAD_RTOL * max(scale, 1e-6), (what, lhs, rhs, scale)


def mixed_problem(seed):
    return synth.random_tiny(seed, n=40, m=60, kmin=1, kmax=14, amin=-7, amax=7)


def team_size_problem():
    rows, rng, n = [], np.random.default_rng(12), 4000
    for width_target in (2, 6, 12, 24, 48, 100, 200, 400, 900):
        for _ in range(3):
            k = int(rng.integers(8, 60))
            cols = rng.choice(n, size=k, replace=False)
            a = rng.integers(1, 4 * max(1, width_target // k) + 2, size=k)
            rows.append((cols, a, -1, int(max(a.max(), min(width_target, a.sum() // 2)))))
    return synth.generators._from_rows(n, -rng.uniform(0, 1, size=n), rows, "team-sizes")


def unit_rows_problem():
    """Rows sum x <= b with unit coefficients: their diagrams' level widths step through every value
    up to about b, so levels of exactly 255, 256, 257, 511, 512 and 513 nodes occur (the boundaries
    of the one-wave kernels' 256-node groups, where a level's terminal slots fall just past its
    groups), next to 2-variable rows."""
    rng, n = np.random.default_rng(21), 3000
    rows = [(rng.choice(n, size=k, replace=False), np.ones(k, np.int64), -1, b) for k, b in ((600, 300), (1100, 520))]
    for _ in range(60):
        rows.append((rng.choice(n, size=2, replace=False), np.ones(2, np.int64), -1, 1))
    return synth.generators._from_rows(n, -rng.uniform(0, 1, size=n), rows, "unit-rows")


CASES = {
    "mixed0": lambda: mixed_problem(0),
    "mixed3": lambda: mixed_problem(3),
    "setcover": lambda: synth.workload("setcover")["problem"],
    "gm-small": lambda: synth.workload("gm", small=True)["problem"],
    "team-sizes": team_size_problem,
    "knapsack-small": lambda: synth.knapsack(n=3000, m=30, seed=9),
    "gm-full": lambda: synth.workload("gm")["problem"],
    "wide-24": lambda: wide_class_problem(24)[0],
    "wide-32": lambda: wide_class_problem(32)[0],
    "unit-rows": unit_rows_problem,
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("direction", [0, 1])
def test_pass_vjp_matches_oracle(orc, case, direction):
    import torch
    p = CASES[case]()
    rng = np.random.default_rng(len(case) + direction)
    om = f32(synth.sigmoid(rng.normal(size=p.nnz)))
    ah = f32(rng.normal(0, 0.3, size=p.nnz))
    say(f"pass vjp {case} dir {direction} E={p.nnz}")
    inst, omt, alt = make_instance(p, om, ah)
    al = host(alt)
    inst.run(2)
    if direction == 1:
        inst.run_pass(0)
    lam_in, M_in = inst.get_state()
    dlo = rng.normal(size=p.nnz)
    dmo = rng.normal(size=p.nnz)
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    dli, dmi, da, dw = (host(t) for t in inst.pass_vjp(direction, lam_in, M_in, dev(dlo), dev(dmo)))
    # the state is left at the pass output
    lam_o, M_o = (host(t) for t in inst.get_state())
    li, mi = host(lam_in), host(M_in)
    *r, gap = orc.pass_vjp(p, om, al, direction, li, mi, f32(dlo), f32(dmo), with_gap=True)
    rowid = np.repeat(np.arange(p.m), np.diff(p.row_ptr))
    tie_row = gap < GAP_MIN
    ok_e = ~tie_row[rowid]
    tie_var = np.zeros(p.n, bool)
    tie_var[p.col[~ok_e]] = True
    ok_v = ~tie_var[p.col]  # dM_in gathers over every edge of the variable
    say(f"  near-tie rows {int(tie_row.sum())}/{p.m}; edges compared {int(ok_e.sum())}/{p.nnz}")
    assert ok_e.sum() >= min(p.nnz, 100)
    close_grad(dli[ok_e], r[0][ok_e], "dlam_in")
    close_grad(dmi[ok_v], r[1][ok_v], "dM_in")
    close_grad(da[ok_e], r[2][ok_e], "d_alpha")
    close_grad(dw[ok_e], r[3][ok_e], "d_omega")
    for a in (dli, dmi, da, dw):
        assert np.isfinite(a).all()
    lo, Mo = li.copy(), mi.copy()
    orc.run_pass(p, om, al, lo, Mo, direction)
    np.testing.assert_allclose(lam_o, lo, atol=1e-4 * np.abs(lo).max())
    # Euler's identity over all rows, then for each near-tie row on its own (seed on that row only)
    terms = np.concatenate([dli * li, dmi * mi])
    euler_close(terms.sum(), f32(dlo) @ lam_o + f32(dmo) @ M_o, np.abs(terms).sum(), "all rows")
    for j in np.flatnonzero(tie_row)[:6]:
        on = (rowid == j).astype(np.float64)
        dl, dm, _, _ = (host(t) for t in inst.pass_vjp(direction, lam_in, M_in, dev(dlo * on), dev(dmo * on)))
        terms = np.concatenate([dl * li, dm * mi])
        euler_close(terms.sum(), f32(dlo * on) @ lam_o + f32(dmo * on) @ M_o, np.abs(terms).sum(), f"row {j}")


# seeds picked so that the first three trajectories take no near-tie decision (the oracle
# reports it); the wide diagrams of the last two always do, and are checked through Euler
@pytest.mark.parametrize("case,T,K,seed", [("mixed0", 3, 2, 23), ("setcover", 4, 3, 3), ("gm-small", 5, 2, 1),
                                           ("team-sizes", 3, 1, 0), ("knapsack-small", 3, 5, 0)])
def test_unrolled_gradient_matches_oracle(orc, case, T, K, seed):
    p = CASES[case]()
    rng = np.random.default_rng(seed)
    om = f32(synth.sigmoid(rng.normal(size=p.nnz)))
    ah = f32(rng.normal(0, 0.3, size=p.nnz))
    say(f"unrolled grad {case} T={T} K={K}")
    inst, omt, alt = make_instance(p, om, ah)
    al = host(alt)
    lb = inst.forward_unrolled(T, K)
    dw, da, dc = (host(t) for t in inst.backward(1.0))
    pc = synth.Problem(p.n, f32(p.c), p.row_ptr, p.col, p.coef, p.sense, p.rhs)
    lb_o, dw_o, da_o, dc_o, gap = orc.unrolled_grad(pc, om, al, T, with_gap=True)
    assert lb == pytest.approx(lb_o, rel=1e-5, abs=1e-6)
    euler_close(dc @ pc.c, lb, np.abs(dc * pc.c).sum(), "<d_c, c> = LB")
    for a in (dw, da, dc):
        assert np.isfinite(a).all()
    say(f"  smallest decision gap on the trajectory {gap:.3g}")
    if gap >= GAP_MIN:  # every decision unique: the gradient is unique
        close_grad(dw, dw_o, "d_omega")
        close_grad(da, da_o, "d_alpha")
        close_grad(dc, dc_o, "d_c")
    # the state is the final one again: the bound is unchanged
    assert inst.lower_bound()[0] == pytest.approx(lb, rel=1e-6, abs=1e-7)


@pytest.mark.parametrize("case,T", [("gm-small", 5), ("knapsack-small", 3), ("wide-32", 2)])
def test_stored_trajectory_matches_checkpoints(case, T):
    """ckpt_every = -1 keeps every pass's node costs and state: the backward sweep then replays nothing,
    and since a recomputed pass reproduces its stored arrays bit for bit, bound and gradients are
    those of checkpoints every iteration, bit for bit; the solver is left at the same final state."""
    p = CASES[case]()
    rng = np.random.default_rng(7)
    om = f32(synth.sigmoid(rng.normal(size=p.nnz)))
    ah = f32(rng.normal(0, 0.3, size=p.nnz))
    say(f"stored trajectory {case} T={T}")
    inst, _, _ = make_instance(p, om, ah)
    lb1 = inst.forward_unrolled(T, 1)
    g1 = [host(t) for t in inst.backward(1.0)]
    s1 = [host(t) for t in inst.get_state()]
    lbs = inst.forward_unrolled(T, -1)
    gs = [host(t) for t in inst.backward(1.0)]
    ss = [host(t) for t in inst.get_state()]
    assert lbs == lb1
    for a, b, name in zip(g1, gs, ("d_omega", "d_alpha", "d_c")):
        np.testing.assert_array_equal(a, b, err_msg=name)
    for a, b in zip(s1, ss):
        np.testing.assert_array_equal(a, b)
    # B left for the next forward pass: one more iteration from here agrees too
    inst.run(1)
    lb_next = inst.lower_bound()[0]
    inst.forward_unrolled(T, 1)
    inst.backward(1.0)
    inst.run(1)
    assert inst.lower_bound()[0] == lb_next


@pytest.mark.parametrize("case,T,K", [("gm-small", 5, 2), ("knapsack-small", 3, 2), ("wide-32", 3, 2),
                                      ("mixed0", 5, 3), ("unit-rows", 3, 2)])
def test_segment_storage_matches_replay(case, T, K):
    """The checkpointed backward sweep keeps each recomputed segment's node costs, states and argmin
    records on the device and reverses it like a stored trajectory; with the adj_replay option it
    replays every pass instead.  Both take every value from the same kernels on the same inputs, so
    bound, gradients and the final state agree bit for bit (T not a multiple of K: a short last
    segment)."""
    p = CASES[case]()
    rng = np.random.default_rng(17)
    om = f32(synth.sigmoid(rng.normal(size=p.nnz)))
    ah = f32(rng.normal(0, 0.3, size=p.nnz))
    say(f"segment storage vs replay {case} T={T} K={K}")
    a, _, _ = make_instance(p, om, ah)
    b, _, _ = make_instance(p, om, ah, adj_replay=True)
    lba, lbb = a.forward_unrolled(T, K), b.forward_unrolled(T, K)
    assert lba == lbb
    ga = [host(t) for t in a.backward(1.0)]
    gb = [host(t) for t in b.backward(1.0)]
    for x, y, name in zip(ga, gb, ("d_omega", "d_alpha", "d_c")):
        assert np.isfinite(x).all()
        np.testing.assert_array_equal(x, y, err_msg=name)
    for x, y in zip(a.get_state(), b.get_state()):
        np.testing.assert_array_equal(host(x), host(y))
    assert a.lower_bound()[0] == b.lower_bound()[0] == pytest.approx(lba, rel=1e-6, abs=1e-7)


def test_stored_trajectory_too_large_is_rejected():
    p = CASES["setcover"]()
    inst, _, _ = make_instance(p, f32(np.full(p.nnz, 0.5)), f32(np.zeros(p.nnz)))
    lb = inst.forward_unrolled(3, 1)
    with pytest.raises(RuntimeError, match="stored trajectory"):
        inst.forward_unrolled(10 ** 8, -1)
    assert inst.lower_bound()[0] == lb  # nothing ran


@pytest.mark.parametrize("case", ["knapsack-small", "team-sizes", "wide-24", "wide-32", "unit-rows"])
def test_dense_routing_matches_listed_routing(case):
    """The reverse sweeps of one-wave diagrams route a level's nonzero adjoints through a per-level
    list, and a level whose list would overflow node by node from the owning lanes; the option
    adj_route_dense takes the second path on every level.  Both follow the same argmins, so pass
    VJPs and unrolled gradients agree up to the order of float sums (a node reached from several
    parents in the pull form, the hi-arc sums), whose rounding accumulates along the paths: a few
    1e-5 relative on the ~1000-level unit-coefficient rows, so the bar is the gradient tests' 1e-4
    (norm-wise and entry-wise with a floor).  A misrouted adjoint would be off by O(1)."""
    import torch
    p = CASES[case]()
    rng = np.random.default_rng(5)
    om = f32(synth.sigmoid(rng.normal(size=p.nnz)))
    ah = f32(rng.normal(0, 0.3, size=p.nnz))
    say(f"dense routing {case}")
    a, _, _ = make_instance(p, om, ah)
    b, _, _ = make_instance(p, om, ah, adj_route_dense=True)
    assert any(s["P"] == 64 for s in a.launch_shapes())
    dev = lambda x: torch.tensor(np.asarray(x, np.float32), device="cuda")

    close = lambda x, y, what: close_grad(x, y, what)

    for direction in (0, 1):
        for inst in (a, b):
            inst.reset()
            inst.run(2)
            if direction == 1:
                inst.run_pass(0)
        (la, Ma), (lb, Mb) = a.get_state(), b.get_state()
        np.testing.assert_array_equal(host(la), host(lb))
        dlo, dmo = rng.normal(size=p.nnz), rng.normal(size=p.nnz)
        ra = [host(t) for t in a.pass_vjp(direction, la, Ma, dev(dlo), dev(dmo))]
        rb = [host(t) for t in b.pass_vjp(direction, lb, Mb, dev(dlo), dev(dmo))]
        for x, y, name in zip(rb, ra, ("dlam_in", "dM_in", "d_alpha", "d_omega")):
            close(x, y, f"dir {direction} {name}")
    for inst in (a, b):
        inst.reset()
    lba, lbb = a.forward_unrolled(3, 1), b.forward_unrolled(3, 1)
    assert lba == lbb
    ga = [host(t) for t in a.backward(1.0)]
    gb = [host(t) for t in b.backward(1.0)]
    for x, y, name in zip(gb, ga, ("d_omega", "d_alpha", "d_c")):
        close(x, y, name)


def test_knapsack_full_reverse_mode():
    """Reverse mode on the full 2,000,000-variable knapsack program in the benchmark's launch
    configuration (one-wave diagrams: sparse routing, recorded argmins).  Rows cannot be sampled
    here (dM_in sums over every row of a variable), so the checks are those that hold at any size:
    Euler's identity for each pass adjoint, <d_c, c> = LB for the unrolled gradient, and the stored
    trajectory against checkpoints every iteration, bit for bit."""
    import torch
    w = synth.workload("knapsack")
    p = w["problem"]
    say(f"knapsack full reverse mode E={p.nnz}: compiling")
    inst, _, _ = make_instance(p, f32(w["omega"]), f32(w["alpha_hat"]))
    assert any(s["P"] == 64 for s in inst.launch_shapes())
    rng = np.random.default_rng(31)
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    inst.run(2)
    for direction in (0, 1):
        lam_in, M_in = inst.get_state()
        li, mi = host(lam_in), host(M_in)
        dlo, dmo = f32(rng.normal(size=p.nnz)), f32(rng.normal(size=p.nnz))
        say(f"  pass vjp dir {direction}")
        dli, dmi, da, dw = (host(t) for t in inst.pass_vjp(direction, lam_in, M_in, dev(dlo), dev(dmo)))
        lam_o, M_o = (host(t) for t in inst.get_state())
        for a in (dli, dmi, da, dw):
            assert np.isfinite(a).all()
        terms = np.concatenate([dli * li, dmi * mi])
        euler_close(terms.sum(), dlo @ lam_o + dmo @ M_o, np.abs(terms).sum(), f"dir {direction}")
    say("  unrolled T=2, checkpoints every iteration and stored")
    lb1 = inst.forward_unrolled(2, 1)
    g1 = [host(t) for t in inst.backward(1.0)]
    lbs = inst.forward_unrolled(2, -1)
    gs = [host(t) for t in inst.backward(1.0)]
    assert lbs == lb1
    for a, b, name in zip(g1, gs, ("d_omega", "d_alpha", "d_c")):
        assert np.isfinite(a).all()
        np.testing.assert_array_equal(a, b, err_msg=name)
    dc = g1[2]
    c = f32(p.c)
    euler_close(dc @ c, lb1, np.abs(dc * c).sum(), "<d_c, c> = LB")
    del inst
    torch.cuda.synchronize()


def test_gm_mini_unrolled_gradient(orc):
    """The 50-assignment-variable graph-matching instance whose oracle gradient is pinned by
    central differences on every coordinate; T = 20, checkpoints every 5."""
    p = synth.graph_matching(n_left=5, n_right=10, cand=10, n_pairs=60, seed=35)
    rng = np.random.default_rng(34)
    om = f32(synth.sigmoid(rng.normal(size=p.nnz)))
    ah = f32(rng.normal(0.0, 0.5, size=p.nnz))
    inst, _, alt = make_instance(p, om, ah)
    al = host(alt)
    lb = inst.forward_unrolled(20, 5)
    dw, da, dc = (host(t) for t in inst.backward(1.0))
    pc = synth.Problem(p.n, f32(p.c), p.row_ptr, p.col, p.coef, p.sense, p.rhs)
    lb_o, dw_o, da_o, dc_o, gap = orc.unrolled_grad(pc, om, al, 20, with_gap=True)
    say(f"  gm mini: smallest decision gap {gap:.3g}")
    assert lb == pytest.approx(lb_o, rel=1e-5, abs=1e-6)
    euler_close(dc @ pc.c, lb, np.abs(dc * pc.c).sum(), "<d_c, c> = LB")
    assert gap >= GAP_MIN  # seeds chosen so that every decision is unique
    close_grad(dw, dw_o, "d_omega")
    close_grad(da, da_o, "d_alpha")
    close_grad(dc, dc_o, "d_c")


def test_gm_full_unrolled_gradient(orc):
    """Full graph-matching shape (1.44M edges), T = 20 with checkpoints every 5, learned-style
    omega and alpha.  Among 600k rows and 40 passes some decisions are near-ties (the oracle
    reports gaps down to ~1e-8), where fp32 and fp64 may pick different (equally valid)
    subgradients and the difference spreads through the shared variables of earlier passes.
    So: the bound to 1e-5, Euler's identity, and the gradients to 1e-4 on at least 99.5% of
    the entries and 2e-3 in norm.  The per-pass adjoint at this size is compared exactly on
    the rows without near-ties by test_pass_vjp_matches_oracle[gm-full]."""
    w = synth.workload("gm")
    p = w["problem"]
    om, ah = f32(w["omega"]), f32(w["alpha_hat"])
    inst, _, alt = make_instance(p, om, ah)
    al = host(alt)
    lb = inst.forward_unrolled(20, 5)
    dw, da, dc = (host(t) for t in inst.backward(1.0))
    pc = synth.Problem(p.n, f32(p.c), p.row_ptr, p.col, p.coef, p.sense, p.rhs)
    lb_o, dw_o, da_o, dc_o, gap = orc.unrolled_grad(pc, om, al, 20, with_gap=True)
    say(f"  gm full: smallest decision gap {gap:.3g}")
    assert lb == pytest.approx(lb_o, rel=1e-5)
    euler_close(dc @ pc.c, lb, np.abs(dc * pc.c).sum(), "<d_c, c> = LB")
    for nm, g, r in (("d_omega", dw, dw_o), ("d_alpha", da, da_o), ("d_c", dc, dc_o)):
        assert np.isfinite(g).all()
        rel = np.linalg.norm(g - r) / np.linalg.norm(r)
        err = np.abs(g - r)
        bad = err > np.maximum(GRAD_RTOL * np.abs(r), GRAD_RTOL * np.abs(r).max())
        say(f"  {nm}: relative norm error {rel:.2e}, entries off {bad.mean():.2e}")
        assert rel <= 2e-3, nm
        assert bad.mean() <= 5e-3, nm


def test_backward_is_linear_in_the_seed_and_checkpoint_free():
    p = CASES["gm-small"]()
    rng = np.random.default_rng(5)
    inst, _, _ = make_instance(p, synth.sigmoid(rng.normal(size=p.nnz)), rng.normal(0, 0.3, size=p.nnz))
    inst.forward_unrolled(6, 2)
    g1 = [host(t) for t in inst.backward(1.0)]
    g2 = [host(t) for t in inst.backward(-2.5)]
    for a, b in zip(g1, g2):
        np.testing.assert_allclose(b, -2.5 * a, rtol=1e-6, atol=1e-6 * max(1.0, np.abs(a).max()))
    inst.forward_unrolled(6, 6)  # one segment: same numbers (replays are bit-exact)
    g3 = [host(t) for t in inst.backward(1.0)]
    for a, b in zip(g1, g3):
        np.testing.assert_array_equal(a, b)


def test_backward_needs_a_recorded_forward():
    import paper_2205_11638_amd as dd
    p = CASES["mixed0"]()
    inst, _, _ = make_instance(p)
    with pytest.raises(dd.DDError) as e:
        inst.backward(1.0)
    assert e.value.code == dd.binding.DD_E_STATE
    inst.forward_unrolled(2)
    inst.run_pass(0)  # the state moved on: the record is stale
    with pytest.raises(dd.DDError):
        inst.backward(1.0)


def test_autograd_function(orc):
    import torch

    from paper_2205_11638_amd.autograd import dual_lower_bound
    p = CASES["gm-small"]()
    rng = np.random.default_rng(1)
    inst, _, _ = make_instance(p)
    c = torch.tensor(p.c, dtype=torch.float32, device="cuda", requires_grad=True)
    om = torch.tensor(synth.sigmoid(rng.normal(size=p.nnz)), dtype=torch.float32, device="cuda", requires_grad=True)
    ah = torch.tensor(rng.normal(0, 0.3, size=p.nnz), dtype=torch.float32, device="cuda", requires_grad=True)
    lb = dual_lower_bound(inst, c, om, ah, 4, 2)
    (-lb).backward()
    pc = synth.Problem(p.n, f32(p.c), p.row_ptr, p.col, p.coef, p.sense, p.rhs)
    al = orc.softmax_alpha(pc, f32(host(ah)))
    lb_o, dw_o, da_o, dc_o, gap = orc.unrolled_grad(pc, f32(host(om)), al, 4, with_gap=True)
    assert lb.item() == pytest.approx(lb_o, rel=1e-5)
    assert gap >= GAP_MIN
    close_grad(-host(c.grad), dc_o, "d_c")
    close_grad(-host(om.grad), dw_o, "d_omega")
    close_grad(-host(ah.grad), orc.softmax_alpha_vjp(pc, al, da_o), "d_alpha_hat")
