"""GPU reverse mode (Alg. 2 through unrolled passes) against the FP64 oracle's literal Alg. 2.

The oracle traces the minimizers s^j(i, beta) of every block explicitly on the partial-sum
diagram; the GPU routes adjoints through argmins of its BDD sweeps.  Where every decision an
output depends on is unique the two must agree: gradients to 1e-4 relative, norm-wise per
parameter vector and entry-wise with a floor of 1e-4 * max |reference|.

Near-ties.  Where the two options of a decision lie within the GPU's rounding error of each
other, fp32 and fp64 may legitimately take different sides, and both results are valid
subgradients.  The oracle reports, per output entry, a flip bound: how far flips of such
decisions can move the entry (0: the entry is determined).  The decision tolerance of row j
(flip_tol) is derived, not chosen: a value the GPU compares is a path cost of row j, a sum of at
most L_j + 2 fp32 terms of size at most s_j = sum_e |lambda_e|, whose rounding is at most
(L_j + 2) u s_j (u = 2^-24), plus sum_e |d lambda_e| for the multipliers that the GPU and the
oracle hold differently (measured: the pass outputs, or both trajectories); two values form a
decision, hence the factor 2.  Determined entries are compared at the gradient bar, the others
within their bound plus the bar, and Euler's identity for positively homogeneous maps (which
every linear piece meeting at the point satisfies) checks the rest.

Long unrolled chains.  Over many passes with shared variables the flips of earlier passes reach
every entry (the flip bounds grow without limit), so the full graph-matching gradient is instead
held to the oracle's own conditioning: the oracle's gradient along its trajectory with the state
rounded to float32 after every pass (fp64 arithmetic otherwise) moves by a measured spread, and
the GPU, whose fp32 arithmetic perturbs each pass by a few such roundings, must lie within 3x
that spread; the oracle chained along the GPU's own trajectory separates the adjoint kernels'
error from the drift of the trajectory.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import coded_and_raw_problem, host, make_instance, say, wide_class_problem

pytestmark = pytest.mark.gpu
GRAD_RTOL = 1e-4
U32 = 2.0 ** -24
# min fraction of entries whose decisions are all unique (flip bound 0) in the per-pass and unrolled checks
MIN_DETERMINED = 0.5


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


def row_sum(prob, x):
    rowid = np.repeat(np.arange(prob.m), np.diff(prob.row_ptr))
    return np.bincount(rowid, weights=x, minlength=prob.m)


def flip_tol(prob, pairs):
    """Decision tolerance of every row (see the module docstring): pairs are (GPU, oracle) multiplier
    arrays the decisions of the compared computation may use."""
    d = np.zeros(prob.nnz)
    s = np.zeros(prob.nnz)
    for g, o in pairs:
        d = np.maximum(d, np.abs(g - o))
        s = np.maximum(s, np.maximum(np.abs(g), np.abs(o)))
    L = np.diff(prob.row_ptr)
    return 2.0 * ((L + 2) * U32 * row_sum(prob, s) + row_sum(prob, d))


def close_bounded(got, ref, bnd, what, scale=None):
    """Determined entries (flip bound 0) at the gradient bar: norm-wise, 1e-4 of the whole vector's
    norm; entry-wise, 1e-4 of the larger of |ref|, max |ref| and the entry's own rounding scale
    (scale: d_omega = Mt (m1 - m0) carries the rounding of path costs of size s_j, so its scale is
    |Mt| s_j, as min-marginals are compared at 1e-4 max(|ref|, s_j)).  Every other entry within its
    flip bound plus that bar.  Returns the fraction of determined entries."""
    got, ref, bnd = (np.asarray(x, dtype=np.float64) for x in (got, ref, bnd))
    if not ref.size:
        return 1.0
    det = bnd == 0
    floor = GRAD_RTOL * max(np.abs(ref).max(), 1e-6)
    bar = np.maximum(GRAD_RTOL * np.abs(ref), floor)
    if scale is not None:
        bar = np.maximum(bar, GRAD_RTOL * np.asarray(scale, dtype=np.float64))
    if det.any():
        dn = np.linalg.norm((got - ref)[det])
        size = np.abs(ref) if scale is None else np.maximum(np.abs(ref), scale)
        assert dn <= GRAD_RTOL * max(np.linalg.norm(size), 1e-6), (what, dn, np.linalg.norm(size))
    bad = np.abs(got - ref) > bnd + bar
    assert not bad.any(), (what, int(bad.sum()), int(np.argmax(np.abs(got - ref) - bnd - bar)))
    return float(det.mean())


def gpu_states(inst, T, lbs=None, start=None):
    """The GPU's 2T + 1 states (lambda, M) before every pass of T iterations from the reset state (or
    from start = (lambda, M) device tensors) and after the last (host float64), by single passes --
    the kernels an unrolled forward launches, so the same bits.  lbs (a list) receives the GPU's lower
    bound after every iteration.  Leaves the instance at the start state."""
    begin = inst.reset if start is None else (lambda: inst.set_state(*start))
    begin()
    out = [tuple(host(t) for t in inst.get_state())]
    for q in range(2 * T):
        inst.run_pass(q % 2)
        out.append(tuple(host(t) for t in inst.get_state()))
        if lbs is not None and q % 2:
            lbs.append(inst.lower_bound()[0])
    begin()
    return out


def trajectory_tolerances(prob, alpha, states_g, states_o, orc):
    """[2T + 1, m]: flip_tol of every pass (its input and output multipliers on both engines) and of
    the seed (the flushed multipliers of the final states)."""
    tol = [flip_tol(prob, [(states_g[q][0], states_o[q][0]), (states_g[q + 1][0], states_o[q + 1][0])])
           for q in range(len(states_g) - 1)]
    var = prob.col.astype(np.int64)

    def flushed(lam, M):
        S = np.zeros(prob.n)
        np.add.at(S, var, M)
        return lam + alpha * S[var]
    tol.append(flip_tol(prob, [(flushed(*states_g[-1]), flushed(*states_o[-1]))]))
    return np.array(tol)


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
    "wide-64": lambda: wide_class_problem(64)[0],
    "unit-rows": unit_rows_problem,
    "coded-raw": coded_and_raw_problem,
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
    lo, Mo = li.copy(), mi.copy()
    orc.run_pass(p, om, al, lo, Mo, direction)
    np.testing.assert_allclose(lam_o, lo, atol=1e-4 * np.abs(lo).max())
    tol = flip_tol(p, [(lam_o, lo)])  # same pass input on both engines
    *r, bnd = orc.pass_vjp(p, om, al, direction, li, mi, f32(dlo), f32(dmo), row_tol=tol)
    for a in (dli, dmi, da, dw):
        assert np.isfinite(a).all()
    det = [close_bounded(g, ref, b, nm, sc) for g, ref, b, nm, sc in
           zip((dli, dmi, da, dw), r, bnd, ("dlam_in", "dM_in", "d_alpha", "d_omega"), (None, None, None, bnd[4]))]
    say("  determined entries " + " ".join(f"{d:.3f}" for d in det))
    assert min(det) >= MIN_DETERMINED
    rowid = np.repeat(np.arange(p.m), np.diff(p.row_ptr))
    tie_row = np.zeros(p.m, bool)
    tie_row[rowid[(bnd[0] > 0) | (bnd[2] > 0) | (bnd[3] > 0)]] = True
    # Euler's identity over all rows, then for each near-tie row on its own (seed on that row only)
    terms = np.concatenate([dli * li, dmi * mi])
    euler_close(terms.sum(), f32(dlo) @ lam_o + f32(dmo) @ M_o, np.abs(terms).sum(), "all rows")
    for j in np.flatnonzero(tie_row)[:6]:
        on = (rowid == j).astype(np.float64)
        dl, dm, _, _ = (host(t) for t in inst.pass_vjp(direction, lam_in, M_in, dev(dlo * on), dev(dmo * on)))
        terms = np.concatenate([dl * li, dm * mi])
        euler_close(terms.sum(), f32(dlo * on) @ lam_o + f32(dmo * on) @ M_o, np.abs(terms).sum(), f"row {j}")


def unrolled_against_oracle(orc, p, om, ah, T, K, what, min_det=MIN_DETERMINED):
    """Unrolled bound and gradient of the GPU (T iterations, checkpoints every K) against the oracle:
    the bound after every iteration to 1e-5, determined gradient entries at the gradient bar, the
    others within their flip bounds (decision tolerances from both engines' trajectories), Euler's
    identity <d_c, c> = LB."""
    inst, omt, alt = make_instance(p, om, ah)
    al = host(alt)
    pc = synth.Problem(p.n, f32(p.c), p.row_ptr, p.col, p.coef, p.sense, p.rhs)
    lbs = []
    states_g = gpu_states(inst, T, lbs)
    states_o = orc.trajectory(pc, om, al, T)
    for t, lb_g in enumerate(lbs):
        lb_t = orc.lower_bound(pc, al, *states_o[2 * t + 2])[0]
        assert lb_g == pytest.approx(lb_t, rel=1e-5, abs=1e-6), (what, t + 1)
    ptol = trajectory_tolerances(pc, al, states_g, states_o, orc)
    lb = inst.forward_unrolled(T, K)
    dw, da, dc = (host(t) for t in inst.backward(1.0))
    lb_o, dw_o, da_o, dc_o, bnd = orc.unrolled_grad(pc, om, al, T, pass_tol=ptol)
    assert lb == pytest.approx(lb_o, rel=1e-5, abs=1e-6)
    euler_close(dc @ pc.c, lb, np.abs(dc * pc.c).sum(), "<d_c, c> = LB")
    for a in (dw, da, dc):
        assert np.isfinite(a).all()
    det = [close_bounded(g, ref, b, nm, sc) for g, ref, b, nm, sc in
           zip((dw, da, dc), (dw_o, da_o, dc_o), bnd[:3], ("d_omega", "d_alpha", "d_c"), (bnd[3], None, None))]
    say(f"  {what}: determined entries " + " ".join(f"{d:.3f}" for d in det))
    assert min(det) >= min_det
    # the state is the final one again: the bound is unchanged
    assert inst.lower_bound()[0] == pytest.approx(lb, rel=1e-6, abs=1e-7)
    return inst, lb


@pytest.mark.parametrize("case,T,K,seed", [("mixed0", 3, 2, 23), ("setcover", 4, 3, 3), ("gm-small", 5, 2, 1),
                                           ("team-sizes", 3, 1, 0), ("knapsack-small", 3, 5, 0),
                                           ("coded-raw", 2, 1, 4)])
def test_unrolled_gradient_matches_oracle(orc, case, T, K, seed):
    p = CASES[case]()
    rng = np.random.default_rng(seed)
    om = f32(synth.sigmoid(rng.normal(size=p.nnz)))
    ah = f32(rng.normal(0, 0.3, size=p.nnz))
    say(f"unrolled grad {case} T={T} K={K}")
    unrolled_against_oracle(orc, p, om, ah, T, K, case)


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


@pytest.mark.parametrize("case", ["knapsack-small", "team-sizes", "wide-24", "wide-32", "wide-64", "unit-rows",
                                  "coded-raw"])
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


def test_knapsack_full_pass_vjp_sampled_rows(orc):
    """Alg. 2 on the full 2,000,000-variable knapsack program in the benchmark's launch configuration,
    checked on the 400 seeded rows of the forward parity test.  The adjoints of the pass outputs are
    random on those rows and zero elsewhere, so the other rows' adjoints are exactly zero, dM_in is the
    sum of the sampled rows' shares per variable, and the oracle (Alg. 2 on the subset, with S per edge
    from the GPU's pass-start M) gives every value; near-ties as in the other per-pass checks."""
    import torch
    w = synth.workload("knapsack")
    p = w["problem"]
    say(f"knapsack full pass adjoint E={p.nnz}: compiling")
    inst, omt, alt = make_instance(p, f32(w["omega"]), f32(w["alpha_hat"]))
    om64, al64 = host(omt), host(alt)
    rows = np.sort(np.random.default_rng(4004).choice(p.m, size=400, replace=False))
    sub = p.subset_rows(rows)
    eidx = np.concatenate([np.arange(p.row_ptr[r], p.row_ptr[r + 1]) for r in rows])
    on = np.zeros(p.nnz, bool)
    on[eidx] = True
    var = p.col.astype(np.int64)
    touched = np.zeros(p.n, bool)
    touched[var[eidx]] = True
    te = touched[var]  # every edge of a variable of the sample
    rng = np.random.default_rng(41)
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    inst.run(2)
    for direction in (0, 1):
        lam_in, M_in = inst.get_state()
        li, mi = host(lam_in), host(M_in)
        S = np.zeros(p.n)
        np.add.at(S, var, mi)
        dlo, dmo = f32(rng.normal(size=p.nnz)) * on, f32(rng.normal(size=p.nnz)) * on
        say(f"  pass vjp dir {direction}")
        dli, dmi, da, dw = (host(t) for t in inst.pass_vjp(direction, lam_in, M_in, dev(dlo), dev(dmo)))
        lam_o, M_o = (host(t) for t in inst.get_state())
        for a in (dli, dmi, da, dw):
            assert np.isfinite(a).all()
        assert not dli[~on].any() and not da[~on].any() and not dw[~on].any() and not dmi[~te].any()
        lo, Mo = orc.rows_pass(sub, om64[eidx], al64[eidx], S[var[eidx]], li[eidx], direction)
        tol = flip_tol(sub, [(lam_o[eidx], lo)])
        dli_o, gS_o, da_o, dw_o, _, _, bnd = orc.rows_pass_vjp(sub, om64[eidx], al64[eidx], S[var[eidx]], direction,
                                                               li[eidx], dlo[eidx], dmo[eidx], row_tol=tol)
        gv, bv = np.zeros(p.n), np.zeros(p.n)
        np.add.at(gv, var[eidx], gS_o)
        np.add.at(bv, var[eidx], bnd[1])
        det = [close_bounded(dli[eidx], dli_o, bnd[0], "dlam_in"),
               close_bounded(dmi[te], gv[var[te]], bv[var[te]], "dM_in"),
               close_bounded(da[eidx], da_o, bnd[2], "d_alpha"),
               close_bounded(dw[eidx], dw_o, bnd[3], "d_omega", bnd[4])]
        say(f"  dir {direction}: {len(rows)} rows, {len(eidx)} edges; determined entries "
            + " ".join(f"{d:.3f}" for d in det))
        assert min(det) >= MIN_DETERMINED
        terms = np.concatenate([dli * li, dmi * mi])
        euler_close(terms.sum(), dlo @ lam_o + dmo @ M_o, np.abs(terms).sum(), f"dir {direction}")
    del inst
    torch.cuda.synchronize()


def test_knapsack_cluster_unrolled(orc):
    """T = 10 forward and adjoint (checkpoints every 5) of the full knapsack's rows on a standalone
    sub-instance: 40 rows grown from the first seeded row through shared variables (rows drawn at
    random from 40,000 share almost no variable, and then the bound does not depend on omega or
    alpha at all).  The bound after every iteration to 1e-5 and the gradient as in the other unrolled
    checks; the oracle's spread under float32 rounding of its states is reported beside it."""
    w = synth.workload("knapsack")
    p = w["problem"]
    rows = np.sort(np.random.default_rng(4004).choice(p.m, size=400, replace=False))
    cl = synth.row_cluster(p, rows[0], 40)
    sub = p.subset_rows(cl)
    eidx = np.concatenate([np.arange(p.row_ptr[r], p.row_ptr[r + 1]) for r in cl])
    om, ah = f32(w["omega"])[eidx], f32(w["alpha_hat"])[eidx]
    del p, w
    say(f"knapsack cluster: {sub.m} rows, {sub.nnz} edges, {int((np.bincount(sub.col) > 1).sum())} shared variables")
    unrolled_against_oracle(orc, sub, om, ah, 10, 5, "knapsack cluster")


def test_gm_mini_unrolled_gradient(orc):
    """The 50-assignment-variable graph-matching instance whose oracle gradient is pinned by
    central differences on every coordinate; T = 20, checkpoints every 5."""
    p = synth.graph_matching(n_left=5, n_right=10, cand=10, n_pairs=60, seed=35)
    rng = np.random.default_rng(34)
    om = f32(synth.sigmoid(rng.normal(size=p.nnz)))
    ah = f32(rng.normal(0.0, 0.5, size=p.nnz))
    unrolled_against_oracle(orc, p, om, ah, 20, 5, "gm mini")


# factor between the GPU's fp32 perturbation of one pass (a few roundings per multiplier: the
# update lambda - M' + alpha S and the sums it uses) and rounding the stored state once
COND_FACTOR = 3.0


def rel_norm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_gm_full_unrolled_gradient(orc):
    """Full graph-matching shape (1.44M edges), T = 20 with checkpoints every 5, learned-style
    omega and alpha.  Over 40 passes and variables in ~42 rows, flips of near-tie decisions reach
    every entry, so the end-to-end gradient is held to the oracle's own conditioning at fp32
    resolution: the oracle's gradient along its trajectory with the state rounded to float32 after
    every pass moves by a spread s (per vector, relative norm), and the GPU must lie within
    COND_FACTOR * s (at least the 1e-4 bar).  Then every step of the GPU's reverse sweep is checked
    on its own inputs: the seed (argmin at the final flushed multipliers) and each of the 40 pass
    adjoints, given the GPU's pass-start state and the adjoints the GPU handed to that pass, against
    the oracle's Alg. 2 on the same inputs, entry by entry with flip bounds; chaining the GPU's pass
    adjoints reproduces its unrolled gradient."""
    import torch
    w = synth.workload("gm")
    p = w["problem"]
    om, ah = f32(w["omega"]), f32(w["alpha_hat"])
    T = 20
    inst, _, alt = make_instance(p, om, ah)
    al = host(alt)
    say("gm full: GPU trajectory")
    states_g = gpu_states(inst, T)
    lb = inst.forward_unrolled(T, 5)
    g = [host(t) for t in inst.backward(1.0)]
    pc = synth.Problem(p.n, f32(p.c), p.row_ptr, p.col, p.coef, p.sense, p.rhs)
    say("gm full: oracle")
    lb_o, *g_o = orc.unrolled_grad(pc, om, al, T)
    assert lb == pytest.approx(lb_o, rel=1e-5)
    euler_close(g[2] @ pc.c, lb, np.abs(g[2] * pc.c).sum(), "<d_c, c> = LB")
    say("gm full: oracle along its float32-rounded trajectory")
    _, *g_r = orc.unrolled_grad_along(pc, om, al, orc.trajectory(pc, om, al, T, round_f32=True))
    for nm, a, ref, rr in zip(("d_omega", "d_alpha", "d_c"), g, g_o, g_r):
        assert np.isfinite(a).all()
        err, spread = rel_norm(a, ref), rel_norm(rr, ref)
        say(f"  {nm}: GPU vs oracle {err:.2e}; oracle spread under fp32 rounding {spread:.2e}")
        assert err <= max(COND_FACTOR * spread, GRAD_RTOL), nm

    # the reverse sweep step by step on the GPU's own inputs
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    var = p.col.astype(np.int64)
    lbar = host(inst.get_state(flushed=True)[0])  # the instance is at the final state again
    x = host(inst.argmin_assignment(flushed=True))
    xo, _, gap = orc.argmin(pc, lbar, row_gaps=True)
    uniq = ~(gap <= flip_tol(pc, [(lbar, lbar)]))[np.repeat(np.arange(p.m), np.diff(p.row_ptr))]
    np.testing.assert_array_equal(x[uniq], xo[uniq])
    say(f"  seed: rows with a near-tie {int((~uniq).sum())} edges of {p.nnz}")
    S = np.zeros(p.n)
    np.add.at(S, var, states_g[-1][1])
    da_c, dw_c = x * S[var], np.zeros(p.nnz)
    gv = np.zeros(p.n)
    np.add.at(gv, var, x * al)
    dl, dM = x, gv[var]
    dets = []
    for q in range(2 * T - 1, -1, -1):
        li, mi = states_g[q]
        out = [host(t) for t in inst.pass_vjp(q % 2, dev(li), dev(mi), dev(dl), dev(dM))]
        lam_out = host(inst.get_state()[0])
        lo, Mo = li.copy(), mi.copy()
        orc.run_pass(pc, om, al, lo, Mo, q % 2)
        *r, bnd = orc.pass_vjp(pc, om, al, q % 2, li, mi, dl, dM, row_tol=flip_tol(pc, [(lam_out, lo)]))
        dets.append([close_bounded(a, ref, b, f"pass {q} {nm}", sc) for a, ref, b, nm, sc in
                     zip(out, r, bnd, ("dlam_in", "dM_in", "d_alpha", "d_omega"), (None, None, None, bnd[4]))])
        dl, dM = out[0], out[1]
        da_c += out[2]
        dw_c += out[3]
    dets = np.array(dets)
    say(f"  passes: determined entries min {dets.min(0).round(3).tolist()} mean {dets.mean(0).round(3).tolist()}")
    assert dets.min() >= MIN_DETERMINED
    deg = np.bincount(var, minlength=p.n).astype(np.float64)
    dc_c = np.where(deg == 0, (pc.c < 0).astype(np.float64), 0.0)
    np.add.at(dc_c, var, dl / np.maximum(deg[var], 1.0))
    for nm, a, cc in zip(("d_omega", "d_alpha", "d_c"), g, (dw_c, da_c, dc_c)):
        say(f"  {nm}: unrolled backward vs its passes chained {rel_norm(a, cc):.2e}")
        assert rel_norm(a, cc) <= 1e-5, nm
    del states_g, inst
    torch.cuda.synchronize()


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
    g4 = [host(t) for t in inst.backward(1.0)]  # one segment kept by the forward: read again
    for a, b in zip(g1, g4):
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


def test_autograd_rejects_a_replaced_record():
    """Two unrolled forwards on one instance (two nodes of a graph): the instance keeps only the
    later record, so the earlier node's backward must fail instead of returning the later one's
    gradients."""
    import torch

    import paper_2205_11638_amd as dd
    from paper_2205_11638_amd.autograd import dual_lower_bound
    p = CASES["gm-small"]()
    rng = np.random.default_rng(2)
    inst, _, _ = make_instance(p)
    c = torch.tensor(p.c, dtype=torch.float32, device="cuda", requires_grad=True)
    om = torch.tensor(synth.sigmoid(rng.normal(size=p.nnz)), dtype=torch.float32, device="cuda", requires_grad=True)
    ah = torch.tensor(rng.normal(0, 0.3, size=p.nnz), dtype=torch.float32, device="cuda", requires_grad=True)
    lb1 = dual_lower_bound(inst, c, om, ah, 3, 1)
    lb2 = dual_lower_bound(inst, c, om, ah, 4, 1)
    with pytest.raises(dd.DDError) as e:
        lb1.backward()
    assert e.value.code == dd.binding.DD_E_STATE
    lb2.backward()  # the current record's node still works
    assert c.grad is not None and torch.isfinite(c.grad).all()
    assert inst.record_serial() >= 0
    inst.run_pass(0)
    assert inst.record_serial() == -1


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
    states_g = gpu_states(inst, 4)  # the parameters the function set are still on the instance
    states_o = orc.trajectory(pc, f32(host(om)), al, 4)
    ptol = trajectory_tolerances(pc, al, states_g, states_o, orc)
    lb_o, dw_o, da_o, dc_o, bnd = orc.unrolled_grad(pc, f32(host(om)), al, 4, pass_tol=ptol)
    assert lb.item() == pytest.approx(lb_o, rel=1e-5)
    assert not any(b.any() for b in bnd[:3])  # every decision of this trajectory is unique
    close_grad(-host(c.grad), dc_o, "d_c")
    close_grad(-host(om.grad), dw_o, "d_omega")
    close_grad(-host(ah.grad), orc.softmax_alpha_vjp(pc, al, da_o), "d_alpha_hat")
