"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: enumeration,
closed forms, Prop. 1's invariants, LP/ILP bounds, a hand-worked example, and
an independent torch implementation of Alg. 1 whose autograd gradient pins
the oracle's literal Alg. 2.
"""
import dataclasses
import json
import os

import numpy as np
import pytest
import torch

import synth
from tests import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def tiny(seed, **kw):
    return synth.random_tiny(seed, **kw)


def uniform_params(p):
    deg = p.degree()
    return np.full(p.nnz, 0.5), 1.0 / deg[p.col]


def learned_params(p, seed):
    rng = np.random.default_rng(seed)
    om = synth.sigmoid(rng.normal(size=p.nnz))
    ah = rng.normal(0.0, 0.5, size=p.nnz)
    return om, ah


# ------------------------------------------------------------------------------------------
# Min-marginals (eq. 8 / Alg. 1 min-marginal line) against enumeration and closed forms
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_min_marginals_match_enumeration(orc, seed):
    p = tiny(seed, n=10, m=6, kmax=9)
    lam = np.random.default_rng(seed + 100).normal(size=p.nnz)
    m0, m1 = orc.min_marginals(p, lam)
    b0, b1 = brute.min_marginals(p, lam)
    np.testing.assert_allclose(m0, b0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(m1, b1, rtol=0, atol=1e-12)
    Ej = orc.energies(p, lam)
    np.testing.assert_allclose(Ej, brute.energies(p, lam), atol=1e-12)
    # invariant: min(m0, m1) = E^j for every variable of row j
    np.testing.assert_allclose(np.minimum(m0, m1), Ej[p.edge_row()], atol=1e-12)


def test_closed_form_at_most_one(orc):
    rng = np.random.default_rng(5)
    L = 7
    p = synth.generators._from_rows(L, np.zeros(L), [(np.arange(L), np.ones(L, np.int32), -1, 1)], "amo")
    lam = rng.normal(size=L)
    m0, m1 = orc.min_marginals(p, lam)
    for i in range(L):
        others = np.delete(lam, i)
        assert m1[i] == pytest.approx(lam[i], abs=1e-14)
        assert m0[i] == pytest.approx(min(0.0, others.min()), abs=1e-14)


def test_closed_form_cover(orc):
    rng = np.random.default_rng(6)
    L = 6
    p = synth.generators._from_rows(L, np.zeros(L), [(np.arange(L), np.ones(L, np.int32), 1, 1)], "cover")
    lam = rng.uniform(0.1, 2.0, size=L)
    m0, m1 = orc.min_marginals(p, lam)
    for i in range(L):
        assert m1[i] == pytest.approx(lam[i], abs=1e-14)
        assert m0[i] == pytest.approx(np.delete(lam, i).min(), abs=1e-14)


def test_argmin_is_optimal(orc):
    p = tiny(3, n=10, m=6, kmax=8)
    lam = np.random.default_rng(1).normal(size=p.nnz)
    x = orc.argmin(p, lam).astype(np.int64)
    sets = brute.row_sets(p)
    for j, X in enumerate(sets):
        a, b = int(p.row_ptr[j]), int(p.row_ptr[j + 1])
        assert any((X == x[a:b]).all(1))                      # feasible
        assert x[a:b] @ lam[a:b] == pytest.approx((X @ lam[a:b]).min(), abs=1e-12)


# ------------------------------------------------------------------------------------------
# Alg. 1 passes: hand-worked example, literal vs incremental, independent torch version
# ------------------------------------------------------------------------------------------

def _gold():
    with open(os.path.join(GOLD, "two_row_iteration.json")) as f:
        g = json.load(f)
    q = g["problem"]
    p = synth.Problem(q["n"], np.array(q["c"]), np.array(q["row_ptr"], np.int64), np.array(q["col"], np.int32),
                      np.array(q["coef"], np.int32), np.array(q["sense"], np.int8), np.array(q["rhs"], np.int64))
    return g, p


@pytest.mark.parametrize("literal", [False, True])
def test_golden_two_row_iteration(orc, literal):
    g, p = _gold()
    om, al = np.array(g["omega"]), np.array(g["alpha"])
    lam = orc.init_lambda(p)
    np.testing.assert_array_equal(lam, g["lambda_init"])
    M = np.zeros(p.nnz)
    assert orc.lower_bound(p, al, lam, M)[0] == g["lb_init"]
    orc.run_pass(p, om, al, lam, M, 0, literal=literal)
    np.testing.assert_array_equal(lam, g["after_forward"]["lambda"])
    np.testing.assert_array_equal(M, g["after_forward"]["M"])
    assert orc.lower_bound(p, al, lam, M)[0] == g["after_forward"]["lb"]
    orc.run_pass(p, om, al, lam, M, 1, literal=literal)
    ab = g["after_backward"]
    np.testing.assert_array_equal(lam, ab["lambda"])
    np.testing.assert_array_equal(M, ab["M"])
    lb, dl, lbar = orc.lower_bound(p, al, lam, M)
    assert lb == ab["lb"] and dl == ab["d_l"]
    np.testing.assert_array_equal(lbar, ab["lambda_bar"])
    m0, m1 = orc.min_marginals(p, lbar)
    np.testing.assert_array_equal(m0, ab["m0_at_lambda_bar"])
    np.testing.assert_array_equal(m1, ab["m1_at_lambda_bar"])
    assert lb <= g["ilp_optimum"]


@pytest.mark.parametrize("seed", range(6))
def test_literal_equals_incremental(orc, seed):
    p = tiny(seed, n=12, m=8, kmax=7)
    om, ah = learned_params(p, seed)
    al = orc.softmax_alpha(p, ah)
    a = orc.run(p, om, al, 6, literal=False)
    b = orc.run(p, om, al, 6, literal=True)
    np.testing.assert_allclose(a[0], b[0], atol=1e-12)
    np.testing.assert_allclose(a[1], b[1], atol=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_trajectory_matches_torch_enumeration(orc, seed):
    p = tiny(seed + 40, n=9, m=6, kmax=6)
    om, ah = learned_params(p, seed)
    al = orc.softmax_alpha(p, ah)
    T = 3
    _, states = brute.dmma_torch(p, torch.tensor(om), torch.tensor(al), T, record=True)
    lam, M = orc.init_lambda(p), np.zeros(p.nnz)
    for k in range(2 * T):
        orc.run_pass(p, om, al, lam, M, k % 2)
        np.testing.assert_allclose(lam, states[k + 1][0].numpy(), atol=1e-12)
        np.testing.assert_allclose(M, states[k + 1][1].numpy(), atol=1e-12)


def test_rows_are_independent_within_a_pass(orc):
    """Reordering the rows gives bitwise the same per-edge result (deferred sums taken at pass start)."""
    p = synth.workload("gm", small=True)["problem"]
    om, ah = learned_params(p, 1)
    al = orc.softmax_alpha(p, ah)
    lam0, M0 = orc.run(p, om, al, 2)
    S = np.zeros(p.n)
    np.add.at(S, p.col.astype(np.int64), M0)
    Se = S[p.col]
    perm = np.random.default_rng(0).permutation(p.m)
    q = p.subset_rows(perm)
    eidx = np.concatenate([np.arange(p.row_ptr[r], p.row_ptr[r + 1]) for r in perm])
    for direction in (0, 1):
        lam, M = orc.rows_pass(p, om, al, Se, lam0, direction)
        lq, Mq = orc.rows_pass(q, om[eidx], al[eidx], Se[eidx], lam0[eidx], direction)
        np.testing.assert_array_equal(lq, lam[eidx])
        np.testing.assert_array_equal(Mq, M[eidx])
        # the full pass with S computed from M0 is the same thing
        lf, Mf = lam0.copy(), M0.copy()
        orc.run_pass(p, om, al, lf, Mf, direction)
        np.testing.assert_array_equal(lf, lam)
        np.testing.assert_array_equal(Mf, M)


# ------------------------------------------------------------------------------------------
# Prop. 1: feasibility and monotonicity; bound validity
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("wl", ["setcover", "indset", "gm"])
def test_prop1_invariants(orc, wl):
    w = synth.workload(wl, small=True)
    p = w["problem"]
    al = orc.softmax_alpha(p, w["alpha_hat"])
    om = w["omega"]
    var = p.col.astype(np.int64)
    deg = p.degree()
    lam, M = orc.init_lambda(p), np.zeros(p.nnz)
    prev_dl = -np.inf
    cov = deg > 0
    for k in range(12):
        orc.run_pass(p, om, al, lam, M, k % 2)
        tot = np.zeros(p.n)
        np.add.at(tot, var, lam + M)
        np.testing.assert_allclose(tot[cov], p.c[cov], rtol=0, atol=1e-12 * max(1.0, np.abs(p.c).max()) * 10)
        lb, dl, lbar = orc.lower_bound(p, al, lam, M)
        tb = np.zeros(p.n)
        np.add.at(tb, var, lbar)
        np.testing.assert_allclose(tb[cov], p.c[cov], atol=1e-11)
        assert dl >= prev_dl - 1e-9 * max(1.0, abs(dl)), (k, dl, prev_dl)
        assert lb >= dl - 1e-9 * max(1.0, abs(dl))
        prev_dl = dl


@pytest.mark.parametrize("seed", range(8))
def test_lb_below_ilp_optimum(orc, seed):
    k = 0
    while True:   # first jointly feasible instance from this seed on
        p = tiny(1000 * seed + k, n=10, m=7, kmax=6, cover_all=True)
        opt = brute.ilp_optimum(p)
        if np.isfinite(opt):
            break
        k += 1
    om, ah = learned_params(p, seed)
    al = orc.softmax_alpha(p, ah)
    lam, M = orc.init_lambda(p), np.zeros(p.nnz)
    for k in range(30):
        orc.run_pass(p, om, al, lam, M, k % 2)
        lb, dl, _ = orc.lower_bound(p, al, lam, M)
        assert lb <= opt + 1e-9 and dl <= lb + 1e-9


@pytest.mark.parametrize("wl", ["setcover", "indset"])
def test_lb_below_lp_optimum(orc, wl):
    from scipy.optimize import linprog
    w = synth.workload(wl, small=True)
    p = w["problem"]
    al = orc.softmax_alpha(p, w["alpha_hat"])
    lam, M = orc.run(p, w["omega"], al, 50)
    lb = orc.lower_bound(p, al, lam, M)[0]
    # LP relaxation: rows as a_j^T x (sense) b_j, 0 <= x <= 1
    import scipy.sparse as sp
    A = sp.csr_matrix((p.coef.astype(float), p.col, p.row_ptr), shape=(p.m, p.n))
    sgn = np.where(p.sense > 0, -1.0, 1.0)
    res = linprog(p.c, A_ub=sp.diags(sgn) @ A, b_ub=sgn * p.rhs, bounds=(0, 1), method="highs")
    assert res.status == 0
    assert lb <= res.fun + 1e-7 * max(1.0, abs(res.fun))
    # the rows' polytopes are integral, so the dual optimum is the LP optimum; DMMA gets close
    assert lb >= res.fun - 0.05 * abs(res.fun)


def test_single_row_lb_is_optimum_every_pass(orc):
    p = tiny(77, n=8, m=1, kmin=8, kmax=8)
    om, ah = learned_params(p, 3)
    al = orc.softmax_alpha(p, ah)
    np.testing.assert_allclose(al, 1.0)
    opt = brute.ilp_optimum(p)
    lam, M = orc.init_lambda(p), np.zeros(p.nnz)
    for k in range(6):
        orc.run_pass(p, om, al, lam, M, k % 2)
        assert orc.lower_bound(p, al, lam, M)[0] == pytest.approx(opt, abs=1e-12)


def test_disjoint_rows_lb_is_optimum(orc):
    rows = [(np.array([0, 1, 2]), np.array([2, -1, 3]), -1, 2), (np.array([3, 4]), np.array([1, 1]), 1, 1),
            (np.array([5, 6, 7]), np.array([1, 1, 1]), 0, 2)]
    p = synth.generators._from_rows(9, np.random.default_rng(2).normal(size=9), rows, "disjoint")
    om, ah = learned_params(p, 9)
    al = orc.softmax_alpha(p, ah)
    opt = brute.ilp_optimum(p)
    lam, M = orc.run(p, om, al, 4)
    assert orc.lower_bound(p, al, lam, M)[0] == pytest.approx(opt, abs=1e-12)


def test_zero_damping_keeps_bound(orc):
    w = synth.workload("setcover")
    p = w["problem"]
    al = orc.softmax_alpha(p, w["alpha_hat"])
    lam0 = orc.init_lambda(p)
    lam, M = orc.run(p, np.zeros(p.nnz), al, 3)
    np.testing.assert_array_equal(lam, lam0)
    assert not M.any()


def test_fastdog_special_case_weights(orc):
    p = synth.workload("gm", small=True)["problem"]
    al = orc.softmax_alpha(p, np.zeros(p.nnz))
    np.testing.assert_allclose(al, 1.0 / p.degree()[p.col], rtol=1e-15)
    al2 = orc.softmax_alpha(p, np.random.default_rng(0).normal(size=p.nnz))
    s = np.zeros(p.n)
    np.add.at(s, p.col.astype(np.int64), al2)
    np.testing.assert_allclose(s[p.degree() > 0], 1.0, rtol=1e-14)


# ------------------------------------------------------------------------------------------
# Alg. 2 and the unrolled gradient: torch autograd over enumeration, central differences
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_pass_vjp_matches_autograd(orc, seed):
    p = tiny(seed + 300, n=9, m=6, kmax=6)
    om, ah = learned_params(p, seed)
    al = orc.softmax_alpha(p, ah)
    rng = np.random.default_rng(seed)
    lam_in, M_in = orc.run(p, om, al, 1)
    for direction in (0, 1):
        dlo, dmo = rng.normal(size=p.nnz), rng.normal(size=p.nnz)
        dli, dmi, da, dw = orc.pass_vjp(p, om, al, direction, lam_in, M_in, dlo, dmo)
        # autograd of the same pass written with enumeration
        L = torch.tensor(lam_in, requires_grad=True)
        Mt = torch.tensor(M_in, requires_grad=True)
        A = torch.tensor(al, requires_grad=True)
        W = torch.tensor(om, requires_grad=True)
        lo, Mo = _torch_pass(p, W, A, L, Mt, direction)
        (lo @ torch.tensor(dlo) + Mo @ torch.tensor(dmo)).backward()
        np.testing.assert_allclose(dli, L.grad.numpy(), atol=1e-10)
        np.testing.assert_allclose(dmi, Mt.grad.numpy(), atol=1e-10)
        np.testing.assert_allclose(da, A.grad.numpy(), atol=1e-10)
        np.testing.assert_allclose(dw, W.grad.numpy(), atol=1e-10)


def _torch_pass(p, W, A, lam, M, direction):
    sets = [torch.tensor(X, dtype=torch.float64) for X in brute.row_sets(p)]
    var = torch.tensor(p.col.astype(np.int64))
    S = torch.zeros(p.n, dtype=torch.float64).index_add(0, var, M)[var]
    lo_parts, M_parts = [], []
    for j, X in enumerate(sets):
        a, b = int(p.row_ptr[j]), int(p.row_ptr[j + 1])
        lj = [lam[a + l] for l in range(b - a)]
        Mj = [None] * (b - a)
        for l in (range(b - a) if direction == 0 else range(b - a - 1, -1, -1)):
            cost = X @ torch.stack(lj)
            Mn = W[a + l] * (cost[X[:, l] == 1].min(dim=0).values - cost[X[:, l] == 0].min(dim=0).values)
            lj[l] = lj[l] - Mn + A[a + l] * S[a + l]
            Mj[l] = Mn
        lo_parts += lj
        M_parts += Mj
    return torch.stack(lo_parts), torch.stack(M_parts)


@pytest.mark.parametrize("seed", range(4))
def test_unrolled_grad_matches_autograd(orc, seed):
    p = tiny(seed + 500, n=9, m=6, kmax=6)
    om, ah = learned_params(p, seed)
    al = orc.softmax_alpha(p, ah)
    T = 3
    lb, dw, da, dc = orc.unrolled_grad(p, om, al, T)
    W = torch.tensor(om, requires_grad=True)
    A = torch.tensor(al, requires_grad=True)
    Cc = torch.tensor(p.c, requires_grad=True)
    lbt, _ = brute.dmma_torch(p, W, A, T, c=Cc)
    lbt.backward()
    assert lb == pytest.approx(lbt.item(), abs=1e-11)
    np.testing.assert_allclose(dw, W.grad.numpy(), atol=1e-10)
    np.testing.assert_allclose(da, A.grad.numpy(), atol=1e-10)
    np.testing.assert_allclose(dc, Cc.grad.numpy(), atol=1e-10)


def test_unrolled_grad_central_differences(orc):
    """Central differences of the oracle's own LB (f64), away from kinks."""
    p = tiny(901, n=10, m=7, kmax=6)
    om, ah = learned_params(p, 4)
    al = orc.softmax_alpha(p, ah)
    T = 4
    lb, dw, da, dc = orc.unrolled_grad(p, om, al, T)
    h = 1e-6
    checked = 0
    for k in range(p.nnz):
        for arr, g in ((om, dw), (al, da)):
            xp, xm = arr.copy(), arr.copy()
            xp[k] += h
            xm[k] -= h
            args_p = (xp, al) if arr is om else (om, xp)
            args_m = (xm, al) if arr is om else (om, xm)
            fp = orc.lb_after(p, *args_p, T)
            fm = orc.lb_after(p, *args_m, T)
            f0 = lb
            # skip coordinates where the LB is not differentiable (one-sided slopes differ)
            if abs((fp - f0) - (f0 - fm)) > 1e-9:
                continue
            assert (fp - fm) / (2 * h) == pytest.approx(g[k], abs=1e-5)
            checked += 1
    for i in range(p.n):
        cp, cm = p.c.copy(), p.c.copy()
        cp[i] += h
        cm[i] -= h
        fp, fm = orc.lb_after(p, om, al, T, c=cp), orc.lb_after(p, om, al, T, c=cm)
        if abs((fp - lb) - (lb - fm)) > 1e-9:
            continue
        assert (fp - fm) / (2 * h) == pytest.approx(dc[i], abs=1e-5)
        checked += 1
    assert checked >= p.nnz


def test_softmax_vjp_matches_autograd(orc):
    p = synth.workload("gm", small=True)["problem"]
    ah = np.random.default_rng(3).normal(size=p.nnz)
    g = np.random.default_rng(4).normal(size=p.nnz)
    al = orc.softmax_alpha(p, ah)
    got = orc.softmax_alpha_vjp(p, al, g)
    A = torch.tensor(ah, requires_grad=True)
    var = torch.tensor(p.col.astype(np.int64))
    mx = torch.zeros(p.n, dtype=torch.float64).index_reduce(0, var, A.detach(), "amax", include_self=False)
    z = torch.exp(A - mx[var])
    den = torch.zeros(p.n, dtype=torch.float64).index_add(0, var, z)
    (z / den[var] @ torch.tensor(g)).backward()
    np.testing.assert_allclose(got, A.grad.numpy(), atol=1e-12)


# ------------------------------------------------------------------------------------------
# Positive homogeneity (every min-marginal, update and bound is a min over path sums, so
# scaling (lambda, M, c) by t > 0 scales every output by t).  Euler's identity then holds for
# the Jacobian of every linear piece that touches the point, so it pins any subgradient the
# reverse mode may pick, ties included.
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("wl", ["gm", "setcover"])
def test_pass_vjp_euler_identity(orc, wl):
    p = synth.workload(wl, small=True)["problem"]
    om, ah = learned_params(p, 11)
    al = orc.softmax_alpha(p, ah)
    lam, M = orc.run(p, om, al, 2)
    rng = np.random.default_rng(12)
    for direction in (0, 1):
        dlo, dmo = rng.normal(size=p.nnz), rng.normal(size=p.nnz)
        dli, dmi, _, _ = orc.pass_vjp(p, om, al, direction, lam, M, dlo, dmo)
        lo, Mo = lam.copy(), M.copy()
        orc.run_pass(p, om, al, lo, Mo, direction)
        lhs = dli @ lam + dmi @ M
        rhs = dlo @ lo + dmo @ Mo
        scale = np.abs(dli * lam).sum() + np.abs(dmi * M).sum()
        assert lhs == pytest.approx(rhs, abs=1e-10 * scale)


@pytest.mark.parametrize("wl", ["gm", "setcover"])
def test_unrolled_grad_euler_identity(orc, wl):
    p = synth.workload(wl, small=True)["problem"]
    om, ah = learned_params(p, 13)
    al = orc.softmax_alpha(p, ah)
    lb, _, _, dc = orc.unrolled_grad(p, om, al, 5)
    assert dc @ p.c == pytest.approx(lb, abs=1e-10 * np.abs(dc * p.c).sum())


def test_argmin_gap_reports_ties(orc):
    p = tiny(77, n=12, m=8, kmax=6)
    x, gap = orc.argmin(p, np.zeros(p.nnz), with_gap=True)
    assert (gap[np.diff(p.row_ptr) > 0] == 0.0).all()  # all-zero costs: every decision is a tie
    lam = np.random.default_rng(5).normal(size=p.nnz)
    x2, gap2 = orc.argmin(p, lam, with_gap=True)
    assert (gap2 > 0).all()  # continuous random costs: unique minimizers
    np.testing.assert_array_equal(x2, orc.argmin(p, lam))
    # a tie made on purpose: two equal-cost optima of a one-row at-most-one constraint
    q = synth.random_tiny(3, n=3, m=1, kmin=3, kmax=3, amin=1, amax=1, senses=(-1,))
    q = dataclasses.replace(q, rhs=np.array([1]))
    _, g = orc.argmin(q, np.array([-1.0, -1.0, 0.5]), with_gap=True)
    assert g[0] == 0.0
    _, g = orc.argmin(q, np.array([-1.0, -1.25, 0.5]), with_gap=True)
    assert g[0] > 0.1
    # absolute gaps: first decision takes var 1 (-1.25) over var 0 (-1): |(-1) - (-1.25)| = 0.25
    _, rel, ab = orc.argmin(q, np.array([-1.0, -1.25, 0.5]), row_gaps=True)
    assert ab[0] == 0.25 and rel[0] == pytest.approx(0.25 / 1.25)


# ------------------------------------------------------------------------------------------
# Alg. 2 on a subset of rows with S given per edge, and the trajectory helpers
# ------------------------------------------------------------------------------------------

def _torch_rows_pass(p, W, A, lam, Se, direction):
    """A pass over every row with the deferred sums given per edge, by enumeration (torch f64)."""
    sets = [torch.tensor(X, dtype=torch.float64) for X in brute.row_sets(p)]
    lo_parts, M_parts = [], []
    for j, X in enumerate(sets):
        a, b = int(p.row_ptr[j]), int(p.row_ptr[j + 1])
        lj = [lam[a + l] for l in range(b - a)]
        Mj = [None] * (b - a)
        for l in (range(b - a) if direction == 0 else range(b - a - 1, -1, -1)):
            cost = X @ torch.stack(lj)
            Mn = W[a + l] * (cost[X[:, l] == 1].min(dim=0).values - cost[X[:, l] == 0].min(dim=0).values)
            lj[l] = lj[l] - Mn + A[a + l] * Se[a + l]
            Mj[l] = Mn
        lo_parts += lj
        M_parts += Mj
    return torch.stack(lo_parts), torch.stack(M_parts)


@pytest.mark.parametrize("seed", range(4))
def test_rows_pass_vjp_matches_autograd(orc, seed):
    """Alg. 2 with S given per edge: the adjoint of S_edge is exactly the edge's share gS = dlambda' alpha."""
    p = tiny(seed + 700, n=9, m=6, kmax=6)
    om, ah = learned_params(p, seed + 1)
    al = orc.softmax_alpha(p, ah)
    rng = np.random.default_rng(seed + 2)
    lam, Se = rng.normal(size=p.nnz), rng.normal(0.0, 0.3, size=p.nnz)
    for direction in (0, 1):
        dlo, dmo = rng.normal(size=p.nnz), rng.normal(size=p.nnz)
        dli, gS, da, dw, _, _ = orc.rows_pass_vjp(p, om, al, Se, direction, lam, dlo, dmo)
        L = torch.tensor(lam, requires_grad=True)
        S = torch.tensor(Se, requires_grad=True)
        A = torch.tensor(al, requires_grad=True)
        W = torch.tensor(om, requires_grad=True)
        lo, Mo = _torch_rows_pass(p, W, A, L, S, direction)
        (lo @ torch.tensor(dlo) + Mo @ torch.tensor(dmo)).backward()
        np.testing.assert_allclose(dli, L.grad.numpy(), atol=1e-10)
        np.testing.assert_allclose(gS, S.grad.numpy(), atol=1e-10)
        np.testing.assert_allclose(da, A.grad.numpy(), atol=1e-10)
        np.testing.assert_allclose(dw, W.grad.numpy(), atol=1e-10)
        lo_o, Mo_o = orc.rows_pass(p, om, al, Se, lam, direction)
        np.testing.assert_allclose(lo_o, lo.detach().numpy(), atol=1e-12)


def test_rows_pass_vjp_on_a_subset_equals_the_whole_pass(orc):
    """Given S, rows are independent: the adjoint of a row subset (S from the whole program's M) equals
    the whole pass's adjoint when the other rows' output adjoints are zero; those rows then get
    exactly zero, and dM_in is the per-variable sum of the subset's shares."""
    w = synth.workload("gm", small=True)
    p = w["problem"]
    om, ah = learned_params(p, 21)
    al = orc.softmax_alpha(p, ah)
    lam, M = orc.run(p, om, al, 2)
    rng = np.random.default_rng(22)
    rows = np.sort(rng.choice(p.m, size=p.m // 5, replace=False))
    sub = p.subset_rows(rows)
    eidx = np.concatenate([np.arange(p.row_ptr[r], p.row_ptr[r + 1]) for r in rows])
    on = np.zeros(p.nnz, bool)
    on[eidx] = True
    var = p.col.astype(np.int64)
    S = np.zeros(p.n)
    np.add.at(S, var, M)
    for direction in (0, 1):
        dlo, dmo = rng.normal(size=p.nnz) * on, rng.normal(size=p.nnz) * on
        dli, dmi, da, dw = orc.pass_vjp(p, om, al, direction, lam, M, dlo, dmo)
        dli_s, gS_s, da_s, dw_s, _, _ = orc.rows_pass_vjp(sub, om[eidx], al[eidx], S[var[eidx]], direction, lam[eidx],
                                                          dlo[eidx], dmo[eidx])
        np.testing.assert_allclose(dli[eidx], dli_s, atol=1e-12)
        np.testing.assert_allclose(da[eidx], da_s, atol=1e-12)
        np.testing.assert_allclose(dw[eidx], dw_s, atol=1e-12)
        assert not dli[~on].any() and not da[~on].any() and not dw[~on].any()
        gv = np.zeros(p.n)
        np.add.at(gv, var[eidx], gS_s)
        np.testing.assert_allclose(dmi, gv[var], atol=1e-12)


def test_unrolled_grad_along_its_own_trajectory(orc):
    """The chain over supplied states reproduces unrolled_grad on the oracle's own trajectory."""
    p = synth.workload("gm", small=True)["problem"]
    om, ah = learned_params(p, 31)
    al = orc.softmax_alpha(p, ah)
    lb, dw, da, dc = orc.unrolled_grad(p, om, al, 4)
    states = orc.trajectory(p, om, al, 4)
    lb2, dw2, da2, dc2 = orc.unrolled_grad_along(p, om, al, states)
    assert lb2 == lb
    for a, b in ((dw, dw2), (da, da2), (dc, dc2)):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())
    lam, M = orc.run(p, om, al, 4)
    np.testing.assert_array_equal(states[-1][0], lam)
    r = orc.trajectory(p, om, al, 4, round_f32=True)
    assert all((s[0] == s[0].astype(np.float32)).all() for s in r[1:])


# ------------------------------------------------------------------------------------------
# Flip bounds: how far near-tie decisions can move the adjoint (the oracle's account of which
# outputs are determined).  Pinned by resolving exact ties both ways with tiny perturbations.
# ------------------------------------------------------------------------------------------

def _tied_rows(seed):
    """Unit-coefficient rows (sum x <= b and sum x >= b) with continuous costs, in which two
    variables of every row get the same multiplier: one exact tie per row."""
    rng = np.random.default_rng(seed)
    n, rows = 14, []
    for j in range(5):
        k = int(rng.integers(4, 7))
        cols = rng.choice(n, size=k, replace=False)
        rows.append((cols, np.ones(k, np.int64), int(rng.choice([-1, 1])), int(rng.integers(1, k))))
    p = synth.generators._from_rows(n, rng.normal(size=n), rows, "tied")
    lam = rng.normal(size=p.nnz)
    for j in range(p.m):
        a, b = int(p.row_ptr[j]), int(p.row_ptr[j + 1])
        i1, i2 = rng.choice(np.arange(a, b), size=2, replace=False)
        lam[i2] = lam[i1]
    return p, lam, rng


def test_flip_bounds_zero_without_ties(orc):
    """A tolerance below every row's smallest decision gap flags nothing; one above it does."""
    p = tiny(801, n=10, m=6, kmax=6)
    om, ah = learned_params(p, 2)
    al = orc.softmax_alpha(p, ah)
    lam, M = orc.run(p, om, al, 1)
    rng = np.random.default_rng(3)
    dlo, dmo = rng.normal(size=p.nnz), rng.normal(size=p.nnz)
    *r, rel, ab = orc.pass_vjp(p, om, al, 0, lam, M, dlo, dmo, row_gaps=True)
    ab = np.where(np.isfinite(ab), ab, 1.0)  # rows with no two-way decision
    assert (ab > 0).all()
    *r2, bnd = orc.pass_vjp(p, om, al, 0, lam, M, dlo, dmo, row_tol=0.5 * ab)
    assert not bnd[:4].any()
    for a, b in zip(r, r2):
        np.testing.assert_array_equal(a, b)
    *_, bnd = orc.pass_vjp(p, om, al, 0, lam, M, dlo, dmo, row_tol=2.0 * ab)
    assert bnd[:4].any()


def test_flip_bounds_cover_tie_resolutions(orc):
    """At a point with exact ties, nudging a tied multiplier by +-eps resolves each tie one way or the
    other (and moves no other decision): every resolved adjoint must lie within the flip bounds
    computed at the tied point, and the ties must matter (the pin is not vacuous)."""
    eps, tol = 1e-9, 1e-7
    seeds_moved = 0
    for seed in range(8):
        p, lam, rng = _tied_rows(900 + seed)
        om = synth.sigmoid(rng.normal(size=p.nnz))
        al = orc.softmax_alpha(p, rng.normal(0.0, 0.5, size=p.nnz))
        M = rng.normal(0.0, 0.2, size=p.nnz)
        moved = 0
        for direction in (0, 1):
            dlo, dmo = rng.normal(size=p.nnz), rng.normal(size=p.nnz)
            *base, bnd = orc.pass_vjp(p, om, al, direction, lam, M, dlo, dmo, row_tol=np.full(p.m, tol))
            for e in range(p.nnz):
                for sgn in (1.0, -1.0):
                    lp = lam.copy()
                    lp[e] += sgn * eps
                    pert = orc.pass_vjp(p, om, al, direction, lp, M, dlo, dmo)
                    for q, (x, y) in enumerate(zip(pert, base)):
                        slack = 1e-6 * max(1.0, np.abs(y).max())  # continuous parts move by O(eps)
                        assert (np.abs(x - y) <= bnd[q] + slack).all(), (seed, direction, e, q)
                        moved += int((np.abs(x - y) > slack).any())
        seeds_moved += moved > 0
    assert seeds_moved >= 5


# ------------------------------------------------------------------------------------------
# Finite differences on the graph-matching shape: every coordinate of a 50-assignment-variable
# instance, and random directions on a 50-variable slice of the full-size instance (T = 20).
# ------------------------------------------------------------------------------------------

def _fd_check(f, f0, g_dot, h, tol, kink=1e-3):
    fp, fm = f(h), f(-h)
    if abs((fp - f0) - (f0 - fm)) > kink * abs(fp - fm) + 1e-12:  # a kink between the two sides
        return None
    return abs((fp - fm) / (2 * h) - g_dot) <= tol * max(1.0, abs(g_dot))


def test_unrolled_grad_fd_gm_mini(orc):
    p = synth.graph_matching(n_left=5, n_right=10, cand=10, n_pairs=60, seed=35)
    assert p.n == 110
    om, ah = learned_params(p, 34)
    al = orc.softmax_alpha(p, ah)
    T = 20
    lb, dw, da, dc = orc.unrolled_grad(p, om, al, T)
    checked = skipped = 0
    for k in range(p.nnz):
        for which, g in (("w", dw), ("a", da)):
            def f(h, k=k, which=which):
                x = (om if which == "w" else al).copy()
                x[k] += h
                return orc.lb_after(p, x, al, T) if which == "w" else orc.lb_after(p, om, x, T)
            r = _fd_check(f, lb, g[k], 1e-6, 1e-5)
            if r is None:
                skipped += 1
                continue
            assert r, (which, k)
            checked += 1
    for i in range(p.n):
        def f(h, i=i):
            c = p.c.copy()
            c[i] += h
            return orc.lb_after(p, om, al, T, c=c)
        r = _fd_check(f, lb, dc[i], 1e-6, 1e-5)
        if r is None:
            skipped += 1
            continue
        assert r, ("c", i)
        checked += 1
    assert checked >= 0.9 * (2 * p.nnz + p.n), (checked, skipped)


@pytest.mark.slow
def test_unrolled_grad_directional_fd_gm_full(orc):
    w = synth.workload("gm")
    p = w["problem"]
    om, ah = w["omega"], w["alpha_hat"]
    al = orc.softmax_alpha(p, ah)
    T = 20
    lb, dw, da, dc = orc.unrolled_grad(p, om, al, T)
    on_e = np.isin(p.col, np.arange(50)).astype(np.float64)  # edges of assignment variables 0..49
    on_v = (np.arange(p.n) < 50).astype(np.float64)
    rng = np.random.default_rng(40)
    checked = 0
    for k in range(8):
        d_w, d_a, d_c = (rng.normal(size=p.nnz) * on_e, rng.normal(size=p.nnz) * on_e * 0.1,
                         rng.normal(size=p.n) * on_v)
        g_dot = dw @ d_w + da @ d_a + dc @ d_c
        # h balances fp64 rounding of a bound of size ~5e4 against the decisions that flip
        # somewhere among 600k rows within +-h (each bends the slope a little)
        r = _fd_check(lambda h: orc.lb_after(p, om + h * d_w, al + h * d_a, T, c=p.c + h * d_c), lb, g_dot, 1e-5,
                      1e-4, kink=1e-2)
        if r is None:
            continue
        assert r, k
        checked += 1
    assert checked >= 6


# ------------------------------------------------------------------------------------------
# Non-parametric update (eq. 2), the output transforms of Alg. 3, and the unrolled gradient
# from an arbitrary start state (a training round starts from the previous round's state)
# ------------------------------------------------------------------------------------------

def test_center_is_the_feasibility_projection(orc):
    p = synth.workload("gm", small=True)["problem"]
    rng = np.random.default_rng(50)
    x, y = rng.normal(size=p.nnz), rng.normal(size=p.nnz)
    cx = orc.center(p, x)
    sums = np.zeros(p.n)
    np.add.at(sums, p.col.astype(np.int64), cx)
    np.testing.assert_allclose(sums, 0.0, atol=1e-12)                   # sums over J_i vanish
    np.testing.assert_allclose(orc.center(p, cx), cx, atol=1e-12)        # idempotent
    assert cx @ y == pytest.approx(x @ orc.center(p, y), abs=1e-10)      # symmetric
    # a variable in one row: its theta is removed entirely
    one = np.bincount(p.col, minlength=p.n)[p.col] == 1
    np.testing.assert_allclose(cx[one], 0.0, atol=1e-15)


def test_nonparam_update_keeps_the_dual_feasible(orc):
    p = synth.workload("gm", small=True)["problem"]
    om, ah = learned_params(p, 51)
    al = orc.softmax_alpha(p, ah)
    lam, M = orc.run(p, om, al, 3)
    th = np.random.default_rng(52).normal(size=p.nnz)
    lam2 = orc.nonparam_update(p, lam, th)
    var = p.col.astype(np.int64)
    tot1, tot2 = np.zeros(p.n), np.zeros(p.n)
    np.add.at(tot1, var, lam + M)
    np.add.at(tot2, var, lam2 + M)
    np.testing.assert_allclose(tot2, tot1, atol=1e-12)   # sum_j (lambda_ij + M_ij) = c_i still holds
    np.testing.assert_allclose(tot1[np.bincount(var, minlength=p.n) > 0],
                               p.c[np.bincount(var, minlength=p.n) > 0], atol=1e-10)


def test_param_transform_vjp_matches_autograd(orc):
    p = synth.workload("gm", small=True)["problem"]
    rng = np.random.default_rng(53)
    wh, ah, th = (rng.normal(size=p.nnz) for _ in range(3))
    g = [rng.normal(size=p.nnz) for _ in range(3)]
    om, al, tt = orc.param_transform(p, wh, ah, th)
    got = orc.param_transform_vjp(p, om, al, *g)
    W, A, Th = (torch.tensor(x, requires_grad=True) for x in (wh, ah, th))
    var = torch.tensor(p.col.astype(np.int64))
    deg = torch.bincount(var, minlength=p.n).to(torch.float64)
    mx = torch.zeros(p.n, dtype=torch.float64).index_reduce(0, var, A.detach(), "amax", include_self=False)
    z = torch.exp(A - mx[var])
    alpha = z / torch.zeros(p.n, dtype=torch.float64).index_add(0, var, z)[var]
    theta = Th - torch.zeros(p.n, dtype=torch.float64).index_add(0, var, Th)[var] / deg[var]
    np.testing.assert_allclose(torch.sigmoid(W).detach().numpy(), om, atol=1e-14)
    np.testing.assert_allclose(alpha.detach().numpy(), al, atol=1e-14)
    np.testing.assert_allclose(theta.detach().numpy(), tt, atol=1e-14)
    (torch.sigmoid(W) @ torch.tensor(g[0]) + alpha @ torch.tensor(g[1]) + theta @ torch.tensor(g[2])).backward()
    for x, t in zip(got, (W, A, Th)):
        np.testing.assert_allclose(x, t.grad.numpy(), atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_unrolled_grad_from_state_matches_autograd(orc, seed):
    p = tiny(seed + 700, n=9, m=6, kmax=6)
    om, ah = learned_params(p, seed + 1)
    al = orc.softmax_alpha(p, ah)
    lam0, M0 = orc.run(p, om, al, 2)
    lam0 = orc.nonparam_update(p, lam0, np.random.default_rng(seed).normal(size=p.nnz))
    T = 2
    lb, dw, da, (dl0, dm0) = orc.unrolled_grad(p, om, al, T, lam0=lam0, M0=M0)
    W = torch.tensor(om, requires_grad=True)
    A = torch.tensor(al, requires_grad=True)
    L0 = torch.tensor(lam0, requires_grad=True)
    M0t = torch.tensor(M0, requires_grad=True)
    lbt, _ = brute.dmma_torch(p, W, A, T, lam0=L0, M0=M0t)
    lbt.backward()
    assert lb == pytest.approx(lbt.item(), abs=1e-11)
    for x, t in ((dw, W), (da, A), (dl0, L0), (dm0, M0t)):
        np.testing.assert_allclose(x, t.grad.numpy(), atol=1e-10)


def test_unrolled_grad_from_state_euler_identity(orc):
    p = synth.workload("gm", small=True)["problem"]
    om, ah = learned_params(p, 54)
    al = orc.softmax_alpha(p, ah)
    lam0, M0 = orc.run(p, om, al, 3)
    lb, _, _, (dl0, dm0) = orc.unrolled_grad(p, om, al, 4, lam0=lam0, M0=M0)
    unc = np.bincount(p.col, minlength=p.n) == 0
    const = np.minimum(p.c[unc], 0.0).sum()
    terms = np.concatenate([dl0 * lam0, dm0 * M0])
    assert terms.sum() == pytest.approx(lb - const, abs=1e-10 * np.abs(terms).sum())


# ------------------------------------------------------------------------------------------
# Smoothed subproblems (feature table of the appendix), read as a soft-min: Gibbs marginals
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("tau", [0.3, 1.0, 10.0])
def test_smoothed_matches_enumeration(orc, tau):
    p = tiny(81, n=12, m=8, kmax=7)
    lam = np.random.default_rng(82).normal(size=p.nnz)
    E, pm = orc.smoothed(p, lam, tau)
    for j, X in enumerate(brute.row_sets(p)):
        a, b = int(p.row_ptr[j]), int(p.row_ptr[j + 1])
        cost = X @ lam[a:b]
        w = np.exp(-(cost - cost.min()) / tau)
        assert E[j] == pytest.approx(cost.min() - tau * np.log(w.sum()), abs=1e-12)
        np.testing.assert_allclose(pm[a:b], (w[:, None] * X).sum(0) / w.sum(), atol=1e-12)


def test_smoothed_limits_and_gradient(orc):
    p = tiny(83, n=12, m=8, kmax=7)
    lam = np.random.default_rng(84).normal(size=p.nnz)
    Ej = orc.energies(p, lam)
    x = orc.argmin(p, lam)
    E, pm = orc.smoothed(p, lam, 1e-4)
    np.testing.assert_allclose(E, Ej, atol=1e-3)           # tau -> 0: the subproblem minimum
    np.testing.assert_allclose(pm, x, atol=1e-6)            # and the minimizing assignment
    for tau in (0.5, 5.0):
        E, pm = orc.smoothed(p, lam, tau)
        sizes = np.array([len(X) for X in brute.row_sets(p)])
        assert (E <= Ej + 1e-12).all() and (E >= Ej - tau * np.log(sizes) - 1e-12).all()
        h = 1e-6
        for e in range(0, p.nnz, 3):   # central differences of E_tau
            lp, lm = lam.copy(), lam.copy()
            lp[e] += h
            lm[e] -= h
            j = int(np.searchsorted(p.row_ptr, e, side="right") - 1)
            d = (orc.smoothed(p, lp, tau)[0][j] - orc.smoothed(p, lm, tau)[0][j]) / (2 * h)
            assert d == pytest.approx(pm[e], abs=1e-6)
