"""Brute-force reference for tiny instances: enumeration of every feasible set X_j.

Independent of both the FP64 oracle (which uses partial-sum dynamic programs)
and the GPU library (which uses reduced BDDs).  Alg. 1 of the paper is written
out directly with min-marginals taken over enumerated assignments; the torch
variant records the computation so autograd yields the exact (sub)gradient of
the unrolled solver -- a third way to get what Alg. 2 computes.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch


def feasible_set(coefs, sense, rhs):
    L = len(coefs)
    xs = np.array(list(itertools.product((0, 1), repeat=L)), dtype=np.int64).reshape(-1, L)
    s = xs @ np.asarray(coefs, dtype=np.int64)
    ok = (s <= rhs) if sense < 0 else (s >= rhs) if sense > 0 else (s == rhs)
    return xs[ok]


def row_sets(prob):
    return [feasible_set(prob.row(j)[1], prob.row(j)[2], prob.row(j)[3]) for j in range(prob.m)]


def min_marginals(prob, lam, sets=None):
    sets = sets or row_sets(prob)
    m0, m1 = np.empty(prob.nnz), np.empty(prob.nnz)
    for j, X in enumerate(sets):
        a, b = int(prob.row_ptr[j]), int(prob.row_ptr[j + 1])
        cost = X @ lam[a:b]
        for l in range(b - a):
            m0[a + l] = cost[X[:, l] == 0].min()
            m1[a + l] = cost[X[:, l] == 1].min()
    return m0, m1


def energies(prob, lam, sets=None):
    sets = sets or row_sets(prob)
    return np.array([(X @ lam[int(prob.row_ptr[j]):int(prob.row_ptr[j + 1])]).min() for j, X in enumerate(sets)])


def ilp_optimum(prob):
    """min <c, x> over x in {0,1}^n satisfying every row (n <= ~18)."""
    n = prob.n
    xs = np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.int64)
    ok = np.ones(xs.shape[0], dtype=bool)
    for j in range(prob.m):
        cols, coefs, sense, rhs = prob.row(j)
        s = xs[:, cols] @ coefs.astype(np.int64)
        ok &= (s <= rhs) if sense < 0 else (s >= rhs) if sense > 0 else (s == rhs)
    return float((xs[ok] @ prob.c).min()) if ok.any() else float("inf")


def dmma_torch(prob, omega, alpha, T, c=None, record=False, lam0=None, M0=None):
    """Alg. 1 with enumerated min-marginals, in torch float64 (differentiable).

    omega, alpha, c (and lam0, M0) may be tensors requiring grad.  Deferred sums are taken at
    the start of each pass; lambda starts at c_i/|J_i|, M at 0 unless a start state (lam0, M0)
    is given; forward passes visit the variables of each row in ascending order, backward
    passes in descending order.  Returns (LB at the flushed multipliers, list of states).
    """
    sets = [torch.tensor(X, dtype=torch.float64) for X in row_sets(prob)]
    E = prob.nnz
    var = torch.tensor(prob.col.astype(np.int64))
    deg = torch.bincount(var, minlength=prob.n).to(torch.float64)
    c = torch.as_tensor(prob.c, dtype=torch.float64) if c is None else c
    if lam0 is None:
        lam = c[var] / deg[var]
        M = torch.zeros(E, dtype=torch.float64)
    else:
        lam, M = lam0, M0
    states = [(lam.detach().clone(), M.detach().clone())]
    ptr = [int(v) for v in prob.row_ptr]
    for t in range(T):
        for direction in (0, 1):
            S = torch.zeros(prob.n, dtype=torch.float64).index_add(0, var, M)
            Se = S[var]
            lam_parts, M_parts = [], []
            for j, X in enumerate(sets):
                a, b = ptr[j], ptr[j + 1]
                lj = [lam[a + l] for l in range(b - a)]
                Mj = [None] * (b - a)
                order = range(b - a) if direction == 0 else range(b - a - 1, -1, -1)
                for l in order:
                    cost = X @ torch.stack(lj)
                    m1 = cost[X[:, l] == 1].min(dim=0).values
                    m0 = cost[X[:, l] == 0].min(dim=0).values
                    Mn = omega[a + l] * (m1 - m0)
                    lj[l] = lj[l] - Mn + alpha[a + l] * Se[a + l]
                    Mj[l] = Mn
                lam_parts.extend(lj)
                M_parts.extend(Mj)
            lam = torch.stack(lam_parts)
            M = torch.stack(M_parts)
            if record:
                states.append((lam.detach().clone(), M.detach().clone()))
    S = torch.zeros(prob.n, dtype=torch.float64).index_add(0, var, M)
    lbar = lam + alpha * S[var]
    lb = sum((X @ lbar[ptr[j]:ptr[j + 1]]).min(dim=0).values for j, X in enumerate(sets))
    unc = deg == 0
    lb = lb + torch.clamp(c[unc], max=0.0).sum()
    return lb, states


def lp_optimum(prob):
    """Optimum of the LP relaxation (rows as written, 0 <= x <= 1) with scipy's HiGHS.  For programs
    whose single rows are integral polytopes (set cover, independent set) this is the optimum of the
    Lagrange dual (D)."""
    import scipy.sparse as sp
    from scipy.optimize import linprog
    A = sp.csr_matrix((prob.coef.astype(float), prob.col, prob.row_ptr), shape=(prob.m, prob.n))
    le, ge, eq = prob.sense < 0, prob.sense > 0, prob.sense == 0
    A_ub = sp.vstack([A[le], -A[ge]]).tocsr()
    b_ub = np.concatenate([prob.rhs[le], -prob.rhs[ge]]).astype(float)
    kw = {"A_eq": A[eq], "b_eq": prob.rhs[eq].astype(float)} if eq.any() else {}
    res = linprog(prob.c, A_ub=A_ub, b_ub=b_ub, bounds=(0, 1), method="highs", **kw)
    assert res.status == 0, res.message
    return float(res.fun)
