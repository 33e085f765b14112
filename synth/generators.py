"""Seeded synthetic binary programs shaped like the paper's workloads.

This module only builds inputs: constraint rows, costs and the per-edge
parameters omega and alpha-hat.  It holds none of the solver's arithmetic and
is shared by the FP64 oracle tests and by the GPU path.

A binary program (Def. 1, Sec. "Lagrange Decomposition") is stored as linear
rows with integer coefficients, one subproblem per row:

    row j:  sum_{p in row_ptr[j]..row_ptr[j+1]} coef[p] * x[col[p]]  (sense[j])  rhs[j]

with sense -1 for <=, 0 for ==, +1 for >=.  Columns are sorted ascending in
each row, so the edge order (row-major, variable ascending) is the canonical
order of every per-edge array (omega, alpha-hat, lambda, M).

The paper's own datasets (cell tracking, graph matching, independent set,
QAPLib) are not available; the generators below stand in for them with the
shapes stated in each docstring.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np


@dataclasses.dataclass
class Problem:
    n: int
    c: np.ndarray          # float64 [n]
    row_ptr: np.ndarray    # int64 [m+1]
    col: np.ndarray        # int32 [nnz], ascending within each row
    coef: np.ndarray       # int32 [nnz]
    sense: np.ndarray      # int8 [m]  (-1: <=, 0: ==, +1: >=)
    rhs: np.ndarray        # int64 [m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row(self, j):
        a, b = int(self.row_ptr[j]), int(self.row_ptr[j + 1])
        return self.col[a:b], self.coef[a:b], int(self.sense[j]), int(self.rhs[j])

    def edge_var(self) -> np.ndarray:
        return self.col.astype(np.int64)

    def edge_row(self) -> np.ndarray:
        return np.repeat(np.arange(self.m, dtype=np.int64), np.diff(self.row_ptr))

    def degree(self) -> np.ndarray:
        """|J_i|: number of rows containing each variable."""
        return np.bincount(self.col, minlength=self.n).astype(np.int64)

    def subset_rows(self, rows) -> "Problem":
        """Standalone sub-instance made of the given rows (variables keep their ids)."""
        rows = np.asarray(rows, dtype=np.int64)
        lens = np.diff(self.row_ptr)[rows]
        ptr = np.zeros(len(rows) + 1, dtype=np.int64)
        ptr[1:] = np.cumsum(lens)
        idx = np.concatenate([np.arange(self.row_ptr[r], self.row_ptr[r + 1]) for r in rows]) \
            if len(rows) else np.zeros(0, dtype=np.int64)
        return Problem(self.n, self.c.copy(), ptr, self.col[idx].copy(), self.coef[idx].copy(),
                       self.sense[rows].copy(), self.rhs[rows].copy(), self.name + "-sub")


def row_cluster(prob, seed_row, k):
    """k rows coupled through shared variables, grown greedily from seed_row: each step adds the row
    that shares the most variables with the rows taken so far (ties: lowest row id).  Returned in
    ascending order.  A sub-instance built this way keeps much of its variables' coupling, unlike
    k rows drawn at random from a large program, which share almost no variable."""
    var_rows = {}
    for j in range(prob.m):
        for v in prob.col[prob.row_ptr[j]:prob.row_ptr[j + 1]]:
            var_rows.setdefault(int(v), []).append(j)
    taken = {int(seed_row)}
    score = {}
    frontier = [int(seed_row)]
    while len(taken) < k:
        for j in frontier:
            for v in prob.col[prob.row_ptr[j]:prob.row_ptr[j + 1]]:
                for r in var_rows[int(v)]:
                    if r not in taken:
                        score[r] = score.get(r, 0) + 1
        if not score:
            break
        best = min(score, key=lambda r: (-score[r], r))
        del score[best]
        taken.add(best)
        frontier = [best]
    return np.sort(np.array(sorted(taken), dtype=np.int64))


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def _from_rows(n, c, rows, name):
    """rows: list of (cols, coefs, sense, rhs); sorts columns within each row."""
    lens = np.array([len(r[0]) for r in rows], dtype=np.int64)
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(lens)
    col = np.empty(ptr[-1], dtype=np.int32)
    coef = np.empty(ptr[-1], dtype=np.int32)
    for j, (cc, aa, _, _) in enumerate(rows):
        o = np.argsort(cc, kind="stable")
        col[ptr[j]:ptr[j + 1]] = np.asarray(cc)[o]
        coef[ptr[j]:ptr[j + 1]] = np.asarray(aa)[o]
    sense = np.array([r[2] for r in rows], dtype=np.int8)
    rhs = np.array([r[3] for r in rows], dtype=np.int64)
    return Problem(n, np.asarray(c, dtype=np.float64), ptr, col, coef, sense, rhs, name)


def _csr_from_sorted_blocks(cols_flat, coefs_flat, lens):
    ptr = np.zeros(len(lens) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(lens)
    rid = np.repeat(np.arange(len(lens)), lens)
    o = np.lexsort((cols_flat, rid))
    return ptr, cols_flat[o].astype(np.int32), coefs_flat[o].astype(np.int32)


def _distinct_rows(rng, n, lens):
    """Per row, len distinct variables drawn uniformly from [0, n) (without replacement).

    Draws iid, then redraws only the repeated entries until none is left; the
    procedure is symmetric in the labels, so every subset is equally likely.
    """
    rid = np.repeat(np.arange(len(lens)), lens)
    cols = rng.integers(0, n, size=int(lens.sum()))
    while True:
        o = np.lexsort((cols, rid))
        cs, rs = cols[o], rid[o]
        dup = np.zeros(cs.size, dtype=bool)
        dup[1:] = (cs[1:] == cs[:-1]) & (rs[1:] == rs[:-1])
        if not dup.any():
            return cs, rs
        cols, rid = cs, rs
        cols[dup] = rng.integers(0, n, size=int(dup.sum()))


# ----------------------------------------------------------------------------------------------
# Workload generators
# ----------------------------------------------------------------------------------------------

def set_cover(n=1000, m=500, seed=1000, kmin=4, kmax=10, rng=None):
    """Set cover: rows sum_{i in S_j} x_i >= 1, |S_j| ~ U{kmin..kmax}, c ~ U[0,1]."""
    rng = rng if rng is not None else np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, size=n)
    lens = rng.integers(kmin, kmax + 1, size=m)
    cols, _ = _distinct_rows(rng, n, lens)
    ptr = np.zeros(m + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(lens)
    coef = np.ones(ptr[-1], dtype=np.int32)
    return Problem(n, c, ptr, cols.astype(np.int32), coef, np.full(m, 1, np.int8),
                   np.ones(m, np.int64), f"setcover-n{n}-m{m}")


def independent_set(n=50000, M=100000, seed=1001, rng=None):
    """Weighted independent set on G(n, M): rows x_u + x_v <= 1 per edge, c = -U[0,1]."""
    rng = rng if rng is not None else np.random.default_rng(seed)
    c = -rng.uniform(0.0, 1.0, size=n)
    have = np.zeros(0, dtype=np.int64)
    while have.size < M:
        k = int((M - have.size) * 1.2) + 16
        u = rng.integers(0, n, size=k)
        v = rng.integers(0, n, size=k)
        keep = u != v
        lo, hi = np.minimum(u, v)[keep], np.maximum(u, v)[keep]
        key = lo.astype(np.int64) * n + hi
        # keep first occurrences in draw order so the result is independent of np.unique's sort
        allk = np.concatenate([have, key])
        _, first = np.unique(allk, return_index=True)
        have = allk[np.sort(first)]
    key = have[:M]
    lo, hi = key // n, key % n
    ptr = np.arange(0, 2 * M + 1, 2, dtype=np.int64)
    col = np.stack([lo, hi], axis=1).reshape(-1).astype(np.int32)
    coef = np.ones(2 * M, dtype=np.int32)
    return Problem(n, c, ptr, col, coef, np.full(M, -1, np.int8), np.ones(M, np.int64),
                   f"indset-n{n}-M{M}")


def graph_matching(n_left=2000, n_right=2000, cand=10, n_pairs=200000, seed=1002, rng=None):
    """Graph-matching-shaped program.

    Assignment variables x_{l,t} (id l*cand+t) choose candidate t of left node l;
    uniqueness rows sum <= 1 per left node and per right node with >= 2 candidates;
    pairwise variables y (ids after the x block) with rows x_a - y >= 0,
    x_b - y >= 0 and x_a + x_b - y <= 1 for distinct compatible pairs (a, b)
    (different left and different right node).  Costs: c_x ~ N(0,1), c_y = -U[0,1].
    """
    rng = rng if rng is not None else np.random.default_rng(seed)
    nx = n_left * cand
    right = np.stack([rng.choice(n_right, size=cand, replace=False) for _ in range(n_left)])
    rflat = right.reshape(-1)
    lflat = np.repeat(np.arange(n_left), cand)
    have = np.zeros(0, dtype=np.int64)
    while have.size < n_pairs:
        k = int((n_pairs - have.size) * 1.3) + 16
        a = rng.integers(0, nx, size=k)
        b = rng.integers(0, nx, size=k)
        ok = (lflat[a] != lflat[b]) & (rflat[a] != rflat[b])
        lo, hi = np.minimum(a, b)[ok], np.maximum(a, b)[ok]
        key = lo.astype(np.int64) * nx + hi
        allk = np.concatenate([have, key])
        _, first = np.unique(allk, return_index=True)
        have = allk[np.sort(first)]
    key = have[:n_pairs]
    pa, pb = key // nx, key % nx
    n = nx + n_pairs
    c = np.concatenate([rng.normal(0.0, 1.0, size=nx), -rng.uniform(0.0, 1.0, size=n_pairs)])
    rows = []
    for l in range(n_left):
        ids = np.arange(l * cand, (l + 1) * cand)
        rows.append((ids, np.ones(cand, np.int32), -1, 1))
    by_r = [[] for _ in range(n_right)]
    for xid, r in enumerate(rflat):
        by_r[r].append(xid)
    for r in range(n_right):
        if len(by_r[r]) >= 2:
            rows.append((np.array(by_r[r]), np.ones(len(by_r[r]), np.int32), -1, 1))
    # pairwise rows, vectorised
    y = nx + np.arange(n_pairs)
    lens_u = np.array([len(r[0]) for r in rows], dtype=np.int64)
    ucol = np.concatenate([r[0] for r in rows]).astype(np.int64)
    ucoef = np.ones(ucol.size, np.int64)
    pcol = np.concatenate([np.stack([pa, y], 1), np.stack([pb, y], 1)], 0).reshape(-1)
    pcoef = np.tile(np.array([1, -1], np.int64), 2 * n_pairs)
    tcol = np.stack([pa, pb, y], 1).reshape(-1)
    tcoef = np.tile(np.array([1, 1, -1], np.int64), n_pairs)
    # row order: uniqueness rows, then for each pair p: (x_a - y >= 0), (x_b - y >= 0), (x_a + x_b - y <= 1)
    pr_ptr = np.zeros(3 * n_pairs + 1, np.int64)
    plen = np.tile(np.array([2, 2, 3], np.int64), n_pairs)
    pr_ptr[1:] = np.cumsum(plen)
    two = pcol.reshape(2, n_pairs, 2)
    twoc = pcoef.reshape(2, n_pairs, 2)
    three = tcol.reshape(n_pairs, 3)
    threec = tcoef.reshape(n_pairs, 3)
    pc = np.concatenate([two[0], two[1], three], axis=1).reshape(-1)        # per pair 7 entries
    pk = np.concatenate([twoc[0], twoc[1], threec], axis=1).reshape(-1)
    lens = np.concatenate([lens_u, plen])
    cols = np.concatenate([ucol, pc])
    coefs = np.concatenate([ucoef, pk])
    ptr, col, coef = _csr_from_sorted_blocks(cols, coefs, lens)
    sense = np.concatenate([np.full(len(rows), -1, np.int8),
                            np.tile(np.array([1, 1, -1], np.int8), n_pairs)])
    rhs = np.concatenate([np.ones(len(rows), np.int64), np.tile(np.array([0, 0, 1], np.int64), n_pairs)])
    return Problem(n, c, ptr, col, coef, sense, rhs, f"gm-{n_left}x{cand}-p{n_pairs}")


def knapsack(n=2_000_000, m=40_000, kmin=50, kmax=200, amax=20, frac=0.4, seed=1004, rng=None):
    """Knapsack rows sum a_i x_i <= floor(frac * sum a_i), a_i ~ U{1..amax}, |row| ~ U{kmin..kmax}, c = -U[0,1]."""
    rng = rng if rng is not None else np.random.default_rng(seed)
    c = -rng.uniform(0.0, 1.0, size=n)
    lens = rng.integers(kmin, kmax + 1, size=m)
    cols, rid = _distinct_rows(rng, n, lens)
    a = rng.integers(1, amax + 1, size=cols.size)
    ptr = np.zeros(m + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(lens)
    sums = np.add.reduceat(a, ptr[:-1]) if m else np.zeros(0, np.int64)
    rhs = np.floor(frac * sums).astype(np.int64)
    return Problem(n, c, ptr, cols.astype(np.int32), a.astype(np.int32), np.full(m, -1, np.int8), rhs,
                   f"knapsack-n{n}-m{m}")


def batch_instances(count=64, seed0=2000, nmin=1e3, nmax=2e5, scale=1.0):
    """Uneven batch: n_k = round(exp(U[ln nmin, ln nmax])) * scale; even k set cover (m=n/2), odd k independent set (M=2n)."""
    out = []
    for k in range(count):
        rng = np.random.default_rng(seed0 + k)
        nk = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax))) * scale))
        nk = max(nk, 16)
        if k % 2 == 0:
            out.append(set_cover(n=nk, m=max(nk // 2, 1), rng=rng))
        else:
            out.append(independent_set(n=nk, M=2 * nk, rng=rng))
    return out


def _enumerate_row(coefs, sense, rhs):
    L = len(coefs)
    xs = np.array(list(itertools.product((0, 1), repeat=L)), dtype=np.int64)
    s = xs @ np.asarray(coefs, dtype=np.int64)
    ok = (s <= rhs) if sense < 0 else (s >= rhs) if sense > 0 else (s == rhs)
    return xs[ok]


def random_tiny(seed, n=8, m=4, kmin=1, kmax=5, amin=-5, amax=5, senses=(-1, 0, 1), cover_all=False):
    """Tiny random binary program for brute-force pins.

    Rows have integer coefficients in [amin, amax] (non-zero), any sense, and are
    redrawn until the feasible set is non-empty and no variable of the row is
    fixed by it (each variable takes both values somewhere in X_j).
    """
    rng = np.random.default_rng(seed)
    rows = []
    while len(rows) < m:
        k = int(rng.integers(kmin, kmax + 1))
        cols = rng.choice(n, size=min(k, n), replace=False)
        coefs = rng.integers(amin, amax + 1, size=cols.size)
        coefs[coefs == 0] = 1
        sense = int(rng.choice(senses))
        lo, hi = int(np.minimum(coefs, 0).sum()), int(np.maximum(coefs, 0).sum())
        rhs = int(rng.integers(lo, hi + 1))
        X = _enumerate_row(coefs, sense, rhs)
        if X.shape[0] == 0 or not np.all(X.min(0) == 0) or not np.all(X.max(0) == 1):
            continue
        rows.append((cols, coefs, sense, rhs))
    if cover_all:
        covered = set(np.concatenate([r[0] for r in rows]).tolist())
        for i in range(n):
            if i not in covered:
                j = int(rng.integers(0, len(rows)))
                # a loose <= row over one more variable keeps every variable free
                rows.append((np.array([i, rows[j][0][0]]), np.array([1, 1]), -1, 2))
    c = rng.normal(0.0, 1.0, size=n)
    return _from_rows(n, c, rows, f"tiny-{seed}")


# ----------------------------------------------------------------------------------------------
# Named workloads (per-edge parameters included)
# ----------------------------------------------------------------------------------------------

WORKLOADS = ("setcover", "indset", "gm", "batch", "knapsack")


def _params(prob, omega_kind, rng):
    E = prob.nnz
    if omega_kind == "half":
        return np.full(E, 0.5), np.zeros(E)
    # learned-style: omega = sigmoid(z), z ~ N(0,1); alpha logits ~ N(0, 0.1)
    omega = sigmoid(rng.normal(0.0, 1.0, size=E))
    ahat = rng.normal(0.0, 0.1, size=E)
    return omega, ahat


def workload(name, small=False):
    """Return dict(problem(s), omega, alpha_hat, T, ...) for a named workload.

    setcover : 1,000 vars, 500 rows sum x >= 1, omega 0.5, alpha uniform, T=200
    indset   : G(50,000, 100,000), omega 0.5, alpha uniform, T=1000
    gm       : graph-matching-shaped, learned-style omega / alpha logits, T=20, checkpoint 5
    batch    : 64 uneven set-cover / independent-set instances, T=500
    knapsack : 2,000,000 vars, 40,000 rows of 50-200 vars, learned-style params, T=10
    small=True shrinks every workload for quick tests (same generators).
    """
    if name == "setcover":
        p = set_cover(seed=1000)
        om, ah = _params(p, "half", None)
        return dict(problem=p, omega=om, alpha_hat=ah, T=200, ckpt=0)
    if name == "indset":
        p = independent_set(n=5000 if small else 50000, M=10000 if small else 100000, seed=1001)
        om, ah = _params(p, "half", None)
        return dict(problem=p, omega=om, alpha_hat=ah, T=1000, ckpt=0)
    if name == "gm":
        if small:
            p = graph_matching(n_left=50, n_right=50, cand=5, n_pairs=400, seed=1002)
        else:
            p = graph_matching(seed=1002)
        rng = np.random.default_rng(3002)
        om, ah = _params(p, "learned", rng)
        return dict(problem=p, omega=om, alpha_hat=ah, T=20, ckpt=5)
    if name == "batch":
        ps = batch_instances(count=8 if small else 64, nmax=2e4 if small else 2e5)
        params = [_params(p, "half", None) for p in ps]
        return dict(problems=ps, omega=[q[0] for q in params], alpha_hat=[q[1] for q in params], T=500, ckpt=0)
    if name == "knapsack":
        if small:
            p = knapsack(n=20000, m=400, seed=1004)
        else:
            p = knapsack(seed=1004)
        rng = np.random.default_rng(3004)
        om, ah = _params(p, "learned", rng)
        return dict(problem=p, omega=om, alpha_hat=ah, T=10, ckpt=5)
    raise ValueError(f"unknown workload {name!r}")
