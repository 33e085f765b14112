"""Host-side checks of the library (no GPU): exports, decision-diagram compiler, input validation."""
import itertools
import os
import re

import numpy as np
import pytest

import synth
from tests import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dd():
    import paper_2205_11638_amd as pkg
    pkg.lib()
    return pkg


def test_every_declared_symbol_is_exported(dd):
    import ctypes
    decl = set()
    for name in os.listdir(os.path.join(ROOT, "include")):
        if name.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", name)).read()
            decl |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dd_\w+)\s*\(", txt, re.M))
    assert len(decl) >= 15
    L = ctypes.CDLL(dd.binding.LIB_PATH)
    for s in sorted(decl):
        assert hasattr(L, s), s
    assert decl <= set(dd.binding.SIGNATURES), decl - set(dd.binding.SIGNATURES)


def _paths(width, arcs):
    """All root-to-1 assignments of a compiled diagram."""
    L = len(width)
    starts = np.concatenate([[0], np.cumsum(width)])
    out = []

    def walk(l, k, x):
        code = int(arcs[starts[l] + k])
        Wn = int(width[l + 1]) if l + 1 < L else 0
        for beta, c in ((0, code & 0xFFFF), (1, code >> 16)):
            if c == Wn:
                continue                    # 0-terminal
            if c == Wn + 1:
                assert l == L - 1           # 1-terminal only below the last level
                out.append(tuple(x + [beta]))
                continue
            assert c < Wn
            walk(l + 1, c, x + [beta])

    walk(0, 0, [])
    return sorted(out)


@pytest.mark.parametrize("seed", range(40))
def test_compiled_paths_are_exactly_the_feasible_set(dd, seed):
    p = synth.random_tiny(seed, n=10, m=3, kmin=1, kmax=9, amin=-6, amax=6)
    for j in range(p.m):
        width, arcs = dd.compile_row(p, j)
        cols, coefs, sense, rhs = p.row(j)
        X = brute.feasible_set(coefs, sense, rhs)
        assert _paths(width, arcs) == sorted(map(tuple, X.tolist()))
        # quasi-reduced: one root, no two nodes of a level with the same children, no dead node
        assert width[0] == 1
        start = 0
        for l, w in enumerate(width):
            lvl = arcs[start:start + w]
            assert len(set(lvl.tolist())) == w
            Wn = width[l + 1] if l + 1 < len(width) else 0
            assert not np.any(((lvl & 0xFFFF) == Wn) & ((lvl >> 16) == Wn))
            start += w


def test_known_shapes(dd):
    p = synth.set_cover(n=30, m=5, seed=3)
    for j in range(p.m):
        w, a = dd.compile_row(p, j)
        L = len(w)
        assert list(w) == [1] + [2] * (L - 1)        # "no 1 yet" / "covered"
    q = synth.independent_set(n=20, M=10, seed=1)
    for j in range(q.m):
        w, a = dd.compile_row(q, j)
        assert list(w) == [1, 2]
    k = synth.knapsack(n=1000, m=3, seed=5)
    for j in range(k.m):
        w, a = dd.compile_row(k, j)
        cols, coefs, sense, rhs = k.row(j)
        assert max(w) <= rhs + 2                      # states are partial sums 0..b plus "always feasible"


@pytest.mark.parametrize("seed", range(12))
def test_child_codes_are_monotone_in_partial_sum_order(dd, seed):
    """Nodes of a level are numbered in increasing partial sum (the always-true node of a <= row
    first), so on <= rows -- with coefficients of both signs -- each level's lo and hi child codes are
    non-decreasing in the node number, the 0-terminal (code = next width) after every node; on the
    last level the codes (0 = 0-terminal, 1 = 1-terminal) are non-increasing.  The one-wave passes
    read the steps of these codes in one nibble each (4-byte codes where a step does not fit)."""
    rng = np.random.default_rng(seed)
    rows, n = [], 60
    for _ in range(6):
        k = int(rng.integers(3, 40))
        a = rng.integers(-8 if seed % 3 == 0 else 1, 21, size=k)
        a[a == 0] = 1
        lo, hi = int(np.minimum(a, 0).sum()), int(np.maximum(a, 0).sum())
        rows.append((rng.choice(n, size=k, replace=False), a, -1, int(rng.integers(lo + (hi - lo) // 4, hi - (hi - lo) // 4 + 1))))
    p = synth.generators._from_rows(n, np.zeros(n), rows, "le-rows")
    steps = 0
    for j in range(p.m):
        try:
            width, arcs = dd.compile_row(p, j)
        except Exception:
            continue  # a forcing or infeasible draw
        start = 0
        for l, w in enumerate(width):
            lvl = arcs[start:start + w].astype(np.int64)
            start += w
            last = l + 1 == len(width)
            for c in (lvl & 0xFFFF, lvl >> 16):
                d = np.diff(-c if last else c)
                assert np.all(d >= 0), (j, l)
                steps += d.size
    assert steps > 0


def _one_row(coefs, sense, rhs, n=None):
    n = n or len(coefs)
    return synth.generators._from_rows(n, np.zeros(n), [(np.arange(len(coefs)), np.array(coefs), sense, rhs)], "r")


def test_errors(dd):
    with pytest.raises(dd.DDError) as e:
        dd.compile_row(_one_row([1, 1], -1, -1), 0)
    assert e.value.code == dd.binding.DD_E_INFEASIBLE
    with pytest.raises(dd.DDError) as e:
        dd.compile_row(_one_row([1, 1], 1, 2), 0)          # x0 + x1 >= 2 fixes both
    assert e.value.code == dd.binding.DD_E_FORCED
    with pytest.raises(dd.DDError) as e:
        dd.compile_row(_one_row([1, 1, 1], 0, 3), 0)
    assert e.value.code == dd.binding.DD_E_FORCED
    bad = _one_row([1, 1], -1, 1)
    bad.col[1] = 0                                         # duplicate variable
    with pytest.raises(dd.DDError) as e:
        dd.compile_row(bad, 0)
    assert e.value.code == dd.binding.DD_E_ARG
    oob = _one_row([1, 1], -1, 1)
    oob.col[1] = 7
    with pytest.raises(dd.DDError) as e:
        dd.compile_row(oob, 0)
    assert e.value.code == dd.binding.DD_E_ARG


def test_create_rejects_bad_input_before_touching_the_gpu(dd):
    p = _one_row([1, 1], -1, 1)
    p.c[0] = np.nan
    with pytest.raises(dd.DDError) as e:
        dd.Instance(p)
    assert e.value.code == dd.binding.DD_E_PARAM
    q = _one_row([1, 1], 1, 2)
    with pytest.raises(dd.DDError) as e:
        dd.Instance(q)
    assert e.value.code == dd.binding.DD_E_FORCED
    r = _one_row([1, 1], -1, 1)
    r.sense[0] = 3
    with pytest.raises(dd.DDError) as e:
        dd.Instance(r)
    assert e.value.code == dd.binding.DD_E_ARG


def test_unsorted_columns_are_sorted(dd):
    p = synth.generators._from_rows(4, np.zeros(4), [(np.array([0, 2, 3]), np.array([3, -2, 1]), -1, 1)], "u")
    w1, a1 = dd.compile_row(p, 0)
    p.col[:] = p.col[::-1].copy()
    p.coef[:] = p.coef[::-1].copy()
    w2, a2 = dd.compile_row(p, 0)
    np.testing.assert_array_equal(w1, w2)
    np.testing.assert_array_equal(a1, a2)


def test_batch_needs_programs(dd):
    with pytest.raises(dd.DDError) as e:
        dd.Batch([])
    assert e.value.code == dd.binding.DD_E_ARG


def test_waves_per_block_limited_to_the_compiled_workgroup_size(dd):
    # the kernels are compiled for workgroups of at most 256 threads (4 waves)
    p = synth.random_tiny(2, n=10, m=5)
    with pytest.raises(dd.DDError) as e:
        dd.Instance(p, waves_per_block=8)
    assert e.value.code == dd.binding.DD_E_ARG


def test_gap_integral(dd):
    # hand-worked: d_init = 0, d* = 10; bounds 0, 5, 8, 10 at 0, 1000, 3000, 4000 ms
    g, gi = dd.gap_integral([0.0, 5.0, 8.0, 10.0], [0.0, 1000.0, 3000.0, 4000.0], 10.0)
    np.testing.assert_allclose(g, [1.0, 0.5, 0.2, 0.0])
    assert gi == pytest.approx(1.0 * 1 + 0.5 * 2 + 0.2 * 1)
    # a bound below the start is clipped to 1; d* not above the start gives 0
    g, _ = dd.gap_integral([1.0, -1.0], [0.0, 10.0], 3.0)
    np.testing.assert_allclose(g, [1.0, 1.0])
    g, gi = dd.gap_integral([1.0, 2.0], [0.0, 10.0], 1.0)
    np.testing.assert_allclose(g, [0.0, 0.0])
    assert gi == 0.0


def test_diagram_wider_than_the_kernels_is_rejected_at_create():
    """The widest one-wave class holds 64 rows of 64 nodes per level: a row whose diagram is wider
    fails at create with DD_E_UNSUPPORTED naming the row, before any device memory is touched."""
    import paper_2205_11638_amd as dd
    rng = np.random.default_rng(0)
    n = 2000
    cols = rng.choice(n, size=600, replace=False)
    a = rng.integers(1, 40, size=600)
    p = synth.generators._from_rows(n, -np.ones(n), [(cols, a, -1, int(0.4 * a.sum()))], "too-wide")
    w, _ = dd.binding.compile_row(p, 0)
    assert w.max() > 4096
    with pytest.raises(dd.DDError) as e:
        dd.Instance(p)
    assert e.value.code == dd.binding.DD_E_UNSUPPORTED and "row 0" in str(e.value) and "4096" in str(e.value)
