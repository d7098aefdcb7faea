"""Graphs of up to 126 vertices (two-word states): tw_decide128 / tw_solve128.

* Up to 64 vertices: every level of the two-word search equals the one-word
  search's and the oracle's (same graphs, same bounds), element by element.
* Beyond 64 vertices (randomly relabelled, so states straddle bit 64): every
  level equals the wide oracle's (plain Python sets of any width, §2 and
  Listing 1), treewidths equal the closed forms (paths 1, ladders and
  triangulated ladders 2, a cycle has no bound-1 order), and orders have
  exactly that width by fill-in.
* n = 127 is rejected.
"""
import random

import numpy as np
import pytest

from oracle import wide as W
from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu


def _relabel(rows, seed):
    n = len(rows)
    perm = list(range(n))
    random.Random(seed).shuffle(perm)
    out = [0] * n
    for i, r in enumerate(rows):
        for j in range(n):
            if (r >> j) & 1:
                out[perm[i]] |= 1 << perm[j]
    return out


def _path(n):
    return W.rows_from_edges(n, [(i, i + 1) for i in range(n - 1)])


def _cycle(n):
    return W.rows_from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def _ladder(m, diagonals=False):
    e = [(c, c + 1) for c in range(m - 1)] + [(m + c, m + c + 1) for c in range(m - 1)]
    e += [(c, m + c) for c in range(m)]
    if diagonals:
        e += [(c, m + c + 1) for c in range(m - 1)]
    return W.rows_from_edges(2 * m, e)


def _as_ints(states):
    return sorted(int(lo) | (int(hi) << 64) for lo, hi in states)


def test_wide_levels_equal_narrow_up_to_64(oracle):
    """G(24, 0.25), G(28, 0.2), a ladder on 64 vertices and a triangulated
    ladder on 60, at tw - 1 and tw: level by level the same sets (sorted low
    words, high words zero), pair counts and answers as the one-word search."""
    from paper_1709_09990_amd import tw as T
    cases = [G.gnp(24, 0.25, 71001), G.gnp(28, 0.2, 53001),
             np.array(_relabel(_ladder(32), 5), dtype=np.uint64),
             np.array(_relabel(_ladder(30, True), 6), dtype=np.uint64)]
    with T.Context(device=0) as c:
        for rows in cases:
            tw = oracle.treewidth_bfs(rows, oracle.mmw(rows))
            for k in (tw - 1, tw):
                print(f"wide vs narrow n={len(rows)} k={k}", flush=True)
                yes_w, lw = c.trace_decide128([int(r) for r in rows], k)
                yes_n, ln = c.trace_decide(rows, k)
                assert yes_w == yes_n == (k >= tw)
                assert len(lw) == len(ln)
                for (lv, cnt, exp, succ, states), nar in zip(lw, ln):
                    assert lv == nar.level and cnt == nar.count
                    assert exp == nar.expansions and succ == nar.successors
                    assert not states[:, 1].any()
                    assert np.array_equal(np.sort(states[:, 0]), np.sort(nar.states))
            got, order, _ = c.solve128([int(r) for r in rows])
            assert got == tw
            assert oracle.order_width(rows, order) == tw


WIDE_CASES = [
    ("path100", _path(100), 1, True),
    ("path100_k0", _path(100), 0, False),
    ("path126", _path(126), 1, True),
    ("cycle70_k1", _cycle(70), 1, False),
    ("ladder35", _ladder(35), 2, True),
    ("ladder35_k1", _ladder(35), 1, False),
    ("tri_ladder40", _ladder(40, True), 2, True),
]


@pytest.mark.parametrize("name,rows,k,yes", WIDE_CASES, ids=[c[0] for c in WIDE_CASES])
def test_wide_levels_equal_oracle(name, rows, k, yes):
    from paper_1709_09990_amd import tw as T
    g = _relabel(rows, 11)
    want_yes, want = W.decide(g, k)
    assert want_yes == yes
    with T.Context(device=0) as c:
        got_yes, levels = c.trace_decide128(g, k)
        y2, st = c.decide128(g, k)
    assert got_yes == y2 == yes
    assert len(levels) == len(want)
    for (lv, cnt, _, _, states), ref in zip(levels, want):
        assert cnt == len(ref)
        assert _as_ints(states) == ref, (name, lv)
    assert st["unique"] == sum(len(x) for x in want[1:])


@pytest.mark.parametrize("name,rows,tw", [("path90", _path(90), 1), ("path126", _path(126), 1),
                                           ("ladder35", _ladder(35), 2), ("tri_ladder45", _ladder(45, True), 2)])
def test_wide_solve_closed_forms(name, rows, tw):
    from paper_1709_09990_amd import tw as T
    g = _relabel(rows, 13)
    with T.Context(device=0) as c:
        got, order, st = c.solve128(g)
    assert got == tw
    assert W.order_width(g, [int(v) for v in order]) == tw
    assert sorted(int(v) for v in order) == list(range(len(g)))


def test_wide_rejects_127():
    from paper_1709_09990_amd import tw as T
    with T.Context(device=0) as c:
        with pytest.raises(T.TwError) as e:
            c.decide128(_path(127), 1)
        assert e.value.status == T.TW_EINVAL
