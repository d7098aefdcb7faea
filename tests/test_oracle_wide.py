"""Pins of the wide-state oracle (graphs of more than 64 vertices).  CPU only.

* Up to 64 vertices its levels equal the C oracle's (two independent codes of
  the same definition).
* Beyond 64 vertices: closed forms (paths have treewidth 1, ladders 2, the
  triangulated ladder 2, a cycle has no bound-1 elimination), every YES gives
  an order whose fill-in width is the bound, and level sizes do not change
  when the vertices are relabelled across the 64-bit boundary.
* A planted 64-bit truncation (edges to vertices >= 64 dropped) changes an
  answer, so the pins see that mistake.
"""
from __future__ import annotations

import random

import numpy as np

from oracle import wide as W
from paper_1709_09990_amd import graphs as G


def _path(n):
    return W.rows_from_edges(n, [(i, i + 1) for i in range(n - 1)])


def _cycle(n):
    return W.rows_from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def _ladder(m, diagonals=False):
    # vertices (r, c) -> r * m + c for rows r = 0, 1
    e = [(c, c + 1) for c in range(m - 1)] + [(m + c, m + c + 1) for c in range(m - 1)]
    e += [(c, m + c) for c in range(m)]
    if diagonals:
        e += [(c, m + c + 1) for c in range(m - 1)]
    return W.rows_from_edges(2 * m, e)


def _relabel(rows, perm):
    n = len(rows)
    out = [0] * n
    for u in range(n):
        for w in range(n):
            if (rows[u] >> w) & 1:
                out[perm[u]] |= 1 << perm[w]
    return out


def test_wide_levels_equal_c_oracle(oracle):
    rng = random.Random(12)
    for t in range(14):
        n = rng.randint(6, 13)
        a = G.gnp(n, rng.uniform(0.15, 0.5), 9400 + t)
        rows = [int(x) for x in a]
        tw, _ = oracle.subset_dp(a)
        for k in range(0, min(n, tw + 2)):
            yes_w, lv_w = W.decide(rows, k)
            yes_c, lv_c, _ = oracle.decide(a, k)
            assert yes_w == yes_c == (tw <= k)
            for i, f in enumerate(lv_w):
                assert np.array_equal(np.array(f, dtype=np.uint64), lv_c[i]), (t, k, i)


def test_beyond_64_vertices_closed_forms():
    for rows, tw in ((_path(100), 1), (_ladder(40), 2), (_ladder(45, diagonals=True), 2)):
        assert len(rows) > 64
        assert W.decide(rows, tw - 1)[0] is False
        yes, levels = W.decide(rows, tw)
        assert yes
        order = W.order_from_levels(rows, tw, levels)
        assert sorted(order) == list(range(len(rows)))
        assert W.order_width(rows, order) == tw
    assert W.decide(_cycle(70), 1)[0] is False
    assert W.order_width(_cycle(70), list(range(70))) == 2


def test_relabelling_across_the_word_boundary():
    rng = random.Random(13)
    rows = _ladder(36)  # 72 vertices
    _, base = W.decide(rows, 2)
    for _ in range(3):
        perm = list(range(72))
        rng.shuffle(perm)
        _, lv = W.decide(_relabel(rows, perm), 2)
        assert [len(f) for f in lv] == [len(f) for f in base]


def test_planted_64bit_truncation_is_caught():
    rng = random.Random(14)
    rows = _ladder(36)
    perm = list(range(72))
    rng.shuffle(perm)
    r = _relabel(rows, perm)
    truncated = [x & (2**64 - 1) for x in r]
    # the truncated graph loses edges and is no longer symmetric: its levels differ
    _, good = W.decide(r, 1)
    _, bad = W.decide(truncated, 1)
    assert [len(f) for f in good] != [len(f) for f in bad]
