"""Pins of O6, the per-state minor-min-width pruning (§3.3 applied to the
graph left after eliminating S).  CPU only.

* H_S equals the graph reached by eliminating the vertices of S one at a time
  with explicit fill-in, in any order (§2: the result does not depend on the
  order) — an independent route to every row.
* The C mmw equals the Python one (sets, written separately); MMW(H_S) equals
  the Python mmw of H_S relabelled in increasing order (tie-breaks by lowest
  index are unchanged by such a relabelling).
* Pruning is sound: every state of a plain level from which some order of the
  remaining vertices stays within width k (found by brute-force search over
  subsets) survives, answers equal the subset DP, and the pruned levels are
  subsets of the plain ones.  A planted slip (pruning at MMW >= k) drops a
  completable state on some graph.
"""
from __future__ import annotations

import random

import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G


def _fill_in(rows, S: int) -> list[int]:
    """Eliminate the vertices of S in a random order with fill-in; rows of
    the rest (0 for eliminated vertices)."""
    n = len(rows)
    nb = [int(r) for r in rows]
    order = [v for v in range(n) if (S >> v) & 1]
    random.Random(S).shuffle(order)
    for v in order:
        N = nb[v]
        for w in range(n):
            if (N >> w) & 1:
                nb[w] |= N & ~(1 << w)
                nb[w] &= ~(1 << v)
        nb[v] = 0
    return [0 if (S >> u) & 1 else nb[u] for u in range(n)]


def _induced_relabelled(rows, S: int) -> list[int]:
    keep = [u for u in range(len(rows)) if not (S >> u) & 1]
    pos = {u: t for t, u in enumerate(keep)}
    out = []
    for u in keep:
        r = 0
        for w in keep:
            if (int(rows[u]) >> w) & 1:
                r |= 1 << pos[w]
        out.append(r)
    return out


def _graphs():
    rng = random.Random(3)
    out = [G.grid(3, 4), G.grid(3, 5), G.petersen(), G.cycle(10), G.complete_bipartite(3, 5),
           G.complete_multipartite([2, 3, 3]), G.disjoint_cliques(3, 4)]
    out += [G.gnp(10 + s % 4, 0.3 + 0.05 * (s % 3), 1300 + s) for s in range(6)]
    out += [G.partial_ktree(12, 3 + s % 3, 0.3, 1400 + s) for s in range(4)]
    out += [G.rgg(12, 5.0, 1500 + s) for s in range(2)]
    return out


def _random_states(rng, n, count):
    return [rng.getrandbits(n) for _ in range(count)]


def test_eliminated_graph_equals_fill_in(oracle):
    rng = random.Random(8)
    for rows in _graphs():
        n = len(rows)
        for S in _random_states(rng, n, 25) + [0, (1 << n) - 1]:
            got = [int(x) for x in oracle.eliminated_graph(rows, S)]
            assert got == _fill_in(rows, S), (rows, S)


def test_c_mmw_equals_python(oracle):
    rng = random.Random(9)
    for t in range(400):
        n = rng.randint(1, 24)
        rows = G.gnp(n, rng.uniform(0.05, 0.8), 1600 + t)
        assert oracle.mmw_c(rows) == oracle.mmw(rows), t
    for rows in _graphs():
        assert oracle.mmw_c(rows) == oracle.mmw(rows)


def test_mmw_eliminated_equals_python_on_relabelled(oracle):
    rng = random.Random(10)
    for rows in _graphs():
        n = len(rows)
        for S in _random_states(rng, n, 20) + [0]:
            H = oracle.eliminated_graph(rows, S)
            want = oracle.mmw(_induced_relabelled(H, S)) if S != (1 << n) - 1 else 0
            assert oracle.mmw_eliminated(rows, S) == want, (rows, S)
    # S = V: nothing left, bound 0; S = {} : the graph itself
    rows = G.complete(7)
    assert oracle.mmw_eliminated(rows, (1 << 7) - 1) == 0
    assert oracle.mmw_eliminated(rows, 0) == 6
    # eliminating one vertex of a cycle leaves a cycle one shorter
    assert oracle.mmw_eliminated(G.cycle(9), 1) == 2


def _completable(rows, k: int) -> dict[int, bool]:
    """R(S): from S, the remaining vertices can be eliminated one at a time
    with every |Q| <= k until n - k - 1 are gone (brute force over subsets)."""
    n = len(rows)
    from functools import lru_cache

    L = max(0, n - k - 1)

    def q(S, v):
        seen = {v}
        stack = [v]
        out = 0
        while stack:
            u = stack.pop()
            for w in range(n):
                if (int(rows[u]) >> w) & 1 and w not in seen:
                    seen.add(w)
                    if (S >> w) & 1:
                        stack.append(w)
                    else:
                        out += 1
        return out

    @lru_cache(maxsize=None)
    def R(S):
        if bin(S).count("1") >= L:
            return True
        return any(not (S >> v) & 1 and q(S, v) <= k and R(S | 1 << v) for v in range(n))

    return R


def test_pruning_is_sound_and_answers_unchanged(oracle):
    pruned_total = plain_total = 0
    for rows in _graphs():
        n = len(rows)
        tw, _ = oracle.subset_dp(rows)
        for k in range(0, min(n, tw + 2)):
            yes0, lv0, _ = oracle.decide(rows, k)
            yes1, lv1, _ = oracle.decide(rows, k, prune_mmw=True)
            assert yes0 == yes1 == (tw <= k), (rows, k)
            R = _completable(rows, k)
            for i, (a, b) in enumerate(zip(lv0, lv1)):
                assert set(b.tolist()) <= set(a.tolist())
                for S in a.tolist():
                    if R(int(S)):
                        assert S in set(b.tolist()), (rows, k, i, S)
                plain_total += len(a)
                pruned_total += len(b)
            # a state that is dropped cannot be completed
            for i, f in enumerate(lv1[:-1]):
                keep = oracle.mmw_keep(rows, k, f)
                for S, kp in zip(f.tolist(), keep):
                    if not kp:
                        assert not R(int(S))
    assert pruned_total < plain_total  # the pruning removes something on these graphs


def test_planted_threshold_slip_drops_completable_states(oracle):
    """Pruning at MMW >= k (keep only MMW <= k - 1) is unsound on some graph."""
    found = False
    for rows in _graphs():
        n = len(rows)
        tw, _ = oracle.subset_dp(rows)
        k = tw
        R = _completable(rows, k)
        f = np.zeros(1, dtype=np.uint64)
        for _ in range(oracle.n_levels(n, k)):
            bad = oracle.mmw_keep(rows, k - 1, f)
            if any(R(int(S)) and not kp for S, kp in zip(f.tolist(), bad)):
                found = True
                break
            f, _, _ = oracle.bfs_level(rows, k, f)
        if found:
            break
    assert found
