"""Pins of the reduction oracle (§3.1: clique skip, disjoint-path edges).

CPU only.  Each function is checked against something other than itself:
brute force over vertex subsets, closed forms, and the subset DP (the plain
definition of treewidth), which the reductions must never change.
"""
from __future__ import annotations

import itertools
import random

import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G


@pytest.fixture(scope="module")
def red(oracle):
    from oracle import reductions as R
    return R


def _is_clique(rows, vs) -> bool:
    return all((int(rows[a]) >> b) & 1 for a, b in itertools.combinations(vs, 2))


def _brute_max_clique(rows) -> list[int]:
    n = len(rows)
    for size in range(n, 0, -1):
        for vs in itertools.combinations(range(n), size):  # ascending, lexicographic order
            if _is_clique(rows, vs):
                return list(vs)
    return []


def _connected_avoiding(rows, s: int, t: int, removed: set[int]) -> bool:
    seen = {s}
    stack = [s]
    while stack:
        a = stack.pop()
        if a == t:
            return True
        for b in range(len(rows)):
            if (int(rows[a]) >> b) & 1 and b not in seen and b not in removed:
                seen.add(b)
                stack.append(b)
    return False


def _brute_min_separator(rows, s: int, t: int) -> int:
    """Smallest vertex set (not containing s, t) whose removal disconnects s
    from t; by Menger's theorem it equals the number of disjoint paths."""
    others = [w for w in range(len(rows)) if w not in (s, t)]
    for size in range(len(others) + 1):
        for X in itertools.combinations(others, size):
            if not _connected_avoiding(rows, s, t, set(X)):
                return size
    return len(others)


def _random_graph(rng: random.Random, n: int, p: float) -> np.ndarray:
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return G.from_edges(n, edges)


def test_max_clique_brute_force(red):
    rng = random.Random(11)
    for _ in range(120):
        n = rng.randint(1, 11)
        rows = _random_graph(rng, n, rng.choice([0.2, 0.4, 0.6, 0.8]))
        assert red.max_clique(rows) == _brute_max_clique(rows)


def test_max_clique_closed_forms(red):
    assert red.max_clique(G.complete(7)) == list(range(7))
    assert len(red.max_clique(G.cycle(9))) == 2
    assert len(red.max_clique(G.petersen())) == 2
    assert len(red.max_clique(G.complete_multipartite([2, 3, 1, 4]))) == 4
    assert len(red.max_clique(G.edgeless(5))) == 1
    for s in range(6):
        k = 2 + s % 4
        assert len(red.max_clique(G.ktree(k + 6, k, 300 + s))) == k + 1


def test_disjoint_paths_menger(red):
    rng = random.Random(5)
    for _ in range(40):
        n = rng.randint(3, 8)
        rows = _random_graph(rng, n, rng.choice([0.3, 0.5, 0.7]))
        P = red.disjoint_paths(rows)
        for u in range(n):
            for v in range(n):
                if u == v or (int(rows[u]) >> v) & 1:
                    assert P[u, v] == 0
                else:
                    assert P[u, v] == _brute_min_separator(rows, u, v), (rows, u, v)


def test_disjoint_paths_closed_forms(red):
    P = red.disjoint_paths(G.cycle(8))
    assert P[0, 4] == 2 and P[1, 3] == 2
    P = red.disjoint_paths(G.complete_bipartite(3, 5))  # sides {0,1,2} and {3..7}
    assert P[0, 1] == 5 and P[3, 7] == 3
    P = red.disjoint_paths(G.petersen())  # 3-connected and 3-regular
    rows = G.petersen()
    for u in range(10):
        for v in range(u + 1, 10):
            if not (int(rows[u]) >> v) & 1:
                assert P[u, v] == 3
    assert red.disjoint_paths(G.path(6))[0, 5] == 1
    assert red.disjoint_paths(G.disjoint_cliques(3, 2))[0, 3] == 0


def _test_graphs():
    rng = random.Random(17)
    out = [G.grid(3, 4), G.grid(4, 4), G.petersen(), G.cycle(9), G.complete_bipartite(3, 4),
           G.complete_multipartite([3, 3, 2]), G.disjoint_cliques(4, 3)]
    out += [G.partial_ktree(13, 3 + s % 3, 0.3, 900 + s) for s in range(6)]
    out += [G.gnp(12 + s % 4, 0.3, 950 + s) for s in range(6)]
    out += [G.rgg(13, 5.0, 980 + s) for s in range(3)]
    out += [_random_graph(rng, 10, 0.45) for _ in range(6)]
    return out


def test_reduced_treewidth_equals_dp(oracle, red):
    for rows in _test_graphs():
        tw, _ = oracle.subset_dp(rows)
        assert red.treewidth_reduced(rows) == tw, rows


def test_augmentation_keeps_the_answer(oracle, red):
    """tw(G_k+) <= k exactly when tw(G) <= k, for every k."""
    for rows in _test_graphs()[:14]:
        tw, _ = oracle.subset_dp(rows)
        P = red.disjoint_paths(rows)
        for k in range(len(rows)):
            twk, _ = oracle.subset_dp(red.augmented_rows(rows, k, P))
            assert (twk <= k) == (tw <= k), (rows, k)


def test_reduced_levels_equal_dp_on_augmented_graph(oracle, red):
    """F_i = {S outside C : |S| = i, TW_{G_k+}(S) <= k}, by the subset DP."""
    for rows in _test_graphs()[:16]:
        n = len(rows)
        C = red.max_clique(rows)
        cmask = sum(1 << c for c in C)
        P = red.disjoint_paths(rows)
        tw, _ = oracle.subset_dp(rows)
        for k in range(max(0, len(C) - 1), min(n, tw + 2)):
            yes, levels = red.decide_reduced(rows, k, C, P)
            assert yes == (tw <= k)
            ref = oracle.frontiers_from_dp(red.augmented_rows(rows, k, P), k)
            for i, lv in enumerate(levels):
                want = np.array([s for s in ref[i] if not int(s) & cmask], dtype=np.uint64)
                assert np.array_equal(lv, want), (k, i)


def test_reduced_decide_below_clique_is_no(red):
    rows = G.complete(6)
    assert red.decide_reduced(rows, 4)[0] is False
    assert red.decide_reduced(rows, 5)[0] is True


def test_reduction_pins_catch_planted_mistakes(oracle, red):
    """Two plausible slips — adding edges at k disjoint paths instead of k + 1,
    and skipping a vertex set that is not a clique — change some treewidth."""
    graphs = _test_graphs()
    wrong_threshold = 0
    wrong_clique = 0
    for rows in graphs:
        tw, _ = oracle.subset_dp(rows)
        n = len(rows)
        P = red.disjoint_paths(rows)
        for k in range(n):
            bad = red.augmented_rows(rows, k - 1, P)  # threshold k instead of k + 1
            if (oracle.subset_dp(bad)[0] <= k) != (tw <= k):
                wrong_threshold += 1
                break
        # skip an edge's endpoints plus a non-neighbour: not a clique
        a = next((u for u in range(n) if int(rows[u])), None)
        if a is None:
            continue
        b = (int(rows[a]) & -int(rows[a])).bit_length() - 1
        c = next((w for w in range(n) if w not in (a, b) and not (int(rows[a]) >> w) & 1), None)
        if c is None:
            continue
        S = [a, b, c]
        for k in range(n):
            yes, _ = red.decide_reduced(rows, k, S, P)
            if yes != (tw <= k):
                wrong_clique += 1
                break
    assert wrong_threshold > 0
    assert wrong_clique > 0
