"""Pins of the CPU oracle against facts that do not come from the oracle.

* Q(S,v) against hand-worked values of the definition (§2) and against an
  independent pure-Python search.
* The width of an order through Q (§2) against explicit fill-in (§2, the
  alternative view) — two definitions.
* O1 (subset DP) against closed forms and against O2 (brute force over all
  n! orders with fill-in widths).
* O4 (Listing 1 with exact dedup, §3.1) against O1 level by level, and
  against closed-form frontier sizes.
* The number of levels (last k+1 vertices free, §3.1) through tw equality.
* Minor-min-width (§3.3) as a lower bound, and on families with known values.
"""
import itertools
import math
import os
import random

import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parse_list(tok):
    return [] if tok == "-" else [int(x) for x in tok.split(",")]


def _golden_q():
    H = G.from_edges(5, [(0, 1), (1, 2), (2, 3), (1, 4)])
    C = G.cycle(6)
    graphs = {"H": H, "C": C}
    cases = []
    with open(os.path.join(GOLDEN, "q_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            g, s, v, q = line.split()
            S = sum(1 << x for x in _parse_list(s))
            cases.append((graphs[g], S, int(v), set(_parse_list(q))))
    return cases


def test_q_hand_examples(oracle):
    cases = _golden_q()
    assert len(cases) >= 10
    for rows, S, v, q in cases:
        assert oracle.q_set_py(rows, S, v) == q
        assert oracle.q_degree(rows, S, v) == len(q)


def test_q_degree_matches_python_search(oracle):
    rng = random.Random(7)
    for t in range(300):
        n = rng.randint(2, 24)
        rows = G.gnp(n, rng.uniform(0.05, 0.6), 100 + t)
        v = rng.randrange(n)
        S = 0
        for u in range(n):
            if u != v and rng.random() < 0.5:
                S |= 1 << u
        assert oracle.q_degree(rows, S, v) == len(oracle.q_set_py(rows, S, v))


def test_order_width_two_definitions(oracle):
    """max_t |Q({order[<t]}, order[t])| equals the fill-in width (§2)."""
    rng = random.Random(11)
    for t in range(200):
        n = rng.randint(1, 16)
        rows = G.gnp(n, rng.uniform(0.1, 0.7), 500 + t)
        order = list(range(n))
        rng.shuffle(order)
        assert oracle.order_width(rows, order) == oracle.order_width_q(rows, order)


def _closed_form_graph(family, params):
    p = _parse_list(params)
    return {
        "complete": lambda: G.complete(p[0]),
        "edgeless": lambda: G.edgeless(p[0]),
        "path": lambda: G.path(p[0]),
        "cycle": lambda: G.cycle(p[0]),
        "grid": lambda: G.grid(p[0], p[1]),
        "bipartite": lambda: G.complete_bipartite(p[0], p[1]),
        "multipartite": lambda: G.complete_multipartite(p),
        "petersen": lambda: G.petersen(),
        "cliques": lambda: G.disjoint_cliques(p[0], p[1]),
    }[family]()


def _closed_forms():
    out = []
    with open(os.path.join(GOLDEN, "closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            fam, params, tw = line.split()
            out.append((fam, params, int(tw)))
    return out


@pytest.mark.parametrize("fam,params,tw", _closed_forms())
def test_dp_closed_forms(oracle, fam, params, tw):
    rows = _closed_form_graph(fam, params)
    got, _ = oracle.subset_dp(rows)
    assert got == tw
    # the level search of Listing 1 agrees
    assert oracle.treewidth_bfs(rows) == tw


def test_dp_random_trees_and_ktrees(oracle):
    for s in range(20):
        n = 2 + s % 15
        assert oracle.subset_dp(G.random_tree(n, s))[0] == 1
    for s in range(12):
        k = 1 + s % 5
        n = k + 1 + (s * 7) % 9
        assert oracle.subset_dp(G.ktree(n, k, 40 + s))[0] == k


def test_dp_partial_ktrees_bounded(oracle):
    for s in range(12):
        k = 2 + s % 4
        rows = G.partial_ktree(14 + s % 5, k, 0.3, 70 + s)
        tw, _ = oracle.subset_dp(rows)
        assert tw <= k


def test_brute_force_equals_dp(oracle):
    """O2 (n! orders, fill-in) pins O1 (subset DP over Q)."""
    rng = random.Random(3)
    count = 0
    for t in range(400):
        n = rng.randint(1, 8 if t < 360 else 9)
        rows = G.gnp(n, rng.uniform(0.1, 0.8), 1000 + t)
        bf, order = oracle.brute_force(rows)
        dp, _ = oracle.subset_dp(rows)
        assert bf == dp, (n, t)
        assert oracle.order_width(rows, order) == bf
        count += 1
    assert count == 400


def test_brute_force_exhaustive_tiny(oracle):
    """Every graph on 5 labelled vertices (1024 of them)."""
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        rows = G.from_edges(5, [pairs[t] for t in range(len(pairs)) if (mask >> t) & 1])
        assert oracle.brute_force(rows)[0] == oracle.subset_dp(rows)[0]


def test_level_search_equals_dp_frontiers(oracle):
    """O4 (Listing 1, exact dedup) reproduces {S : |S|=i, TW(S) <= k}."""
    rng = random.Random(5)
    for t in range(24):
        n = rng.randint(4, 16)
        rows = G.gnp(n, rng.uniform(0.15, 0.6), 2000 + t)
        tw, table = oracle.subset_dp(rows)
        for k in range(0, n):
            yes, levels, stats = oracle.decide(rows, k)
            ref = oracle.frontiers_from_dp(rows, k, table)
            assert len(levels) == len(ref)
            for a, b in zip(levels, ref):
                assert np.array_equal(a, b)
            assert yes == (k >= tw)
            # E_i is |F_i| * (n - i) by definition
            for i, (cand, gen) in enumerate(stats):
                assert cand == len(levels[i]) * (n - i)
                assert len(levels[i + 1]) <= gen <= cand


def test_level_count_reading(oracle):
    """tw = min{k : F_{n-k-1}(k) non-empty} equals TW(V) (last k+1 vertices free)."""
    for t in range(30):
        rows = G.gnp(6 + t % 10, 0.35, 3000 + t)
        assert oracle.treewidth_bfs(rows) == oracle.subset_dp(rows)[0]


def test_closed_form_frontier_sizes(oracle):
    """Edgeless at k=0 and disjoint K_c at k >= c-1: every subset is feasible,
    so |F_i| = C(n,i) and G_i = C(n,i)(n-i); at k = c-2, F_1 is empty."""
    n = 14
    yes, levels, stats = oracle.decide(G.edgeless(n), 0)
    assert yes
    for i, f in enumerate(levels):
        assert len(f) == math.comb(n, i)
    for i, (cand, gen) in enumerate(stats):
        assert gen == math.comb(n, i) * (n - i) == cand
    c, copies = 4, 4
    rows = G.disjoint_cliques(c, copies)
    yes, levels, _ = oracle.decide(rows, c - 1)
    assert yes and all(len(f) == math.comb(c * copies, i) for i, f in enumerate(levels))
    yes, levels, _ = oracle.decide(rows, c - 2)
    assert not yes and len(levels[1]) == 0


def test_frontier_monotone_in_k(oracle):
    """F_i(k) is a subset of F_i(k+1)."""
    rows = G.gnp(15, 0.3, 4242)
    _, table = oracle.subset_dp(rows)
    for k in range(0, 12):
        a = oracle.frontiers_from_dp(rows, k, table)
        b = oracle.frontiers_from_dp(rows, k + 1, table)
        for i in range(len(b)):
            if i < len(a):
                assert np.isin(a[i], b[i]).all()


def test_mmw_lower_bound(oracle):
    rng = random.Random(9)
    for t in range(300):
        n = rng.randint(1, 14)
        rows = G.gnp(n, rng.uniform(0.05, 0.8), 5000 + t)
        assert oracle.mmw(rows) <= oracle.subset_dp(rows)[0]
    for t in range(30):
        rows = G.partial_ktree(16, 3 + t % 5, 0.3, 6000 + t)
        assert oracle.mmw(rows) <= oracle.subset_dp(rows)[0]


def test_mmw_known_values(oracle):
    for n in range(2, 12):
        assert oracle.mmw(G.complete(n)) == n - 1
    for n in range(3, 12):
        assert oracle.mmw(G.cycle(n)) == 2
    for s in range(10):
        assert oracle.mmw(G.random_tree(2 + s, s)) == 1
    assert oracle.mmw(G.edgeless(9)) == 0
    assert oracle.mmw(G.complete(1)) == 0
    for a, b in [(2, 5), (3, 3), (3, 7)]:
        assert oracle.mmw(G.complete_bipartite(a, b)) == min(a, b)


def test_set_hashes_order_independent(oracle):
    x = np.array([5, 17, 1 << 40, 3], dtype=np.uint64)
    assert oracle.set_hashes(x) == oracle.set_hashes(x[::-1].copy())
    assert oracle.set_hashes(x) != oracle.set_hashes(x[:3])
    assert oracle.set_hashes(np.zeros(0, dtype=np.uint64)) == (0, 0, 0)


def test_set_hashes_pinned(oracle):
    """The level digests: the sum uses splitmix64's output function (its
    published sequence from seed 0 starts 0xe220a8397b1dcdaf,
    0x6e789e6aa1b965f4: the output function of the state after one and two
    increments of 0x9e3779b97f4a7c15); both digests add over disjoint unions;
    dropping, duplicating or replacing one state changes them."""
    gamma = 0x9E3779B97F4A7C15
    x = np.array([gamma, (2 * gamma) % 2**64], dtype=np.uint64)
    assert [int(v) for v in oracle._mix_a(x)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]
    rng = np.random.default_rng(5)
    for _ in range(20):
        a = np.unique(rng.integers(0, 2**62, size=int(rng.integers(2, 2000)), dtype=np.uint64))
        b = np.unique(rng.integers(2**62, 2**63, size=int(rng.integers(1, 2000)), dtype=np.uint64))
        ca, sa, xa = oracle.set_hashes(a)
        cb, sb, xb = oracle.set_hashes(b)
        assert oracle.set_hashes(np.concatenate([a, b])) == (ca + cb, (sa + sb) % 2**64, xa ^ xb)
        full = oracle.set_hashes(a)
        dropped = oracle.set_hashes(a[1:])
        dup = oracle.set_hashes(np.concatenate([a, a[:1]]))
        repl = a.copy()
        repl[0] = np.uint64(2**63 + 7)
        replaced = oracle.set_hashes(repl)
        for other in (dropped, dup, replaced):
            assert other[1] != full[1] and other[2] != full[2] or other[0] != full[0]
        assert replaced[0] == full[0] and replaced[1] != full[1] and replaced[2] != full[2]
        # a duplicated state leaves the xor digest unchanged but not the sum or the count
        assert dup[1] != full[1] and dup[0] == full[0] + 1


def test_pins_catch_planted_mistakes(oracle):
    """Mistakes planted in a copy of the oracle's Q (on the CPU) are caught by
    the pins above: counting v itself, or dropping the 'through S only' rule."""
    def q_counts_v(rows, S, v):
        return len(oracle.q_set_py(rows, S, v)) + 1

    def q_any_path(rows, S, v):
        # reach through every vertex, not only those in S
        n = len(rows)
        seen, todo = {v}, [v]
        while todo:
            u = todo.pop()
            for w in range(n):
                if (int(rows[u]) >> w) & 1 and w not in seen:
                    seen.add(w)
                    todo.append(w)
        return len([w for w in seen if w != v and not (S >> w) & 1])

    def width(rows, order, q):
        S, w = 0, 0
        for v in order:
            w = max(w, q(rows, S, v))
            S |= 1 << v
        return w

    cases = _golden_q()
    for bad in (q_counts_v, q_any_path):
        caught = any(bad(r, S, v) != len(q) for r, S, v, q in cases)
        rng = random.Random(1)
        for t in range(50):
            n = rng.randint(3, 9)
            rows = G.gnp(n, 0.4, 9000 + t)
            order = list(range(n))
            rng.shuffle(order)
            caught |= width(rows, order, bad) != oracle.order_width(rows, order)
        assert caught


def test_tree_decomposition_checker(oracle):
    """Hand-made decompositions: valid ones pass, each broken condition fails."""
    P4 = G.path(4)  # 0-1-2-3
    bags = [0b0011, 0b0110, 0b1100]
    assert oracle.is_tree_decomposition(P4, bags, [-1, 0, 1])
    assert oracle.decomposition_width(bags) == 1
    assert not oracle.is_tree_decomposition(P4, [0b0011, 0b1100], [-1, 0])          # edge 1-2 uncovered
    assert not oracle.is_tree_decomposition(P4, [0b0011, 0b0100, 0b1110], [-1, 0, 1])  # bags of 1 disconnected
    assert not oracle.is_tree_decomposition(P4, bags, [1, 2, 0])                     # parent cycle
    assert not oracle.is_tree_decomposition(P4, [0b0011, 0b0110], [-1, 0])           # vertex 3 missing
    C4 = G.cycle(4)
    assert oracle.is_tree_decomposition(C4, [0b0111, 0b1101], [-1, 0])
    assert not oracle.is_tree_decomposition(C4, [0b0011, 0b0110, 0b1100], [-1, 0, 1])  # edge 3-0 uncovered
    # two components: a forest with two roots
    two = G.disjoint_cliques(2, 2)
    assert oracle.is_tree_decomposition(two, [0b0011, 0b1100], [-1, -1])
