"""GPU parity of per-state minor-min-width pruning (TW_MMW_PRUNE, §3.3)
against the oracle's O6: levels of decide(k) equal the oracle's (successors
of the states with MMW(H_S) <= k), answers and orders equal the plain ones.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu


def _graphs_small():
    out = [G.grid(4, 5), G.petersen(), G.complete_multipartite([3, 3, 2]), G.disjoint_cliques(4, 3),
           G.cycle(12), G.complete_bipartite(4, 5), G.complete(6), G.path(9)]
    out += [G.gnp(16 + s % 8, 0.3, 8100 + s) for s in range(6)]
    out += [G.partial_ktree(20 + s % 5, 4 + s % 3, 0.3, 8200 + s) for s in range(4)]
    out += [G.rgg(22, 6.0, 8300 + s) for s in range(3)]
    return out


def _compare(oracle, rows, k, yes_ref, ref_levels, yes, levels, allowed=None):
    assert yes == yes_ref, k
    n = len(rows)
    for lv in levels:
        ref = ref_levels[lv.level]
        got = np.sort(lv.states)
        assert lv.count == len(ref), (k, lv.level, lv.count, len(ref))
        assert np.array_equal(got, ref), (k, lv.level)
        if lv.level == 0:
            continue
        for t in range(min(len(got), 300)):
            S, v = int(lv.states[t]), int(lv.last_v[t])
            assert v < n and (S >> v) & 1
            assert oracle.q_degree(rows, S & ~(1 << v), v) <= k
            # the state it came from was kept by the pruning
            assert oracle.mmw_eliminated(rows, S & ~(1 << v)) <= k
    for ref in ref_levels[len(levels):]:
        assert len(ref) == 0


def test_pruned_levels_match_oracle(oracle):
    from paper_1709_09990_amd import tw as T
    with T.Context(device=0, mmw_prune=T.TW_MMW_PRUNE) as c:
        for rows in _graphs_small():
            n = len(rows)
            tw, _ = oracle.subset_dp(rows)
            for k in range(max(0, oracle.mmw(rows) - 1), min(n, tw + 2)):
                yes_ref, ref_levels, _ = oracle.decide(rows, k, prune_mmw=True)
                yes, levels = c.trace_decide(rows, k)
                _compare(oracle, rows, k, yes_ref, ref_levels, yes, levels)


def test_pruned_levels_64bit_keys(oracle):
    """n > 32 (64-bit keys) on graphs whose levels stay small (the oracle's
    pruned search takes seconds): the 3 x 12 grid (tw 3, levels up to 3e5),
    the 2 x 20 ladder (tw 2) and the 40-path (tw 1)."""
    from paper_1709_09990_amd import tw as T
    with T.Context(device=0, mmw_prune=T.TW_MMW_PRUNE) as c:
        for rows, tw in ((G.grid(3, 12), 3), (G.grid(2, 20), 2), (G.path(40), 1)):
            for k in (tw - 1, tw):
                print(f"pruned 64-bit n={len(rows)} k={k}", flush=True)
                yes_ref, ref_levels, _ = oracle.decide(rows, k, prune_mmw=True)
                yes, levels = c.trace_decide(rows, k)
                _compare(oracle, rows, k, yes_ref, ref_levels, yes, levels)


def test_pruned_with_reductions_match_oracle(oracle):
    from oracle import reductions as R
    from paper_1709_09990_amd import tw as T
    with T.Context(device=0, mmw_prune=T.TW_MMW_PRUNE, reductions=T.TW_REDUCE_CLIQUE_PATHS) as c:
        for rows in _graphs_small()[8:]:
            n = len(rows)
            tw, _ = oracle.subset_dp(rows)
            C = R.max_clique(rows)
            P = R.disjoint_paths(rows)
            for k in range(max(0, len(C) - 1), min(n, tw + 2)):
                yes_ref, ref_levels = R.decide_reduced(rows, k, C, P, prune_mmw=True)
                yes, levels = c.trace_decide(rows, k)
                _compare(oracle, R.augmented_rows(rows, k, P), k, yes_ref, ref_levels, yes, levels)


def test_pruned_solve_equals_plain(oracle):
    from paper_1709_09990_amd import tw as T
    graphs = _graphs_small() + [G.partial_ktree(30, 6, 0.3, 8500), G.gnp(26, 0.2, 8501)]
    with T.Context(device=0) as plain, T.Context(device=0, mmw_prune=T.TW_MMW_PRUNE) as p:
        for rows in graphs:
            tw0, _, st0 = plain.solve(rows)
            tw1, order, st1 = p.solve(rows)
            assert tw1 == tw0
            assert oracle.order_width(rows, order) == tw1
            assert st1["states_expanded"] <= st0["states_expanded"]
        # decide below the graph's own MMW: the root is pruned, NO
        rows = G.complete(7)
        assert p.decide(rows, 5)[0] is False and p.decide(rows, 6)[0] is True


def test_pruned_full_size_and_batch(oracle):
    from paper_1709_09990_amd import tw as T
    w = G.workload_single_n40()
    graphs = G.workload_batch(24, seed0=8600, n_lo=12, n_hi=24)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    with T.Context(device=0, mmw_prune=T.TW_MMW_PRUNE) as p:
        print("pruned solve partial8tree40", flush=True)
        tw, order, _ = p.solve(w["partial8tree40"])
        assert tw == 8 and oracle.order_width(w["partial8tree40"], order) == 8
        tws, orders, status, _ = p.solve_batch(graphs)
        assert list(status) == [0] * len(graphs) and list(tws) == want
        for rows, t, o in zip(graphs, tws, orders):
            assert oracle.order_width(rows, o) == t
