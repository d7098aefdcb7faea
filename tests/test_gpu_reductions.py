"""GPU parity of the §3.1 reductions (TW_REDUCE_CLIQUE_PATHS) against the oracle.

Levels of decide(k) equal the reduction oracle's (subsets outside the
maximum clique, feasible in G_k+), answers equal the plain ones, and the
batched and single paths agree.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def red():
    from oracle import reductions as R
    return R


@pytest.fixture(scope="module")
def rctx():
    from paper_1709_09990_amd import tw as T
    c = T.Context(device=0, reductions=T.TW_REDUCE_CLIQUE_PATHS)
    yield c
    c.close()


def _graphs_small():
    out = [G.grid(4, 5), G.petersen(), G.complete_multipartite([3, 3, 2]), G.disjoint_cliques(4, 3),
           G.cycle(12), G.complete_bipartite(4, 5)]
    out += [G.gnp(18 + s % 6, 0.3, 7100 + s) for s in range(5)]
    out += [G.partial_ktree(20 + s % 6, 4 + s % 3, 0.3, 7200 + s) for s in range(5)]
    out += [G.rgg(22, 6.0, 7300 + s) for s in range(3)]
    return out


def _compare_levels(oracle, rows, k, yes_ref, ref_levels, yes, levels, C, Gk):
    assert yes == yes_ref, k
    cmask = sum(1 << c for c in C)
    assert len(levels) <= len(ref_levels)
    for lv in levels:
        ref = ref_levels[lv.level]
        got = np.sort(lv.states)
        assert lv.count == len(ref), (k, lv.level, lv.count, len(ref))
        assert np.array_equal(got, ref), (k, lv.level)
        assert not np.any(got & np.uint64(cmask))
        for t in range(min(len(got), 500) if lv.level > 0 else 0):
            S, v = int(lv.states[t]), int(lv.last_v[t])
            assert (S >> v) & 1 and not (cmask >> v) & 1
            assert oracle.q_degree(Gk, S & ~(1 << v), v) <= k
    if len(levels) < len(ref_levels):
        assert levels[-1].count == 0


def test_reduced_levels_match_oracle(oracle, red, rctx):
    for rows in _graphs_small():
        n = len(rows)
        tw, _ = oracle.subset_dp(rows)
        C = red.max_clique(rows)
        P = red.disjoint_paths(rows)
        for k in range(max(0, len(C) - 1), min(n, tw + 2)):
            yes_ref, ref_levels = red.decide_reduced(rows, k, C, P)
            yes, levels = rctx.trace_decide(rows, k)
            _compare_levels(oracle, rows, k, yes_ref, ref_levels, yes, levels, C,
                            red.augmented_rows(rows, k, P))


def test_reduced_decide_below_clique_bound(rctx):
    rows = G.complete_multipartite([1, 1, 1, 1, 1, 3])  # contains K_6
    for k in range(0, 5):
        assert rctx.decide(rows, k)[0] is False
    assert rctx.decide(rows, len(rows) - 1)[0] is True


def test_reduced_64bit_levels(oracle, red, rctx):
    """n > 32 (64-bit keys): levels against the reduction oracle."""
    for rows in (G.partial_ktree(36, 5, 0.3, 7400),):
        C = red.max_clique(rows)
        P = red.disjoint_paths(rows)
        tw = red.treewidth_reduced(rows)
        for k in (tw - 1, tw):
            if k < len(C) - 1:
                continue
            yes_ref, ref_levels = red.decide_reduced(rows, k, C, P)
            yes, levels = rctx.trace_decide(rows, k)
            _compare_levels(oracle, rows, k, yes_ref, ref_levels, yes, levels, C,
                            red.augmented_rows(rows, k, P))


def test_reduced_solve_equals_plain(oracle):
    from paper_1709_09990_amd import tw as T
    graphs = _graphs_small() + [G.partial_ktree(30, 6, 0.3, 7500), G.gnp(28, 0.2, 7501)]
    with T.Context(device=0) as plain, T.Context(device=0, reductions=T.TW_REDUCE_CLIQUE_PATHS) as r:
        for rows in graphs:
            tw0, _, st0 = plain.solve(rows)
            tw1, order, st1 = r.solve(rows)
            assert tw1 == tw0
            assert oracle.order_width(rows, order) == tw1
            assert st1["expansions"] <= st0["expansions"]


def test_reduced_batch_equals_single(oracle):
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(40, seed0=7600, n_lo=10, n_hi=26)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    with T.Context(device=0, reductions=T.TW_REDUCE_CLIQUE_PATHS) as r:
        tws, orders, status, st = r.solve_batch(graphs)
        assert list(status) == [0] * len(graphs)
        assert list(tws) == want
        for rows, tw, order in zip(graphs, tws, orders):
            assert oracle.order_width(rows, order) == tw
        # graphs forced through the single-graph path agree too
    with T.Context(device=0, reductions=T.TW_REDUCE_CLIQUE_PATHS, batch_graph_states=64) as r2:
        tws2, _, status2, _ = r2.solve_batch(graphs[:12])
    assert list(status2) == [0] * 12 and list(tws2) == want[:12]


def test_reduced_full_size_bench_graphs(oracle):
    """The n = 40 bench graphs: same treewidth as the plain search (13 and 8,
    the values the plain full-size runs certify), fewer expansions."""
    from paper_1709_09990_amd import tw as T
    w = G.workload_single_n40()
    with T.Context(device=0, reductions=T.TW_REDUCE_CLIQUE_PATHS) as r:
        for name, tw_want in (("partial8tree40", 8), ("gnp40_p015", 13)):
            print(f"reduced solve {name}", flush=True)
            tw, order, st = r.solve(w[name])
            assert tw == tw_want
            assert oracle.order_width(w[name], order) == tw
            # the order's tree decomposition is valid and has width tw
            bags, parent, width = T.tree_decomposition(w[name], order)
            assert width == tw and oracle.is_tree_decomposition(w[name], bags, parent)


def test_learned_start_with_reductions_is_exact(oracle):
    """The network trained on reduced-search labels only moves the start bound
    and admission: answers equal the oracle's, orders have that width."""
    import os
    from paper_1709_09990_amd import tw as T
    w = os.path.join(os.path.dirname(T.__file__), "weights", "mpnn_mixture_n16_30_reduced.bin")
    graphs = G.workload_batch(32, seed0=7700, n_lo=14, n_hi=26)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    with T.Context(device=0, reductions=T.TW_REDUCE_CLIQUE_PATHS, k_policy=T.TW_K_LEARNED, weights_path=w) as c:
        tws, orders, status, _ = c.solve_batch(graphs)
        assert list(status) == [0] * len(graphs) and list(tws) == want
        for rows, tw, order in zip(graphs, tws, orders):
            assert oracle.order_width(rows, order) == tw
        for rows, tw in zip(graphs[:6], want[:6]):
            assert c.solve(rows)[0] == tw
