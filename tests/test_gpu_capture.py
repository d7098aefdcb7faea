"""The captured level loop (options.capture = TW_CAPTURE_AUTO): each bound's
level loop (Listing 1, §3.1) replayed as one HIP graph must give exactly what
the host-driven loop gives — the same treewidths, orders of that width and the
same work counters level for level summed (states expanded, feasible pairs,
new states, largest level, levels run) — replay after replay, with other
launches and host waits of the program between the replays."""
import pytest

from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu

KEYS = ("expansions", "successors", "unique", "states_expanded", "peak_frontier", "decisions", "levels")


def _pairs(graphs, cap_kw, off_kw, oracle):
    from paper_1709_09990_amd import tw as T
    with T.Context(device=0, **cap_kw) as cap, T.Context(device=0, capture=T.TW_CAPTURE_OFF, **off_kw) as off:
        replays = 0
        for rows in graphs:
            tw_a, order_a, st_a = cap.solve(rows)
            # eager work of the program between replays
            tw_b, order_b, st_b = off.solve(rows)
            for k in {max(0, tw_b - 1), tw_b}:
                yes_a, sd_a = cap.decide(rows, k)
                yes_b, sd_b = off.decide(rows, k)
                assert yes_a == yes_b == (k >= tw_b)
                for key in KEYS:
                    assert sd_a[key] == sd_b[key], (key, k)
            assert tw_a == tw_b
            assert oracle.order_width(rows, order_a) == tw_a
            for key in KEYS:
                assert st_a[key] == st_b[key], (key, st_a[key], st_b[key])
            # one launch per bound searched on the captured path, one per level on the other
            assert st_b["launches"] == st_b["levels"]
            if st_a["levels"]:
                assert st_a["launches"] < st_a["levels"]
            replays += st_a["launches"]
        return replays


def test_captured_equals_host_loop(oracle):
    """G(20, 0.3) seeds 1001..1032 and graphs of other sizes and families."""
    graphs = [G.workload_single_small(1001 + t) for t in range(32)]
    graphs += G.workload_batch(24, seed0=44000, n_lo=6, n_hi=24)
    graphs += [G.cycle(11), G.grid(4, 5), G.petersen(), G.complete(7)]
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    replays = _pairs(graphs, {}, {}, oracle)
    assert replays > len(graphs)
    from paper_1709_09990_amd import tw as T
    with T.Context(device=0) as c:
        assert [c.solve(r)[0] for r in graphs] == want


def test_captured_with_reductions(oracle):
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(24, seed0=45000, n_lo=10, n_hi=24)
    red = {"reductions": T.TW_REDUCE_CLIQUE_PATHS}
    _pairs(graphs, red, red, oracle)


def test_captured_learned_start(oracle):
    """A learned start above tw replays the captured loop downwards (YES after
    YES) before the certifying NO; counters equal the host-driven loop's."""
    import os
    from paper_1709_09990_amd import tw as T
    w = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1709_09990_amd", "weights",
                     "mpnn_mixture_n16_30.bin")
    kw = {"k_policy": T.TW_K_LEARNED, "weights_path": w}
    graphs = G.workload_batch(16, seed0=46000, n_lo=16, n_hi=24)
    _pairs(graphs, kw, kw, oracle)
