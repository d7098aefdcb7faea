"""What the trained start-bound network gains (the learned part of the
batched solver): on held-out graphs of the training mixture, the committed
weights make the batched search try fewer bounds and expand fewer (S, v)
pairs than the ascending search from the minor-min-width bound, with the same
treewidth for every graph.  Deterministic: predictions, bounds and the exact
levels do not depend on timing."""
import os

import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1709_09990_amd",
                       "weights")


@pytest.mark.parametrize("reduced", [False, True], ids=["plain_search", "with_reductions"])
def test_trained_network_saves_bounds_and_expansions(oracle, reduced):
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(160, seed0=600000, n_lo=20, n_hi=28)   # held out: training used seeds 500000+
    base = {"reductions": T.TW_REDUCE_CLIQUE_PATHS} if reduced else {}
    wfile = "mpnn_mixture_n16_30_reduced.bin" if reduced else "mpnn_mixture_n16_30.bin"
    with T.Context(device=0, **base) as c:
        tw_p, _, st_p, stats_p, per_p = c.solve_batch(graphs, graph_stats=True)
    with T.Context(device=0, k_policy=T.TW_K_LEARNED, weights_path=os.path.join(WEIGHTS, wfile), **base) as c:
        tw_l, orders, st_l, stats_l, per_l = c.solve_batch(graphs, graph_stats=True)
    assert list(st_p) == [0] * len(graphs) and list(st_l) == [0] * len(graphs)
    assert np.array_equal(tw_p, tw_l)
    for rows, tw, order in zip(graphs, tw_l, orders):
        assert oracle.order_width(rows, order) == tw
    print(f"bounds {stats_l['decisions']} vs {stats_p['decisions']}, "
          f"expansions {stats_l['expansions']} vs {stats_p['expansions']}", flush=True)
    assert stats_l["decisions"] < stats_p["decisions"]
    assert stats_l["expansions"] < stats_p["expansions"]
    # the start bounds are the network's: not all equal to the lower bound
    assert sum(1 for a, b in zip(per_l, per_p) if a["start_k"] != b["start_k"]) >= 10
