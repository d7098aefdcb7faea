"""Level-by-level parity of the batched search against the oracle.

tw_trace_batch records, for every graph solved in the batch, every level its
search built (bound k, level i, |level i|, feasible pairs from level i-1, two
order-independent digests).  Each record must equal the oracle's level search
(Listing 1 with exact duplicate removal, §3.1) for that bound: the same count,
the same feasible-pair count and the same digests of the same set of states.
The bounds must follow the search of §3.1 from the start bound: ascending
from the lower bound until the first YES, or, from a learned start, down
after each YES and up after each NO until a YES at t meets a NO at t-1.
"""
import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu

# oracle levels per (graph, bound), shared by the tests of this module
_CACHE: dict = {}


def _oracle_levels(oracle, rows, k, cache):
    key = (rows.tobytes(), k)
    if key not in cache:
        yes, levels, stats = oracle.decide(rows, k)
        recs = []
        for i in range(1, len(levels)):
            c, hs, hx = oracle.set_hashes(levels[i])
            recs.append((k, i, c, stats[i - 1][1], hs, hx))
            if c == 0:
                break
        cache[key] = (yes, recs)
    return cache[key]


def _check_graph(oracle, rows, recs, tw, lb, start_k, cache):
    """Records of one graph: grouped by bound in the order run, each group the
    oracle's levels of that bound; the bounds follow the certifying search."""
    assert recs, "a batched graph recorded no level"
    groups = []
    for r in recs:
        if not groups or groups[-1][0] != r[0] or r[1] == 1:
            groups.append((r[0], []))
        groups[-1][1].append(r)
    ks = [k for k, _ in groups]
    assert ks[0] == start_k, (ks, start_k)
    known_no, best_yes = lb - 1, len(rows) - 1
    for k, got in groups:
        yes, want = _oracle_levels(oracle, rows, k, cache)
        assert got == want, (k, got[:3], want[:3])
        if yes:
            best_yes = min(best_yes, k)
        else:
            known_no = max(known_no, k)
    # the search stops exactly when YES at t meets NO at t-1 (or t = lower bound)
    assert best_yes == tw and known_no == tw - 1
    return len(groups)


def _run(ctx, oracle, graphs, cache, first_arena=0):
    tws, orders, status, per, records = ctx.trace_batch(graphs, first_arena_states=first_arena)
    assert list(status) == [0] * len(graphs)
    batched = 0
    bounds = []
    for t, rows in enumerate(graphs):
        lb = oracle.mmw(rows)
        tw = int(tws[t])
        assert oracle.order_width(rows, orders[t]) == tw
        if per[t]["path"] != 0:
            assert records[t] == []
            continue
        batched += 1
        bounds.append(_check_graph(oracle, rows, records[t], tw, lb, per[t]["start_k"], cache))
    return tws, per, batched, bounds


@pytest.mark.parametrize("schedule", ["rounds", "persistent"])
def test_batch_levels_equal_oracle(oracle, schedule):
    """120 graphs of the uneven mixture (n 12..24), ascending bounds: every
    level of every bound of every graph equals the oracle's."""
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(120, seed0=41000, n_lo=12, n_hi=24)
    sched = T.TW_BATCH_ROUNDS if schedule == "rounds" else T.TW_BATCH_PERSISTENT
    cache = _CACHE
    with T.Context(device=0, batch_schedule=sched) as c:
        tws, per, batched, bounds = _run(c, oracle, graphs, cache)
    assert batched >= 110, batched
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    assert list(tws) == want
    assert sum(bounds) > batched  # several graphs needed more than one bound


def test_batch_levels_after_arena_retry(oracle):
    """A first arena of 2048 states: graphs whose levels outgrow it are run
    again in the batch with four times the arena (level rounds); the records of
    that second attempt equal the oracle's levels too."""
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(64, seed0=42000, n_lo=12, n_hi=22)
    cache = _CACHE
    with T.Context(device=0, batch_schedule=T.TW_BATCH_ROUNDS) as c:
        tws, per, batched, _ = _run(c, oracle, graphs, cache, first_arena=2048)
    # graphs batched although one bound's levels hold more than the first arena
    retried = 0
    for t, rows in enumerate(graphs):
        if per[t]["path"] != 0:
            continue
        lb = oracle.mmw(rows)
        need = max(1 + sum(len(lv) for lv in oracle.decide(rows, k)[1][1:]) for k in range(lb, int(tws[t]) + 1))
        if need > 2048:
            retried += 1
    assert retried >= 8, retried
    assert batched >= 24, batched


def test_batch_levels_many_bounds_learned(oracle, tmp_path):
    """A network whose prediction is tw = n starts every graph at n-2, so the
    batched search moves down through many YES bounds, reusing each graph's
    tagged table across all of them; every level of every bound still equals
    the oracle's."""
    from paper_1709_09990_amd import tw as T
    p = np.zeros(T.mpnn_param_count(), dtype=np.float32)
    p[-2] = 1.0   # bias of the tw/n output
    p[-1] = 0.0   # predicted peak 0: the default arena
    wpath = tmp_path / "start_high.bin"
    T.write_weights(str(wpath), p)
    graphs = G.workload_batch(24, seed0=43000, n_lo=14, n_hi=20)
    cache = _CACHE
    with T.Context(device=0, k_policy=T.TW_K_LEARNED, weights_path=str(wpath)) as c:
        tws, per, batched, bounds = _run(c, oracle, graphs, cache)
    assert batched >= 20
    assert max(bounds) > 8, bounds
    assert all(per[t]["start_k"] == len(graphs[t]) - 2 for t in range(len(graphs)) if per[t]["path"] == 0)
