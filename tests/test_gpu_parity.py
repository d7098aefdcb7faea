"""GPU parity: the HIP path against the CPU oracle, element by element.

Every level of every bound k is compared as a set (the device writes states
in a nondeterministic order, so both sides are sorted): the same states, the
same counts, the same numbers of candidate and feasible (S, v) pairs.  Each
state's recorded last vertex must lead back into the previous level with a
feasible degree.  Treewidth must equal O1's and the returned order must have
exactly that width by the oracle's fill-in count.
"""
import math

import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1709_09990_amd import tw as T
    c = T.Context(device=0)
    yield c
    c.close()


def _check_levels(oracle, rows, k, levels_gpu, ref_levels, ref_stats=None):
    n = len(rows)
    assert len(levels_gpu) <= len(ref_levels)
    for lv in levels_gpu:
        i = lv.level
        ref = ref_levels[i]
        got = np.sort(lv.states)
        assert lv.count == len(ref), (k, i, lv.count, len(ref))
        assert np.array_equal(got, ref), (k, i)
        assert len(np.unique(got)) == len(got)
        if i > 0:
            assert lv.expansions == len(ref_levels[i - 1]) * (n - i + 1)
            if ref_stats is not None:
                assert lv.successors == ref_stats[i - 1][1], (k, i)
            # the recorded creator leads back into level i-1 with degree <= k
            prev = ref_levels[i - 1]
            sample = np.arange(len(got)) if len(got) <= 4000 else np.linspace(0, len(got) - 1, 4000).astype(int)
            for t in sample:
                S = int(lv.states[t])
                v = int(lv.last_v[t])
                assert (S >> v) & 1
                P = S & ~(1 << v)
                idx = np.searchsorted(prev, np.uint64(P))
                assert idx < len(prev) and int(prev[idx]) == P
                assert oracle.q_degree(rows, P, v) <= k
    # levels stop early only after an empty one
    if len(levels_gpu) < len(ref_levels):
        assert levels_gpu[-1].count == 0


def _parity_all_k(oracle, ctx, rows, k_values=None):
    n = len(rows)
    tw, table = oracle.subset_dp(rows)
    if k_values is None:
        k_values = range(max(0, oracle.mmw(rows) - 1), min(n, tw + 2))
    for k in k_values:
        ref_levels = oracle.frontiers_from_dp(rows, k, table)
        yes, levels = ctx.trace_decide(rows, k)
        assert yes == (k >= tw), (k, tw)
        _check_levels(oracle, rows, k, levels, ref_levels)
    return tw


def test_small_graph_32bit_levels_match_dp(oracle, ctx):
    """G(20, 0.3), seed 1001: every level for every k around tw equals O1."""
    rows = G.workload_single_small(1001)
    tw = _parity_all_k(oracle, ctx, rows)
    got_tw, order, st = ctx.solve(rows)
    assert got_tw == tw
    assert oracle.order_width(rows, order) == tw
    assert sorted(order.tolist()) == list(range(len(rows)))


@pytest.mark.parametrize("seed", range(1002, 1033))
def test_small_graph_seeds(oracle, ctx, seed):
    rows = G.workload_single_small(seed)
    tw, table = oracle.subset_dp(rows)
    got_tw, order, st = ctx.solve(rows)
    assert got_tw == tw
    assert oracle.order_width(rows, order) == tw
    # levels at tw and tw-1 against O1 with feasible-pair counts from O4
    for k in (tw - 1, tw):
        if k < 0:
            continue
        ref_levels = oracle.frontiers_from_dp(rows, k, table)
        _, _, ref_stats = oracle.decide(rows, k)
        yes, levels = ctx.trace_decide(rows, k)
        assert yes == (k == tw)
        _check_levels(oracle, rows, k, levels, ref_levels, ref_stats)


@pytest.mark.parametrize("n,p,seed", [(8, 0.5, 1), (13, 0.4, 2), (17, 0.25, 3), (22, 0.2, 4),
                                       (24, 0.15, 5), (28, 0.25, 6), (30, 0.3, 7), (32, 0.35, 8),
                                       (32, 0.25, 9)])
def test_random_graphs_32bit(oracle, ctx, n, p, seed):
    """Sizes up to the 32-bit boundary; O4 supplies levels and pair counts."""
    rows = G.gnp(n, p, 11000 + seed)
    lb = oracle.mmw(rows)
    tw = oracle.treewidth_bfs(rows, lb)
    got_tw, order, _ = ctx.solve(rows)
    assert got_tw == tw
    assert oracle.order_width(rows, order) == tw
    for k in (tw - 1, tw):
        if k < 0:
            continue
        _, ref_levels, ref_stats = oracle.decide(rows, k)
        _, levels = ctx.trace_decide(rows, k)
        _check_levels(oracle, rows, k, levels, ref_levels, ref_stats)


@pytest.mark.parametrize("maker", [
    lambda: G.gnp(34, 0.3, 12001),
    lambda: G.gnp(38, 0.35, 12002),
    lambda: G.grid(3, 12),
    lambda: G.complete_bipartite(20, 20),
    lambda: G.gnp(44, 0.4, 12008),
    lambda: G.gnp(56, 0.45, 12010),
    lambda: G.gnp(64, 0.5, 12009),
    lambda: G.complete_multipartite([8] * 8),
    lambda: G.path(64),
])
def test_random_graphs_64bit(oracle, ctx, maker):
    """n > 32 (64-bit keys); O4 supplies the levels."""
    rows = maker()
    lb = oracle.mmw(rows)
    tw = oracle.treewidth_bfs(rows, lb)
    got_tw, order, _ = ctx.solve(rows)
    assert got_tw == tw
    assert oracle.order_width(rows, order) == tw
    for k in (tw - 1, tw):
        if k < 0:
            continue
        _, ref_levels, ref_stats = oracle.decide(rows, k)
        _, levels = ctx.trace_decide(rows, k)
        _check_levels(oracle, rows, k, levels, ref_levels, ref_stats)


def test_closed_form_sizes_edgeless(ctx):
    """Edgeless n=24 at k=0: |F_i| = C(24, i) (2.7 M states at the peak), each
    generated (i+1) times — the hash dedup against a closed form."""
    n = 24
    yes, levels = ctx.trace_decide(G.edgeless(n), 0)
    assert yes and len(levels) == n
    for lv in levels:
        assert lv.count == math.comb(n, lv.level)
        if lv.level > 0:
            assert lv.successors == math.comb(n, lv.level - 1) * (n - lv.level + 1)
        assert len(np.unique(lv.states)) == lv.count
        assert np.all(np.bitwise_count(lv.states) == lv.level)


def test_closed_form_counts_64bit(ctx):
    """Every subset is feasible for the edgeless graph at any k and for
    disjoint K_c at k >= c-1, so with L = n-k-1 levels the counts are binomial
    sums.  Edgeless n=40 at k=31 reaches C(40, 8) = 77 M states."""
    n, k = 40, 31
    L = n - k - 1
    yes, st = ctx.decide(G.edgeless(n), k)
    assert yes
    assert st["unique"] == sum(math.comb(n, i) for i in range(1, L + 1))
    assert st["successors"] == sum(math.comb(n, i) * (n - i) for i in range(0, L))
    assert st["expansions"] == st["successors"]
    assert st["peak_frontier"] == math.comb(n, L)
    rows = G.disjoint_cliques(4, 9)
    n = len(rows)
    yes, levels = ctx.trace_decide(rows, 29)
    assert yes
    for lv in levels:
        assert lv.count == math.comb(n, lv.level)
        assert len(np.unique(lv.states)) == lv.count
    yes, st = ctx.decide(rows, 27)
    assert yes and st["peak_frontier"] == math.comb(n, 8)
    yes, levels = ctx.trace_decide(rows, 2)
    assert not yes and levels[1].count == 0 and len(levels) == 2


def test_path_closed_form_levels(ctx):
    """Path on 64 vertices at k=1: the feasible sets of size i are a prefix
    plus a suffix, i+1 of them."""
    yes, levels = ctx.trace_decide(G.path(64), 1)
    assert yes
    for lv in levels:
        assert lv.count == lv.level + 1


@pytest.mark.parametrize("rows,tw", [
    (G.complete(1), 0), (G.complete(2), 1), (G.edgeless(5), 0), (G.complete(12), 11),
    (G.petersen(), 4), (G.complete_bipartite(3, 5), 3), (G.grid(4, 5), 4), (G.cycle(9), 2),
    (G.complete(40), 39), (G.edgeless(20), 0), (G.path(64), 1),
    (G.disjoint_cliques(5, 3), 4),
])
def test_edge_cases_and_closed_forms(oracle, ctx, rows, tw):
    got, order, _ = ctx.solve(rows)
    assert got == tw
    assert oracle.order_width(rows, order) == tw
    n = len(rows)
    assert ctx.decide(rows, n - 1)[0]          # k >= n-1: YES with no level
    if tw > 0:
        assert not ctx.decide(rows, tw - 1)[0]


def test_overflow_regrow_replay_is_exact(oracle, ctx):
    """A tiny first guess forces overflow -> regrow -> replay at every level;
    the levels must be identical and the retries counted."""
    from paper_1709_09990_amd import tw as T
    rows = G.workload_single_small(1001)
    tw, table = oracle.subset_dp(rows)
    with T.Context(device=0, capacity_override=1) as small:
        yes, levels = small.trace_decide(rows, tw)
        assert yes
        _check_levels(oracle, rows, tw, levels, oracle.frontiers_from_dp(rows, tw, table))
        _, st = small.decide(rows, tw)
        assert st["retries"] > 0
        got, order, _ = small.solve(rows)
        assert got == tw and oracle.order_width(rows, order) == tw


def test_capacity_limit_is_an_error(ctx):
    from paper_1709_09990_amd import tw as T
    with T.Context(device=0, max_states=100) as lim:
        with pytest.raises(T.TwError) as e:
            lim.decide(G.edgeless(20), 0)
        assert e.value.status == T.TW_ECAPACITY


def test_invalid_arguments(ctx):
    from paper_1709_09990_amd import tw as T
    with pytest.raises(T.TwError) as e:
        ctx.decide(np.array([0b10, 0b00], dtype=np.uint64), 1)
    assert e.value.status == T.TW_EINVAL
    with pytest.raises(T.TwError) as e:
        ctx.decide(G.path(4), -1)
    assert e.value.status == T.TW_EINVAL


def test_batch_equals_single(oracle, ctx):
    graphs = G.workload_batch(24, seed0=31000, n_lo=8, n_hi=26)
    tws, orders, status, st = ctx.solve_batch(graphs)
    for rows, tw, order, s in zip(graphs, tws, orders, status):
        assert s == 0
        single, _, _ = ctx.solve(rows)
        assert tw == single
        assert oracle.order_width(rows, order) == tw


def _bloom_ctx():
    from paper_1709_09990_amd import tw as T
    return T.Context(device=0, dedup=T.TW_DEDUP_BLOOM)


def test_bloom_levels_subset_of_exact(oracle):
    """Bloom variant (§3.2): every level is a subset of the exact level (false
    positives only drop states), and with m/n >= 24 bits and 17 probes the
    losses stay near the (1 - e^(-17/24))^17 ~ 1e-5 per-insert rate."""
    cases = [(G.workload_single_small(1001), None), (G.edgeless(22), 0), (G.gnp(30, 0.3, 12007), None)]
    with _bloom_ctx() as bctx:
        for rows, k in cases:
            if k is None:
                k = oracle.treewidth_bfs(rows, oracle.mmw(rows))
            _, exact, _ = oracle.decide(rows, k)
            _, levels = bctx.trace_decide(rows, k)
            dropped = 0
            total = 0
            for lv in levels:
                got = np.unique(lv.states)
                ref = exact[lv.level]
                assert np.isin(got, ref).all(), (k, lv.level)
                dropped += len(ref) - len(got)
                total += len(ref)
            assert dropped <= 1e-4 * total + 10, (dropped, total)


def test_bloom_solve_validated(oracle):
    with _bloom_ctx() as bctx:
        for seed in (1001, 1002, 1003):
            rows = G.workload_single_small(seed)
            tw, _ = oracle.subset_dp(rows)
            got, order, _ = bctx.solve(rows)
            # a Bloom answer is an upper bound proved by its order; here it is exact
            assert oracle.order_width(rows, order) == got
            assert got == tw


def test_batch_persistent_matches_oracle(oracle):
    """One persistent launch over graphs of uneven n (8..30): every treewidth
    equals the oracle's and every order has exactly that width."""
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(96, seed0=32000, n_lo=8, n_hi=30)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    with T.Context(device=0, timing=True) as c:
        tws, orders, status, st = c.solve_batch(graphs)
    assert list(status) == [0] * len(graphs)
    assert list(tws) == want
    for rows, tw, order in zip(graphs, tws, orders):
        assert oracle.order_width(rows, order) == tw
    assert st["launches"] >= 1


def test_batch_fallback_on_small_arena(oracle):
    """A tiny per-graph arena forces graphs out of the persistent launch onto
    the single-graph path; answers are unchanged."""
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(24, seed0=33000, n_lo=12, n_hi=28)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    with T.Context(device=0, batch_graph_states=512, batch_chunk=64) as c:
        tws, orders, status, _ = c.solve_batch(graphs)
    assert list(status) == [0] * len(graphs)
    assert list(tws) == want
    for rows, tw, order in zip(graphs, tws, orders):
        assert oracle.order_width(rows, order) == tw


@pytest.mark.parametrize("seed", [0, 1])
def test_learned_start_is_exact(oracle, tmp_path, seed):
    """The learned start bound only changes where the search begins: with any
    network (here an untrained one, so predictions land above and below tw)
    the batched and single answers equal the oracle's, orders have that width,
    and the per-graph start bounds differ from the plain lower bounds."""
    from oracle import mpnn_ref as M
    from paper_1709_09990_amd import tw as T
    p = M.flatten(M.init_params(100 + seed)).astype(np.float32)
    # bias the tw head so the start lands well inside [lb, n-2]
    p[-2] = 0.45 if seed == 0 else 0.2
    wpath = str(tmp_path / "w.bin")
    T.write_weights(wpath, p)
    graphs = G.workload_batch(40, seed0=34000 + 100 * seed, n_lo=8, n_hi=26)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    with T.Context(device=0, k_policy=T.TW_K_LEARNED, weights_path=wpath) as c:
        tws, orders, status, st, per = c.solve_batch(graphs, graph_stats=True)
        assert list(status) == [0] * len(graphs)
        assert list(tws) == want
        for rows, tw, order in zip(graphs, tws, orders):
            assert oracle.order_width(rows, order) == tw
        starts = [q["start_k"] for q in per]
        assert any(s != T.mmw(r) for s, r in zip(starts, graphs))
        for rows, tw in list(zip(graphs, want))[:8]:
            got, order, _ = c.solve(rows)
            assert got == tw and oracle.order_width(rows, order) == tw


def test_batch_graph_stats_peak(oracle):
    """Per-graph peak of the certifying run equals the oracle's largest level
    of decide(tw)."""
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(16, seed0=35000, n_lo=8, n_hi=22)
    with T.Context(device=0) as c:
        tws, _, status, _, per = c.solve_batch(graphs, graph_stats=True)
    for rows, tw, q in zip(graphs, tws, per):
        _, levels, _ = oracle.decide(rows, int(tw))
        assert q["peak_yes"] == max(len(f) for f in levels)


def test_autotune_candidates_agree(tmp_path, monkeypatch):
    """Every autotuner candidate (task size, load factor, probe scheme) gives
    the same answers; the tuned choice is cached and reused."""
    from paper_1709_09990_amd import autotune
    monkeypatch.setenv("TW_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    graphs = G.workload_batch(24, seed0=36000, n_lo=10, n_hi=22)
    opts = autotune.tuned_options(graphs, sample=24)
    assert set(opts) == {"batch_chunk", "load_factor", "probe"}
    assert autotune.tuned_options(graphs) == opts


@pytest.mark.parametrize("maker", [
    lambda: G.workload_single_small(1001),
    lambda: G.gnp(26, 0.2, 13001),
    lambda: G.gnp(38, 0.35, 12002),
    lambda: G.grid(3, 12),
    lambda: G.gnp(56, 0.45, 12010),
])
def test_partitioned_insert_levels_match(oracle, maker):
    """The two-phase insert (expand + scatter by hash range, then insert
    partition by partition), forced at small sizes: every level equals the
    oracle's, with the same feasible-pair counts; also under overflow replay."""
    from paper_1709_09990_amd import tw as T
    rows = maker()
    tw = oracle.treewidth_bfs(rows, oracle.mmw(rows))
    for kw in ({"partition": 2}, {"partition": 2, "capacity_override": 7}):
        with T.Context(device=0, **kw) as c:
            got, order, _ = c.solve(rows)
            assert got == tw and oracle.order_width(rows, order) == tw
            for k in (tw - 1, tw):
                if k < 0:
                    continue
                _, ref_levels, ref_stats = oracle.decide(rows, k)
                _, levels = c.trace_decide(rows, k)
                _check_levels(oracle, rows, k, levels, ref_levels, ref_stats)


def test_probe_rate_reference():
    """The random-access reference kernel runs in every mode and rejects bad arguments."""
    from paper_1709_09990_amd import tw as T
    for mode in range(6):
        r = T.probe_rate(64 << 20, 1 << 22, mode)
        assert math.isfinite(r) and r > 1e6, (mode, r)
    for bad in ((64 << 20, 1 << 22, 6), (64 << 20, 1 << 22, -1), (1024, 1 << 22, 0), (64 << 20, 0, 0)):
        with pytest.raises(T.TwError):
            T.probe_rate(*bad)


def test_bloom_certified_answers_are_exact(oracle):
    """Bloom search whose NO answers are re-decided exactly (§3.2 filter, exact
    certificate): every answer equals the oracle's."""
    from paper_1709_09990_amd import tw as T
    graphs = [G.gnp(20, 0.3, 8100 + s) for s in range(4)] + [G.partial_ktree(34, 5, 0.3, 8200)]
    with T.Context(device=0, dedup=T.TW_DEDUP_BLOOM_CERTIFIED) as c:
        for rows in graphs:
            tw = oracle.treewidth_bfs(rows, oracle.mmw(rows))
            for k in (tw - 1, tw):
                assert c.decide(rows, k)[0] == (k >= tw)
            got, order, _ = c.solve(rows)
            assert got == tw and oracle.order_width(rows, order) == tw
        tws, _, status, _ = c.solve_batch(graphs)
        assert list(status) == [0] * len(graphs)
        assert list(tws) == [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]


def test_invalid_options_rejected():
    from paper_1709_09990_amd import tw as T
    for kw in ({"dedup": 5}, {"reductions": 3}, {"batch_schedule": 3}):
        with pytest.raises(T.TwError) as e:
            T.Context(device=0, **kw)
        assert e.value.status == T.TW_EINVAL


def test_batch_rounds_many_graphs(oracle):
    """More graphs than one plan tile (1024): the level-round schedule and the
    persistent queue both give the oracle's treewidths."""
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(1100, seed0=39000, n_lo=6, n_hi=13)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    for sched in (T.TW_BATCH_ROUNDS, T.TW_BATCH_PERSISTENT):
        with T.Context(device=0, batch_schedule=sched) as c:
            tws, orders, status, _ = c.solve_batch(graphs)
        assert list(status) == [0] * len(graphs)
        assert list(tws) == want, sched
        for rows, tw, order in list(zip(graphs, tws, orders))[::50]:
            assert oracle.order_width(rows, order) == tw


def test_batch_mixed_sizes_up_to_64(oracle):
    """Graphs above the batched limit (n > 48) go through the single-graph path
    inside the same call; trivial graphs (tw = n - 1) need no search."""
    from paper_1709_09990_amd import tw as T
    small = [G.gnp(18, 0.3, 9100), G.gnp(20, 0.25, 9102)]
    graphs = [G.path(64), G.path(49), G.complete(5), small[0], G.edgeless(1), small[1]]
    want = [1, 1, 4, oracle.subset_dp(small[0])[0], 0, oracle.subset_dp(small[1])[0]]
    for sched in (T.TW_BATCH_ROUNDS, T.TW_BATCH_PERSISTENT):
        with T.Context(device=0, batch_schedule=sched) as c:
            tws, orders, status, _, per = c.solve_batch(graphs, graph_stats=True)
        assert list(status) == [0] * len(graphs)
        assert list(tws) == want
        for rows, tw, order in zip(graphs, tws, orders):
            assert oracle.order_width(rows, order) == tw
        assert [q["path"] for q in per][:3] == [1, 1, 2]


def test_degenerate_inputs(ctx):
    """An empty batch, the largest n (64) at its extreme bounds, a single vertex."""
    tws, orders, status, st = ctx.solve_batch([])
    assert len(tws) == 0 and len(status) == 0
    K64 = G.complete(64)
    assert ctx.decide(K64, 63)[0] is True      # k >= n - 1: YES with no level
    assert ctx.decide(K64, 62)[0] is False     # one level of 64 states, none feasible
    tw, order, _ = ctx.solve(K64)
    assert tw == 63 and sorted(order) == list(range(64))
    tw, order, _ = ctx.solve(G.edgeless(1))
    assert tw == 0 and list(order) == [0]
