"""The caller's device range (options.workspace) and the overflow hook
(options.fault_inject_level) of the C-ABI.

With a workspace every device buffer of the context is carved from the
caller's range: the levels must be exactly those of a context that allocates
its own memory, and a range too small for a level must give TW_ENOMEM, never
a wrong answer.  The overflow hook forces the regrow -> replay path of the
level loop (no answer is ever traded for memory, §3.1 levels kept exact): the
replayed levels equal the oracle's, retries are counted, and a replay that
cannot grow past max_states fails with TW_ECAPACITY.
"""
import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu


def _levels(ctx, rows, k):
    yes, levels = ctx.trace_decide(rows, k)
    return yes, [(lv.level, lv.count, lv.successors, np.sort(lv.states).tobytes()) for lv in levels]


class _DeviceRange:
    """A caller-owned device buffer from the HIP runtime the library uses
    (hipMalloc / hipFree through ctypes)."""

    def __init__(self, nbytes):
        import ctypes
        from paper_1709_09990_amd import tw as T
        T.load()
        self._hip = ctypes.CDLL("libamdhip64.so.7", mode=ctypes.RTLD_GLOBAL)
        self.ptr = ctypes.c_void_p()
        assert self._hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(nbytes)) == 0

    def free(self):
        if self.ptr:
            self._hip.hipFree(self.ptr)
            self.ptr = None


def _device_range(nbytes):
    r = _DeviceRange(nbytes)
    return r, r.ptr.value


def test_workspace_levels_equal_own_memory(oracle):
    from paper_1709_09990_amd import tw as T
    cases = [(G.workload_single_small(1001), None), (G.gnp(30, 0.2, 51001), None),
             (G.partial_ktree(36, 6, 0.3, 51002), None)]
    buf, ptr = _device_range(1 << 30)
    with T.Context(device=0) as own, T.Context(device=0, workspace=ptr, workspace_bytes=1 << 30) as ws:
        for rows, k in cases:
            if k is None:
                k = oracle.treewidth_bfs(rows, oracle.mmw(rows))
            print(f"workspace case n={len(rows)} k={k}", flush=True)
            assert _levels(ws, rows, k) == _levels(own, rows, k)
            tw_ws, order_ws, _ = ws.solve(rows)
            tw_own, _, _ = own.solve(rows)
            assert tw_ws == tw_own == k
            assert oracle.order_width(rows, order_ws) == k
    buf.free()


def test_workspace_batch_and_too_small(oracle):
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(32, seed0=52000, n_lo=10, n_hi=24)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    buf, ptr = _device_range(256 << 20)
    with T.Context(device=0, workspace=ptr, workspace_bytes=256 << 20) as ws:
        tws, orders, status, _ = ws.solve_batch(graphs)
        assert list(status) == [0] * len(graphs) and list(tws) == want
        for rows, tw, order in zip(graphs, tws, orders):
            assert oracle.order_width(rows, order) == tw
    # 1 MiB cannot hold the levels of G(30, 0.2) at its treewidth: an error, not an answer
    small, sptr = _device_range(1 << 20)
    rows = G.gnp(30, 0.2, 51001)
    k = oracle.treewidth_bfs(rows, oracle.mmw(rows))
    with T.Context(device=0, workspace=sptr, workspace_bytes=1 << 20) as tiny:
        with pytest.raises(T.TwError) as e:
            tiny.decide(rows, k)
        assert e.value.status == T.TW_ENOMEM
        # the context stays usable for what fits
        yes, _ = tiny.decide(G.path(12), 1)
        assert yes
    buf.free()
    small.free()


@pytest.mark.parametrize("level", [1, 4, 9])
def test_fault_inject_replays_exact_levels(oracle, level):
    from paper_1709_09990_amd import tw as T
    rows = G.gnp(28, 0.2, 53001)
    k = oracle.treewidth_bfs(rows, oracle.mmw(rows))
    _, ref, _ = oracle.decide(rows, k)
    with T.Context(device=0, fault_inject_level=level) as c:
        yes, levels = c.trace_decide(rows, k)
        assert yes
        for lv in levels:
            assert np.array_equal(np.sort(lv.states), ref[lv.level]), lv.level
        yes2, st = c.decide(rows, k)
        assert yes2 and st["retries"] >= 1
        tw, order, st2 = c.solve(rows)
        assert tw == k and oracle.order_width(rows, order) == k
        assert st2["retries"] >= 1


def test_fault_inject_capacity_error(oracle):
    """max_states equal to the largest level lets decide(k) through, but not
    when that level's first build is forced to overflow: the replay cannot
    grow past the cap, so the call fails with TW_ECAPACITY."""
    from paper_1709_09990_amd import tw as T
    rows = G.gnp(28, 0.2, 53001)
    k = oracle.treewidth_bfs(rows, oracle.mmw(rows))
    _, ref, _ = oracle.decide(rows, k)
    sizes = [len(x) for x in ref]
    peak = max(sizes)
    level = sizes.index(peak)
    assert level >= 2 and peak > 1
    with T.Context(device=0, max_states=peak, capacity_override=peak) as c:
        yes, st = c.decide(rows, k)
        assert yes and st["retries"] == 0
    with T.Context(device=0, max_states=peak, capacity_override=peak, fault_inject_level=level) as c:
        with pytest.raises(T.TwError) as e:
            c.decide(rows, k)
        assert e.value.status == T.TW_ECAPACITY


def test_fault_inject_batch_falls_back(oracle):
    """In the batched search a graph reaching the injected level leaves the
    batch for the single-graph path (whose replay rebuilds the level); every
    answer is unchanged."""
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(24, seed0=54000, n_lo=12, n_hi=24)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    with T.Context(device=0, fault_inject_level=3) as c:
        tws, orders, status, st, per = c.solve_batch(graphs, graph_stats=True)
    assert list(status) == [0] * len(graphs) and list(tws) == want
    for rows, tw, order in zip(graphs, tws, orders):
        assert oracle.order_width(rows, order) == tw
    # every graph whose bounds reach level 3 went to the single-graph path
    assert sum(1 for p in per if p["path"] == 1) >= 20
    assert st["retries"] >= 1


def test_batch_memory_shortfall_falls_back(oracle):
    """Batch arenas too large for the device (2^35 states per graph): the
    batched launch cannot get its memory, and its graphs are solved on the
    single-graph path instead of failing the call; every answer is returned."""
    from paper_1709_09990_amd import tw as T
    graphs = G.workload_batch(12, seed0=55000, n_lo=12, n_hi=22)
    want = [oracle.treewidth_bfs(r, oracle.mmw(r)) for r in graphs]
    with T.Context(device=0, batch_graph_states=1 << 35) as c:
        tws, orders, status, _, per = c.solve_batch(graphs, graph_stats=True)
    assert list(status) == [0] * len(graphs) and list(tws) == want
    assert all(p["path"] in (1, 2) for p in per)
    for rows, tw, order in zip(graphs, tws, orders):
        assert oracle.order_width(rows, order) == tw
