"""tw_solve_noalloc, the entry point for callers that cannot allocate: every
device buffer of the call lies in the library's static scratch.  Its answers
and work counters must equal tw_solve's (Listing 1 with exact duplicate
removal, §3.1), call after call on the same scratch, the second call on a
smaller graph; sizes beyond its limits are errors."""
import pytest

from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu

KEYS = ("expansions", "successors", "unique", "states_expanded", "peak_frontier", "decisions", "levels")


def test_noalloc_equals_solve(oracle):
    """Calls in a row on one context, each graph smaller than the one before
    (n 30, 28, 20, 9).  The levels of the n <= 28 graphs fit the scratch's
    share for kept levels, so the work counters match tw_solve's exactly; G(30,
    0.15) keeps only two levels in the scratch and rebuilds its order by the
    restricted re-run, so only its answer and order are compared."""
    from paper_1709_09990_amd import tw as T
    cases = [(G.gnp(30, 0.15, 61002), False), (G.gnp(28, 0.2, 61001), True),
             (G.workload_single_small(1001), True), (G.cycle(9), True)]
    with T.Context(device=0) as c:
        for rows, same_work in cases:
            print(f"noalloc n={len(rows)}", flush=True)
            tw_a, order_a, st_a = c.solve_noalloc(rows)
            tw_b, order_b, st_b = c.solve(rows)
            assert tw_a == tw_b == oracle.treewidth_bfs(rows, oracle.mmw(rows))
            assert oracle.order_width(rows, order_a) == tw_a
            if same_work:
                for key in KEYS:
                    assert st_a[key] == st_b[key], key


def test_noalloc_limits():
    from paper_1709_09990_amd import tw as T
    with T.Context(device=0) as c:
        with pytest.raises(T.TwError) as e:
            c.solve_noalloc(G.path(33))
        assert e.value.status == T.TW_EINVAL
        # every subset of 32 isolated vertices is a state at bound 0: far beyond 64 MiB
        with pytest.raises(T.TwError) as e:
            c.solve_noalloc(G.edgeless(32))
        assert e.value.status == T.TW_ECAPACITY
        # the context and the scratch stay usable
        tw, order, _ = c.solve_noalloc(G.cycle(12))
        assert tw == 2
        tw2, _, _ = c.solve(G.cycle(12))
        assert tw2 == 2
