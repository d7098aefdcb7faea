"""The C-ABI library loads and exports every function include/tw.h declares;
host-only entry points (validation, minor-min-width, fill-in width) agree with
the oracle.  No device call is made here."""
import ctypes
import os
import random
import re

import numpy as np
import pytest

from paper_1709_09990_amd import graphs as G
from paper_1709_09990_amd import tw as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "tw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(tw_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    names = _header_functions()
    assert "tw_decide" in names and "tw_solve" in names and "tw_solve_batch" in names
    assert set(names) == set(T.EXPORTS)
    lib = ctypes.CDLL(T.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    L = T.load()
    for s in range(5):
        assert L.tw_status_str(s)


def test_mmw_matches_oracle(oracle):
    rng = random.Random(21)
    for t in range(300):
        n = rng.randint(1, 40)
        rows = G.gnp(n, rng.uniform(0.05, 0.7), 7000 + t)
        assert T.mmw(rows) == oracle.mmw(rows), t
    for t in range(40):
        rows = G.partial_ktree(20 + t, 4 + t % 6, 0.3, 7500 + t)
        assert T.mmw(rows) == oracle.mmw(rows)
    for rows in G.workload_single_n40().values():
        assert T.mmw(rows) == oracle.mmw(rows)
    assert T.mmw(G.complete(64)) == oracle.mmw(G.complete(64)) == 63


def test_order_width_matches_oracle(oracle):
    rng = random.Random(22)
    for t in range(300):
        n = rng.randint(1, 64)
        rows = G.gnp(n, rng.uniform(0.02, 0.4), 8000 + t)
        order = list(range(n))
        rng.shuffle(order)
        assert T.order_width(rows, order) == oracle.order_width(rows, order)
    assert T.order_width(G.path(3), [0, 0, 1]) == -1


@pytest.mark.parametrize("rows", [
    np.array([0b10, 0b00], dtype=np.uint64),          # not symmetric
    np.array([0b01], dtype=np.uint64),                # self-loop
    np.array([0b100, 0b000], dtype=np.uint64),        # bit beyond n
    np.zeros(0, dtype=np.uint64),                     # n = 0
])
def test_invalid_graphs_rejected_on_host(rows):
    with pytest.raises(T.TwError) as e:
        T.mmw(rows)
    assert e.value.status == T.TW_EINVAL


def test_network_features_match_reference():
    """Node features of the learned start bound, host side, against the
    independent reference implementation (degree and core number)."""
    from oracle import mpnn_ref as M
    for t in range(40):
        rows = G.workload_batch(1, seed0=9000 + t, n_lo=5, n_hi=64)[0]
        X, _, _ = M.features(rows)
        got = T.mpnn_features(rows)
        assert np.allclose(got, X[:, :4].astype(np.float32))
    assert T.mpnn_param_count() == M.N_PARAMS


def test_reductions_match_oracle():
    """Host prep of the §3.1 reductions (clique, disjoint-path counts) equals
    the oracle's independent implementation."""
    from oracle import reductions as R
    rng = random.Random(23)
    graphs = [G.grid(4, 5), G.petersen(), G.cycle(11), G.complete(6), G.edgeless(4),
              G.complete_bipartite(3, 6), G.complete_multipartite([2, 3, 4]), G.disjoint_cliques(3, 3)]
    graphs += [G.gnp(rng.randint(8, 24), rng.choice([0.15, 0.3, 0.5]), 1200 + s) for s in range(16)]
    graphs += [G.partial_ktree(rng.randint(10, 26), rng.randint(3, 7), 0.3, 1300 + s) for s in range(8)]
    graphs += [G.rgg(rng.randint(10, 26), 6.0, 1400 + s) for s in range(6)]
    w = G.workload_single_n40()
    graphs += [w["gnp40_p015"], w["partial8tree40"]]
    for rows in graphs:
        clique, paths = T.reductions(rows)
        assert clique == R.max_clique(rows)
        assert np.array_equal(paths.astype(np.int32), np.minimum(R.disjoint_paths(rows), 255))


def test_tree_decomposition_from_orders(oracle):
    """tw_tree_decomposition on optimal orders (oracle brute force) and on
    random orders: a valid decomposition whose width is the order's width."""
    rng = random.Random(31)
    graphs = [G.petersen(), G.grid(3, 3), G.cycle(7), G.complete_bipartite(2, 4), G.disjoint_cliques(3, 2)]
    graphs += [G.gnp(rng.randint(5, 9), 0.4, 1500 + s) for s in range(10)]
    for rows in graphs:
        n = len(rows)
        tw, best = oracle.brute_force(rows)
        bags, parent, width = T.tree_decomposition(rows, best)
        assert width == tw == oracle.decomposition_width(bags)
        assert oracle.is_tree_decomposition(rows, bags, parent)
        for _ in range(5):
            order = list(range(n))
            rng.shuffle(order)
            bags, parent, width = T.tree_decomposition(rows, order)
            assert width == oracle.order_width(rows, order)
            assert oracle.is_tree_decomposition(rows, bags, parent)
    with pytest.raises(T.TwError):
        T.tree_decomposition(G.path(3), [0, 0, 1])


def test_invalid_options_rejected_before_any_device_call():
    """tw_ctx_create validates the option enums before touching a device, so
    a bad value is TW_EINVAL even on a machine without a GPU."""
    bad = [dict(dedup=7), dict(reductions=3), dict(batch_schedule=3), dict(batch_schedule=-1),
           dict(mmw_prune=2), dict(mmw_prune=-1)]
    for kw in bad:
        with pytest.raises(T.TwError) as e:
            T.Context(device=0, **kw)
        assert e.value.status == T.TW_EINVAL, kw


def test_batch_schedule_values():
    """The batch schedule enum: the automatic choice is 0, the zero a
    zero-initialised options struct carries, and the binding's default."""
    import inspect
    assert (T.TW_BATCH_AUTO, T.TW_BATCH_ROUNDS, T.TW_BATCH_PERSISTENT) == (0, 1, 2)
    assert inspect.signature(T.Context.__init__).parameters["batch_schedule"].default == T.TW_BATCH_AUTO
    hdr = open(os.path.join(ROOT, "include", "tw.h")).read()
    assert "enum { TW_BATCH_AUTO = 0, TW_BATCH_ROUNDS = 1, TW_BATCH_PERSISTENT = 2 };" in hdr
