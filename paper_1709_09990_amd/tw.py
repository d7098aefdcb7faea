"""ctypes binding of libtw.so (include/tw.h): argument marshalling only.

Every step of the search runs in the HIP library; this module converts numpy
arrays to pointers and status codes to exceptions.  If the library has not
been built, every call raises — there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtw.so")

TW_OK, TW_EINVAL, TW_ENOMEM, TW_EDEVICE, TW_ECAPACITY = range(5)
TW_DEDUP_EXACT, TW_DEDUP_BLOOM, TW_DEDUP_BLOOM_CERTIFIED = 0, 1, 2
TW_K_ASCENDING, TW_K_LEARNED = 0, 1
TW_REDUCE_NONE, TW_REDUCE_CLIQUE_PATHS = 0, 1
TW_BATCH_AUTO, TW_BATCH_ROUNDS, TW_BATCH_PERSISTENT = 0, 1, 2
TW_MMW_NONE, TW_MMW_PRUNE = 0, 1
TW_CAPTURE_AUTO, TW_CAPTURE_OFF = 0, 1


class TwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tw status {status}: {msg}")
        self.status = status


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("adj", ctypes.POINTER(ctypes.c_uint64))]


class _Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_size_t),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("dedup", ctypes.c_int),
        ("load_factor", ctypes.c_float),
        ("k_policy", ctypes.c_int),
        ("weights_path", ctypes.c_char_p),
        ("max_states", ctypes.c_uint64),
        ("capacity_override", ctypes.c_uint64),
        ("timing", ctypes.c_int),
        ("probe", ctypes.c_int),
        ("partition", ctypes.c_int),
        ("batch_graph_states", ctypes.c_uint64),
        ("batch_chunk", ctypes.c_uint32),
        ("batch_schedule", ctypes.c_int),
        ("reductions", ctypes.c_int),
        ("mmw_prune", ctypes.c_int),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("fault_inject_level", ctypes.c_int),
        ("capture", ctypes.c_int),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("states_expanded", ctypes.c_uint64),
        ("expansions", ctypes.c_uint64),
        ("successors", ctypes.c_uint64),
        ("unique", ctypes.c_uint64),
        ("peak_frontier", ctypes.c_uint64),
        ("decisions", ctypes.c_uint32),
        ("levels", ctypes.c_uint32),
        ("retries", ctypes.c_uint32),
        ("launches", ctypes.c_uint32),
        ("seconds", ctypes.c_double),
        ("kernel_seconds", ctypes.c_double),
    ]


class _LevelRecord(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("level", ctypes.c_int32),
        ("count", ctypes.c_uint64),
        ("expansions", ctypes.c_uint64),
        ("successors", ctypes.c_uint64),
        ("states", ctypes.POINTER(ctypes.c_uint64)),
        ("last_v", ctypes.POINTER(ctypes.c_uint8)),
    ]


class _GraphStats(ctypes.Structure):
    _fields_ = [
        ("peak_yes", ctypes.c_uint64),
        ("expansions", ctypes.c_uint64),
        ("states_expanded", ctypes.c_uint64),
        ("start_k", ctypes.c_int32),
        ("decisions", ctypes.c_uint32),
        ("path", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("peak_any", ctypes.c_uint64),
    ]


class _BatchLevel(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("level", ctypes.c_int32),
        ("count", ctypes.c_uint64),
        ("successors", ctypes.c_uint64),
        ("digest_sum", ctypes.c_uint64),
        ("digest_xor", ctypes.c_uint64),
    ]


_SINK = ctypes.CFUNCTYPE(None, ctypes.POINTER(_LevelRecord), ctypes.c_void_p)

# every function declared in include/tw.h
EXPORTS = (
    "tw_ctx_create", "tw_ctx_destroy", "tw_decide", "tw_solve", "tw_solve_batch",
    "tw_trace_decide", "tw_mmw", "tw_order_width", "tw_status_str", "tw_last_error",
    "tw_mpnn_param_count", "tw_mpnn_features", "tw_mpnn_create", "tw_mpnn_destroy",
    "tw_mpnn_set_params", "tw_mpnn_get_params", "tw_mpnn_predict", "tw_mpnn_gradients",
    "tw_mpnn_train_step", "tw_probe_rate", "tw_reductions", "tw_tree_decomposition",
    "tw_trace_batch", "tw_solve_noalloc", "tw_mpnn_trace_floats", "tw_mpnn_trace",
    "tw_decide128", "tw_solve128", "tw_trace_decide128", "tw_mmw128", "tw_order_width128",
)

_lib = None


def load():
    """Load libtw.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(python -m paper_1709_09990_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.tw_ctx_create.argtypes = [P(_Options), P(ctypes.c_void_p)]
    L.tw_ctx_destroy.argtypes = [ctypes.c_void_p]
    L.tw_ctx_destroy.restype = None
    L.tw_decide.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_int32, P(ctypes.c_int32), P(_Stats)]
    L.tw_solve.argtypes = [ctypes.c_void_p, P(_Graph), P(ctypes.c_int32), P(ctypes.c_int32), P(_Stats)]
    L.tw_solve_noalloc.argtypes = [ctypes.c_void_p, P(_Graph), P(ctypes.c_int32), P(ctypes.c_int32), P(_Stats)]
    L.tw_solve_batch.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_uint32, P(ctypes.c_int32),
                                 P(ctypes.c_int32), P(ctypes.c_int), P(_GraphStats), P(_Stats)]
    L.tw_trace_decide.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_int32, _SINK, ctypes.c_void_p,
                                  P(ctypes.c_int32)]
    L.tw_trace_batch.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                 P(_BatchLevel), P(ctypes.c_uint32), P(ctypes.c_int32), P(ctypes.c_int32),
                                 P(ctypes.c_int), P(_GraphStats)]
    L.tw_mmw.argtypes = [P(_Graph), P(ctypes.c_int32)]
    L.tw_order_width.argtypes = [P(_Graph), P(ctypes.c_int32), P(ctypes.c_int32)]
    L.tw_tree_decomposition.argtypes = [P(_Graph), P(ctypes.c_int32), P(ctypes.c_uint64), P(ctypes.c_int32),
                                        P(ctypes.c_int32)]
    L.tw_reductions.argtypes = [P(_Graph), P(ctypes.c_uint64), P(ctypes.c_uint8)]
    L.tw_probe_rate.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                P(ctypes.c_double)]
    L.tw_status_str.argtypes = [ctypes.c_int]
    L.tw_status_str.restype = ctypes.c_char_p
    L.tw_last_error.argtypes = [ctypes.c_void_p]
    L.tw_last_error.restype = ctypes.c_char_p
    f32p = P(ctypes.c_float)
    L.tw_mpnn_param_count.argtypes = []
    L.tw_mpnn_param_count.restype = ctypes.c_uint32
    L.tw_mpnn_features.argtypes = [P(_Graph), f32p]
    L.tw_mpnn_create.argtypes = [ctypes.c_int, ctypes.c_void_p, f32p, P(ctypes.c_void_p)]
    L.tw_mpnn_destroy.argtypes = [ctypes.c_void_p]
    L.tw_mpnn_destroy.restype = None
    L.tw_mpnn_set_params.argtypes = [ctypes.c_void_p, f32p]
    L.tw_mpnn_get_params.argtypes = [ctypes.c_void_p, f32p]
    L.tw_mpnn_predict.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_uint32, f32p]
    L.tw_mpnn_gradients.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_uint32, f32p, f32p, f32p]
    L.tw_decide128.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_int32, P(ctypes.c_int32), P(_Stats)]
    L.tw_solve128.argtypes = [ctypes.c_void_p, P(_Graph), P(ctypes.c_int32), P(ctypes.c_int32), P(_Stats)]
    L.tw_trace_decide128.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_int32, _SINK, ctypes.c_void_p,
                                     P(ctypes.c_int32)]
    L.tw_mmw128.argtypes = [P(_Graph), P(ctypes.c_int32)]
    L.tw_order_width128.argtypes = [P(_Graph), P(ctypes.c_int32), P(ctypes.c_int32)]
    for name in ("tw_decide128", "tw_solve128", "tw_trace_decide128", "tw_mmw128", "tw_order_width128"):
        getattr(L, name).restype = ctypes.c_int
    L.tw_mpnn_trace_floats.argtypes = []
    L.tw_mpnn_trace_floats.restype = ctypes.c_uint32
    L.tw_mpnn_trace.argtypes = [ctypes.c_void_p, P(_Graph), f32p, f32p, f32p]
    L.tw_mpnn_trace.restype = ctypes.c_int
    L.tw_mpnn_train_step.argtypes = [ctypes.c_void_p, P(_Graph), ctypes.c_uint32, f32p, ctypes.c_float,
                                     ctypes.c_float, f32p]
    for name in ("tw_ctx_create", "tw_decide", "tw_solve", "tw_solve_batch", "tw_trace_decide",
                 "tw_mmw", "tw_order_width", "tw_mpnn_features", "tw_mpnn_create", "tw_mpnn_set_params",
                 "tw_mpnn_get_params", "tw_mpnn_predict", "tw_mpnn_gradients", "tw_mpnn_train_step",
                 "tw_probe_rate", "tw_reductions", "tw_tree_decomposition", "tw_trace_batch",
                 "tw_solve_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _graph128(rows):
    """A graph of up to 126 vertices from rows given as Python integers (or
    anything int() accepts): two words per row, low then high."""
    n = len(rows)
    words = np.zeros(max(1, 2 * n), dtype=np.uint64)
    for i, r in enumerate(rows):
        r = int(r)
        words[2 * i] = r & (2**64 - 1)
        words[2 * i + 1] = (r >> 64) & (2**64 - 1)
    g = _Graph()
    g.n = n
    g.adj = words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    return g, words


def _graph(rows):
    a = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
    g = _Graph(len(a), a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return g, a


def _stats_dict(s: _Stats) -> dict:
    return {name: getattr(s, name) for name, _ in _Stats._fields_}


def mmw(rows) -> int:
    L = load()
    g, keep = _graph(rows)
    out = ctypes.c_int32(0)
    st = L.tw_mmw(ctypes.byref(g), ctypes.byref(out))
    if st != TW_OK:
        raise TwError(st, L.tw_status_str(st).decode())
    return out.value


def reductions(rows) -> tuple[list[int], np.ndarray]:
    """(maximum clique skipped by TW_REDUCE_CLIQUE_PATHS, n x n disjoint-path counts)."""
    L = load()
    g, keep = _graph(rows)
    n = len(keep)
    clique = ctypes.c_uint64(0)
    paths = np.zeros(n * n, dtype=np.uint8)
    st = L.tw_reductions(ctypes.byref(g), ctypes.byref(clique), paths.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if st != TW_OK:
        raise TwError(st, L.tw_status_str(st).decode())
    return [v for v in range(n) if (clique.value >> v) & 1], paths.reshape(n, n)


def tree_decomposition(rows, order) -> tuple[list[int], list[int], int]:
    """(bags as vertex masks, parent per bag or -1, width) from an elimination order."""
    L = load()
    g, keep = _graph(rows)
    n = len(keep)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    bags = np.zeros(n, dtype=np.uint64)
    parent = np.zeros(n, dtype=np.int32)
    width = ctypes.c_int32(0)
    st = L.tw_tree_decomposition(ctypes.byref(g), o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 bags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 parent.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(width))
    if st != TW_OK:
        raise TwError(st, L.tw_status_str(st).decode())
    return [int(b) for b in bags], [int(p) for p in parent], width.value


def order_width(rows, order) -> int:
    L = load()
    g, keep = _graph(rows)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    out = ctypes.c_int32(0)
    st = L.tw_order_width(ctypes.byref(g), o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          ctypes.byref(out))
    if st != TW_OK:
        raise TwError(st, L.tw_status_str(st).decode())
    return out.value


def probe_rate(bytes_: int, count: int, mode: int = 0, device: int = 0) -> float:
    """Random operations per second on a device buffer of bytes_ bytes (see
    tw_probe_rate: mode 0 random 16-byte loads, 1 random 64-bit CAS, 2 loads
    with eight in flight per lane)."""
    L = load()
    sec = ctypes.c_double(0.0)
    st = L.tw_probe_rate(int(device), int(bytes_), int(count), int(mode), ctypes.byref(sec))
    if st != TW_OK:
        raise TwError(st, L.tw_status_str(st).decode())
    return count / sec.value


@dataclass
class Level:
    k: int
    level: int
    count: int
    expansions: int
    successors: int
    states: np.ndarray
    last_v: np.ndarray


class Context:
    """A device context (one host thread at a time)."""

    def __init__(self, device: int = 0, stream=None, dedup: int = TW_DEDUP_EXACT,
                 load_factor: float = 0.0, max_states: int = 0, capacity_override: int = 0,
                 timing: bool = False, k_policy: int = TW_K_ASCENDING, weights_path: str | None = None,
                 batch_graph_states: int = 0, batch_chunk: int = 0, probe: int = 0, partition: int = 0,
                 reductions: int = TW_REDUCE_NONE, batch_schedule: int = TW_BATCH_AUTO,
                 mmw_prune: int = TW_MMW_NONE, workspace: int = 0, workspace_bytes: int = 0,
                 fault_inject_level: int = 0, capture: int = 0):
        L = load()
        self._L = L
        o = _Options()
        o.struct_size = ctypes.sizeof(_Options)
        o.device = device
        o.stream = ctypes.c_void_p(stream) if stream else None
        o.dedup = dedup
        o.load_factor = load_factor
        o.k_policy = k_policy
        self._wp = weights_path.encode() if weights_path else None
        o.weights_path = self._wp
        o.max_states = max_states
        o.capacity_override = capacity_override
        o.timing = 1 if timing else 0
        o.probe = probe
        o.partition = partition
        o.batch_graph_states = batch_graph_states
        o.batch_chunk = batch_chunk
        o.reductions = reductions
        o.mmw_prune = mmw_prune
        o.batch_schedule = batch_schedule
        o.workspace = ctypes.c_void_p(workspace) if workspace else None
        o.workspace_bytes = workspace_bytes
        o.fault_inject_level = fault_inject_level
        o.capture = capture
        h = ctypes.c_void_p()
        st = L.tw_ctx_create(ctypes.byref(o), ctypes.byref(h))
        if st != TW_OK:
            raise TwError(st, "tw_ctx_create: " + L.tw_status_str(st).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.tw_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int):
        if st != TW_OK:
            msg = self._L.tw_last_error(self._h).decode()
            raise TwError(st, msg or self._L.tw_status_str(st).decode())

    def decide(self, rows, k: int, stats_on_error: dict | None = None):
        """(yes, stats).  On an error the counters of the levels built go to
        stats_on_error (when given) before TwError is raised."""
        g, keep = _graph(rows)
        yes = ctypes.c_int32(0)
        s = _Stats()
        st = self._L.tw_decide(self._h, ctypes.byref(g), int(k), ctypes.byref(yes), ctypes.byref(s))
        if st != TW_OK and stats_on_error is not None:
            stats_on_error.update(_stats_dict(s))
        self._check(st)
        return bool(yes.value), _stats_dict(s)

    def solve(self, rows):
        g, keep = _graph(rows)
        tw = ctypes.c_int32(0)
        order = np.zeros(len(keep), dtype=np.int32)
        s = _Stats()
        self._check(self._L.tw_solve(self._h, ctypes.byref(g), ctypes.byref(tw),
                                     order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(s)))
        return tw.value, order, _stats_dict(s)

    def decide128(self, rows, k: int):
        """decide(k) for a graph of up to 126 vertices (rows as Python ints)."""
        g, keep = _graph128(rows)
        yes = ctypes.c_int32(0)
        s = _Stats()
        self._check(self._L.tw_decide128(self._h, ctypes.byref(g), int(k), ctypes.byref(yes), ctypes.byref(s)))
        return bool(yes.value), _stats_dict(s)

    def solve128(self, rows):
        g, keep = _graph128(rows)
        tw = ctypes.c_int32(0)
        order = np.zeros(max(1, len(rows)), dtype=np.int32)
        s = _Stats()
        self._check(self._L.tw_solve128(self._h, ctypes.byref(g), ctypes.byref(tw),
                                        order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(s)))
        return tw.value, order[:len(rows)], _stats_dict(s)

    def trace_decide128(self, rows, k: int):
        """decide(k) for a graph of up to 126 vertices with every level:
        (level, count, expansions, successors, states) where states is a
        (count, 2) uint64 array of (low, high) words in the order found."""
        g, keep = _graph128(rows)
        levels = []

        def sink(rec_p, user):
            r = rec_p.contents
            c = int(r.count)
            w = np.ctypeslib.as_array(r.states, shape=(2 * c,)).copy() if c else np.zeros(0, np.uint64)
            levels.append((r.level, c, int(r.expansions), int(r.successors), w.reshape(c, 2)))

        cb = _SINK(sink)
        yes = ctypes.c_int32(0)
        self._check(self._L.tw_trace_decide128(self._h, ctypes.byref(g), int(k), cb, None, ctypes.byref(yes)))
        return bool(yes.value), levels

    def solve_noalloc(self, rows):
        """tw_solve_noalloc: as solve, with every device buffer of the call in
        the library's static scratch (ascending bounds; n <= 32)."""
        g, keep = _graph(rows)
        tw = ctypes.c_int32(0)
        order = np.zeros(len(keep), dtype=np.int32)
        s = _Stats()
        self._check(self._L.tw_solve_noalloc(self._h, ctypes.byref(g), ctypes.byref(tw),
                                             order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             ctypes.byref(s)))
        return tw.value, order, _stats_dict(s)

    def solve_batch(self, graphs, graph_stats: bool = False):
        """tw, orders, statuses, stats (and per-graph stats dicts if asked)."""
        arrs = [np.ascontiguousarray(np.asarray(r, dtype=np.uint64)) for r in graphs]
        gs = (_Graph * max(1, len(arrs)))()
        for t, a in enumerate(arrs):
            gs[t].n = len(a)
            gs[t].adj = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        cnt = len(arrs)
        tws = np.zeros(max(1, cnt), dtype=np.int32)
        orders = np.zeros(max(1, sum(len(a) for a in arrs)), dtype=np.int32)
        status = np.zeros(max(1, cnt), dtype=np.int32)
        s = _Stats()
        gst = (_GraphStats * max(1, cnt))()
        self._check(self._L.tw_solve_batch(
            self._h, gs, cnt, tws.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), gst, ctypes.byref(s)))
        out_orders, off = [], 0
        for a in arrs:
            out_orders.append(orders[off:off + len(a)].copy())
            off += len(a)
        res = (tws[:cnt].copy(), out_orders, status[:cnt].copy(), _stats_dict(s))
        if graph_stats:
            per = [{name: getattr(gst[t], name) for name, _ in _GraphStats._fields_ if name != "reserved"}
                   for t in range(cnt)]
            return res + (per,)
        return res

    def trace_batch(self, graphs, max_records: int = 4096, first_arena_states: int = 0):
        """tw_solve_batch with per-level records of the batched graphs:
        (tws, orders, statuses, per-graph stats dicts, records) where
        records[t] is a list of (k, level, count, successors, digest_sum,
        digest_xor) tuples in the order the levels were built (empty for
        graphs solved off the batch)."""
        arrs = [np.ascontiguousarray(np.asarray(r, dtype=np.uint64)) for r in graphs]
        cnt = len(arrs)
        gs = (_Graph * max(1, cnt))()
        for t, a in enumerate(arrs):
            gs[t].n = len(a)
            gs[t].adj = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        tws = np.zeros(max(1, cnt), dtype=np.int32)
        orders = np.zeros(max(1, sum(len(a) for a in arrs)), dtype=np.int32)
        status = np.zeros(max(1, cnt), dtype=np.int32)
        gst = (_GraphStats * max(1, cnt))()
        recs = (_BatchLevel * (max(1, cnt) * int(max_records)))()
        nrec = np.zeros(max(1, cnt), dtype=np.uint32)
        self._check(self._L.tw_trace_batch(
            self._h, gs, cnt, int(first_arena_states), int(max_records), recs,
            nrec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
            tws.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), gst))
        out_orders, off = [], 0
        for a in arrs:
            out_orders.append(orders[off:off + len(a)].copy())
            off += len(a)
        per = [{name: getattr(gst[t], name) for name, _ in _GraphStats._fields_ if name != "reserved"}
               for t in range(cnt)]
        records = []
        for t in range(cnt):
            m = min(int(nrec[t]), int(max_records))
            if int(nrec[t]) > int(max_records):
                raise RuntimeError(f"graph {t}: {int(nrec[t])} levels recorded, above max_records")
            base = t * int(max_records)
            records.append([(recs[base + j].k, recs[base + j].level, int(recs[base + j].count),
                             int(recs[base + j].successors), int(recs[base + j].digest_sum),
                             int(recs[base + j].digest_xor)) for j in range(m)])
        return tws[:cnt].copy(), out_orders, status[:cnt].copy(), per, records

    def trace_decide(self, rows, k: int):
        """decide(k) returning every level (states unordered) as Level records."""
        g, keep = _graph(rows)
        levels: list[Level] = []

        def sink(rec_p, user):
            r = rec_p.contents
            c = int(r.count)
            states = np.ctypeslib.as_array(r.states, shape=(c,)).copy() if c else np.zeros(0, np.uint64)
            lastv = np.ctypeslib.as_array(r.last_v, shape=(c,)).copy() if c else np.zeros(0, np.uint8)
            levels.append(Level(r.k, r.level, c, int(r.expansions), int(r.successors), states, lastv))

        cb = _SINK(sink)
        yes = ctypes.c_int32(0)
        self._check(self._L.tw_trace_decide(self._h, ctypes.byref(g), int(k), cb, None, ctypes.byref(yes)))
        return bool(yes.value), levels


def _graph_array(graphs):
    arrs = [np.ascontiguousarray(np.asarray(r, dtype=np.uint64)) for r in graphs]
    gs = (_Graph * max(1, len(arrs)))()
    for t, a in enumerate(arrs):
        gs[t].n = len(a)
        gs[t].adj = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    return gs, arrs


def mpnn_param_count() -> int:
    return int(load().tw_mpnn_param_count())


def mpnn_features(rows) -> np.ndarray:
    L = load()
    g, keep = _graph(rows)
    out = np.zeros((64, 4), dtype=np.float32)
    st = L.tw_mpnn_features(ctypes.byref(g), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    if st != TW_OK:
        raise TwError(st, "tw_mpnn_features")
    return out


class Mpnn:
    """The learned start-bound network on the device (bf16 MFMA kernels)."""

    def __init__(self, params: np.ndarray, device: int = 0):
        L = load()
        self._L = L
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != mpnn_param_count():
            raise ValueError("wrong parameter count")
        h = ctypes.c_void_p()
        self._check(L.tw_mpnn_create(device, None, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     ctypes.byref(h)))
        self._h = h

    def _check(self, st):
        if st != TW_OK:
            raise TwError(st, self._L.tw_status_str(st).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.tw_mpnn_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def params(self) -> np.ndarray:
        out = np.zeros(mpnn_param_count(), dtype=np.float32)
        self._check(self._L.tw_mpnn_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self._L.tw_mpnn_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def predict(self, graphs) -> np.ndarray:
        gs, keep = _graph_array(graphs)
        out = np.zeros((max(1, len(graphs)), 2), dtype=np.float32)
        self._check(self._L.tw_mpnn_predict(self._h, gs, len(graphs),
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out[:len(graphs)]

    def gradients(self, graphs, targets):
        gs, keep = _graph_array(graphs)
        t = np.ascontiguousarray(targets, dtype=np.float32)
        loss = ctypes.c_float(0)
        g = np.zeros(mpnn_param_count(), dtype=np.float32)
        self._check(self._L.tw_mpnn_gradients(self._h, gs, len(graphs),
                                              t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                              ctypes.byref(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return loss.value, g

    def trace(self, rows, target):
        """One graph's forward and backward pass with the kernels' float32
        intermediates (tw_mpnn_trace): a dict of 64 x 64 arrays per quantity
        (M, Z, dZ: lists over layers 0..2; P, dH: dicts for layers 1, 2; dH3),
        r [128], y [2], and the gradient vector."""
        gs, keep = _graph_array([rows])
        t = np.ascontiguousarray(target, dtype=np.float32)
        nf = int(self._L.tw_mpnn_trace_floats())
        tr = np.zeros(nf, dtype=np.float32)
        g = np.zeros(mpnn_param_count(), dtype=np.float32)
        self._check(self._L.tw_mpnn_trace(self._h, gs, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          tr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        blk = 4096

        def m(off):
            return tr[off:off + blk].reshape(64, 64).astype(np.float64)
        r0 = 6 * blk
        dh3 = r0 + 256
        dz = dh3 + blk
        pp = dz + 3 * blk
        dh = pp + 2 * blk
        out = {"M": [m(l * blk) for l in range(3)], "Z": [m(3 * blk + l * blk) for l in range(3)],
               "r": tr[r0:r0 + 128].astype(np.float64), "y": tr[r0 + 128:r0 + 130].astype(np.float64),
               "dH3": m(dh3), "dZ": [m(dz + l * blk) for l in range(3)],
               "P": {l: m(pp + (l - 1) * blk) for l in (1, 2)}, "dH": {l: m(dh + (l - 1) * blk) for l in (1, 2)}}
        return out, g

    def train_step(self, graphs, targets, lr: float, weight_decay: float = 0.0) -> float:
        gs, keep = _graph_array(graphs)
        t = np.ascontiguousarray(targets, dtype=np.float32)
        loss = ctypes.c_float(0)
        self._check(self._L.tw_mpnn_train_step(self._h, gs, len(graphs),
                                               t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                               float(lr), float(weight_decay), ctypes.byref(loss)))
        return loss.value


WEIGHTS_MAGIC = b"TWMPNN01"


def write_weights(path: str, params) -> None:
    """Write network parameters in the file format tw_ctx_create reads for
    the learned start bound: magic, uint32 count, float32 values (little-endian)."""
    p = np.ascontiguousarray(params, dtype="<f4")
    with open(path, "wb") as f:
        f.write(WEIGHTS_MAGIC)
        f.write(np.uint32(p.size).astype("<u4").tobytes())
        f.write(p.tobytes())


def read_weights(path: str) -> np.ndarray:
    with open(path, "rb") as f:
        if f.read(8) != WEIGHTS_MAGIC:
            raise ValueError("not a network parameter file")
        count = int(np.frombuffer(f.read(4), dtype="<u4")[0])
        return np.frombuffer(f.read(4 * count), dtype="<f4").copy()


def mmw128(rows) -> int:
    g, keep = _graph128(rows)
    lb = ctypes.c_int32(0)
    st = load().tw_mmw128(ctypes.byref(g), ctypes.byref(lb))
    if st != TW_OK:
        raise TwError(st, "tw_mmw128")
    return lb.value
