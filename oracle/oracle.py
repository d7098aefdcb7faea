"""CPU oracle for exact treewidth (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg import this module.  The product library never does, and this module
imports nothing from the product package.

The arithmetic lives in plain C (``tw_oracle.c``, built into
``libtworacle.so``); this file is argument marshalling plus a few functions
written directly in Python:

* ``mmw`` — the minor-min-width lower bound of §3.3 (repeatedly contract a
  minimum-degree vertex into a minimum-degree neighbour; the second-smallest
  degree of every minor met is a lower bound on treewidth), with the
  tie-breaks read as "lowest index first" and degree-0 vertices deleted.
* ``q_set_py`` — Q(S,v) of §2 as an explicit set, by breadth-first search in
  pure Python, for the tiniest cases.
* ``set_hashes`` — count plus two order-independent 64-bit digests of a set
  of states, used to compare very large frontiers without sorting.

Functions and their sources:
    q_degree            §2 definition of Q(S,v); DFS of Listing 1 (§3.1)
    subset_dp           Held-Karp style recurrence over subsets (§1, §2)
    frontiers_from_dp   level i for bound k: {S : |S| = i, TW(S) <= k}
    brute_force         min over all orders of the fill-in width (§2)
    order_width         fill-in width of one order (§2)
    bfs_level / decide  Listing 1 (§3.1) with exact duplicate removal
    eliminated_graph    H_S, the graph left after eliminating S (§2)
    mmw_eliminated /    MMW(H_S) and the per-state pruning test of §3.3
      mmw_keep
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libtworacle.so")
_lib = None

u64p = ctypes.POINTER(ctypes.c_uint64)
u8p = ctypes.POINTER(ctypes.c_uint8)
i32p = ctypes.POINTER(ctypes.c_int32)
i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.tworacle_q_degree.argtypes = [ctypes.c_int, u64p, ctypes.c_uint64, ctypes.c_int]
        L.tworacle_q_degree.restype = ctypes.c_int
        L.tworacle_subset_dp.argtypes = [ctypes.c_int, u64p, u8p, ctypes.c_int]
        L.tworacle_subset_dp.restype = ctypes.c_int
        L.tworacle_frontier_from_table.argtypes = [ctypes.c_int, u8p, ctypes.c_int, ctypes.c_int,
                                                   u64p, ctypes.c_int64]
        L.tworacle_frontier_from_table.restype = ctypes.c_int64
        L.tworacle_order_width.argtypes = [ctypes.c_int, u64p, i32p]
        L.tworacle_order_width.restype = ctypes.c_int
        L.tworacle_brute_force.argtypes = [ctypes.c_int, u64p, i32p]
        L.tworacle_brute_force.restype = ctypes.c_int
        L.tworacle_bfs_level.argtypes = [ctypes.c_int, u64p, ctypes.c_int, u64p, ctypes.c_int64,
                                         ctypes.POINTER(u64p), i64p, i64p, ctypes.c_int]
        L.tworacle_bfs_level_masked.argtypes = [ctypes.c_int, u64p, ctypes.c_int, ctypes.c_uint64, u64p,
                                                ctypes.c_int64, ctypes.POINTER(u64p), i64p, i64p, ctypes.c_int]
        L.tworacle_bfs_level_masked.restype = ctypes.c_int64
        L.tworacle_bfs_level_part.argtypes = [ctypes.c_int, u64p, ctypes.c_int, ctypes.c_uint64, u64p,
                                              ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(u64p),
                                              i64p, i64p, ctypes.c_int]
        L.tworacle_bfs_level_part.restype = ctypes.c_int64
        L.tworacle_free.argtypes = [ctypes.c_void_p]
        L.tworacle_free.restype = None
        L.tworacle_bfs_level.restype = ctypes.c_int64
        L.tworacle_count_feasible.argtypes = [ctypes.c_int, u64p, ctypes.c_int, u64p,
                                              ctypes.c_int64, i64p, ctypes.c_int]
        L.tworacle_count_feasible.restype = ctypes.c_int64
        L.tworacle_max_threads.argtypes = []
        L.tworacle_max_threads.restype = ctypes.c_int
        L.tworacle_eliminated_graph.argtypes = [ctypes.c_int, u64p, ctypes.c_uint64, u64p]
        L.tworacle_eliminated_graph.restype = ctypes.c_int
        L.tworacle_mmw.argtypes = [ctypes.c_int, u64p]
        L.tworacle_mmw.restype = ctypes.c_int
        L.tworacle_mmw_eliminated.argtypes = [ctypes.c_int, u64p, ctypes.c_uint64]
        L.tworacle_mmw_eliminated.restype = ctypes.c_int
        L.tworacle_mmw_keep.argtypes = [ctypes.c_int, u64p, ctypes.c_int, u64p, ctypes.c_int64, u8p,
                                        ctypes.c_int]
        L.tworacle_mmw_keep.restype = ctypes.c_int64
        _lib = L
    return _lib


def _rows(rows) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
    if a.ndim != 1 or not 1 <= len(a) <= 64:
        raise ValueError("rows must be a 1-D array of 1..64 adjacency masks")
    return a


def _p(a, t):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------------------
# Q(S, v) and widths
# ---------------------------------------------------------------------------

def q_degree(rows, S: int, v: int) -> int:
    a = _rows(rows)
    d = lib().tworacle_q_degree(len(a), _p(a, u64p), int(S), int(v))
    if d < 0:
        raise ValueError("bad (S, v)")
    return d


def q_set_py(rows, S: int, v: int) -> set[int]:
    """Q(S,v) (§2) by breadth-first search in pure Python."""
    n = len(rows)
    adj = [[j for j in range(n) if (int(rows[i]) >> j) & 1] for i in range(n)]
    seen = {v}
    todo = [v]
    out = set()
    while todo:
        u = todo.pop()
        for w in adj[u]:
            if w in seen:
                continue
            seen.add(w)
            if (S >> w) & 1:
                todo.append(w)
            else:
                out.add(w)
    return out


def order_width(rows, order) -> int:
    """Fill-in width of an elimination order (§2, alternative view)."""
    a = _rows(rows)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    if len(o) != len(a):
        raise ValueError("order length != n")
    w = lib().tworacle_order_width(len(a), _p(a, u64p), _p(o, i32p))
    if w < 0:
        raise ValueError("order is not a permutation")
    return w


def order_width_q(rows, order) -> int:
    """Width of an order through the Q definition: max_t |Q({order[<t]}, order[t])|."""
    S = 0
    w = 0
    for v in order:
        w = max(w, q_degree(rows, S, int(v)))
        S |= 1 << int(v)
    return w


def brute_force(rows) -> tuple[int, list[int]]:
    """O2: min fill-in width over all n! orders (n <= 10)."""
    a = _rows(rows)
    o = np.zeros(len(a), dtype=np.int32)
    tw = lib().tworacle_brute_force(len(a), _p(a, u64p), _p(o, i32p))
    if tw < 0:
        raise ValueError("brute force limited to n <= 10")
    return tw, o.tolist()


# ---------------------------------------------------------------------------
# O1: subset dynamic programme
# ---------------------------------------------------------------------------

def subset_dp(rows, threads: int = 0) -> tuple[int, np.ndarray]:
    """TW(S) for every subset S; returns (tw(G), table)."""
    a = _rows(rows)
    n = len(a)
    if n > 30:
        raise ValueError("subset DP limited to n <= 30")
    table = np.zeros(1 << n, dtype=np.uint8)
    tw = lib().tworacle_subset_dp(n, _p(a, u64p), _p(table, u8p), threads)
    return tw, table


def frontier_from_table(n: int, table: np.ndarray, i: int, k: int) -> np.ndarray:
    L = lib()
    cnt = L.tworacle_frontier_from_table(n, _p(table, u8p), i, k, None, 0)
    out = np.zeros(max(cnt, 1), dtype=np.uint64)
    L.tworacle_frontier_from_table(n, _p(table, u8p), i, k, _p(out, u64p), cnt)
    return out[:cnt]


def n_levels(n: int, k: int) -> int:
    """Levels of the bound-k search: the last k+1 vertices may go in any
    order (§3.1, third optimisation), so n-k-1 levels decide it."""
    return max(0, n - k - 1)


def frontiers_from_dp(rows, k: int, table: np.ndarray | None = None) -> list[np.ndarray]:
    """[F_0, ..., F_L] for bound k, with F_i = {S : |S| = i, TW(S) <= k}."""
    a = _rows(rows)
    n = len(a)
    if table is None:
        _, table = subset_dp(a)
    return [frontier_from_table(n, table, i, k) for i in range(n_levels(n, k) + 1)]


# ---------------------------------------------------------------------------
# O4: the level search of Listing 1 with exact duplicate removal
# ---------------------------------------------------------------------------

def bfs_level(rows, k: int, frontier: np.ndarray, threads: int = 0, allowed: int | None = None,
              parts: int = 1, part: int = 0):
    """One level: returns (next frontier sorted, feasible pairs, candidate pairs).
    With `allowed`, only those vertices may be added (candidates count only them).
    With parts > 1 (a power of two), only the successors of group `part` of
    `parts` (a fixed function of the successor key) and their pairs."""
    a = _rows(rows)
    n = len(a)
    f = np.ascontiguousarray(np.asarray(frontier, dtype=np.uint64))
    ptr = u64p()
    gen = ctypes.c_int64(0)
    cand = ctypes.c_int64(0)
    mask = (2**64 - 1) if allowed is None else int(allowed) & (2**64 - 1)
    L = lib()
    cnt = L.tworacle_bfs_level_part(n, _p(a, u64p), int(k), mask, _p(f, u64p), len(f), int(parts),
                                    int(part), ctypes.byref(ptr), ctypes.byref(gen), ctypes.byref(cand),
                                    threads)
    if cnt < 0:
        raise RuntimeError("oracle bfs_level failed (bad argument or out of memory)")
    try:
        out = np.ctypeslib.as_array(ptr, shape=(cnt,)).copy() if cnt else np.zeros(0, dtype=np.uint64)
    finally:
        L.tworacle_free(ptr)
    return out, gen.value, cand.value


def bfs_level_grouped(rows, k: int, frontier: np.ndarray, parts: int, threads: int = 0):
    """One level built group by group (bounded memory): returns (next level,
    unsorted across groups, feasible pairs, candidate pairs)."""
    outs, gen, cand = [], 0, 0
    for p in range(parts):
        o, g, c = bfs_level(rows, k, frontier, threads, parts=parts, part=p)
        outs.append(o)
        gen += g
        cand += c
    nxt = np.concatenate(outs) if outs else np.zeros(0, dtype=np.uint64)
    return nxt, gen, cand


def decide(rows, k: int, keep_levels: bool = True, threads: int = 0, on_level=None,
           prune_mmw: bool = False):
    """decide(k) by Listing 1: YES iff the last level is non-empty.

    Returns (yes, levels, stats) where levels = [F_0..F_L] (sorted arrays; only
    the counts when keep_levels is False) and stats holds per-level
    (candidates E_i, feasible G_i).  With prune_mmw (O6, §3.3) a state S with
    MMW(H_S) > k is not expanded: level i+1 holds the successors of the kept
    states of level i (the stored levels themselves are not filtered)."""
    a = _rows(rows)
    n = len(a)
    L = n_levels(n, k)
    f = np.zeros(1, dtype=np.uint64)
    levels = [f if keep_levels else 1]
    stats = []
    for i in range(L):
        if prune_mmw:
            f = f[mmw_keep(a, k, f, threads)]
        nxt, gen, cand = bfs_level(a, k, f, threads)
        stats.append((cand, gen))
        if on_level is not None:
            on_level(i + 1, nxt, cand, gen)
        levels.append(nxt if keep_levels else len(nxt))
        f = nxt
        if len(f) == 0:
            # empty frontier: NO, and every later level is empty too
            for _ in range(i + 1, L):
                levels.append(np.zeros(0, dtype=np.uint64) if keep_levels else 0)
                stats.append((0, 0))
            break
    return len(f) > 0, levels, stats


def treewidth_bfs(rows, k0: int = 0, threads: int = 0) -> int:
    """Smallest k >= k0 with decide(k) YES (Listing 1's outer loop)."""
    a = _rows(rows)
    for k in range(max(0, k0), len(a)):
        yes, _, _ = decide(a, k, keep_levels=False, threads=threads)
        if yes:
            return k
    return len(a) - 1


def count_feasible(rows, k: int, states: np.ndarray, threads: int = 0):
    a = _rows(rows)
    s = np.ascontiguousarray(np.asarray(states, dtype=np.uint64))
    cand = ctypes.c_int64(0)
    feas = lib().tworacle_count_feasible(len(a), _p(a, u64p), int(k), _p(s, u64p), len(s),
                                         ctypes.byref(cand), threads)
    return feas, cand.value


def max_threads() -> int:
    return lib().tworacle_max_threads()


# ---------------------------------------------------------------------------
# minor-min-width (§3.3)
# ---------------------------------------------------------------------------

def mmw(rows) -> int:
    """Minor-min-width with the second-smallest-degree improvement (§3.3).

    Each round: record the second-smallest degree of the current minor (a
    lower bound while at least two vertices remain); take the lowest-index
    vertex v of minimum degree; if it is isolated delete it, otherwise contract
    v into its lowest-index minimum-degree neighbour u (u keeps its label and
    gains v's other neighbours)."""
    n = len(rows)
    nb = {v: {j for j in range(n) if (int(rows[v]) >> j) & 1} for v in range(n)}
    lb = 0
    while len(nb) >= 2:
        degs = sorted(len(s) for s in nb.values())
        lb = max(lb, degs[1])
        v = min(nb, key=lambda x: (len(nb[x]), x))
        if not nb[v]:
            del nb[v]
            continue
        u = min(nb[v], key=lambda x: (len(nb[x]), x))
        for w in nb[v]:
            nb[w].discard(v)
            if w != u:
                nb[w].add(u)
                nb[u].add(w)
        del nb[v]
    return lb


# ---------------------------------------------------------------------------
# O6: per-state minor-min-width (§3.3 on the graph left after eliminating S)
# ---------------------------------------------------------------------------

def eliminated_graph(rows, S: int) -> np.ndarray:
    """Rows of H_S: row u = Q(S, u) for u outside S, 0 for u in S."""
    a = _rows(rows)
    out = np.zeros(len(a), dtype=np.uint64)
    if lib().tworacle_eliminated_graph(len(a), _p(a, u64p), int(S), _p(out, u64p)) != 0:
        raise ValueError("bad graph")
    return out


def mmw_c(rows) -> int:
    """The C implementation of mmw (same rounds and tie-breaks)."""
    a = _rows(rows)
    return lib().tworacle_mmw(len(a), _p(a, u64p))


def mmw_eliminated(rows, S: int) -> int:
    """MMW(H_S), on the vertices outside S."""
    a = _rows(rows)
    return lib().tworacle_mmw_eliminated(len(a), _p(a, u64p), int(S))


def mmw_keep(rows, k: int, states: np.ndarray, threads: int = 0) -> np.ndarray:
    """Boolean mask: MMW(H_S) <= k for each state."""
    a = _rows(rows)
    s = np.ascontiguousarray(np.asarray(states, dtype=np.uint64))
    keep = np.zeros(len(s), dtype=np.uint8)
    if len(s):
        r = lib().tworacle_mmw_keep(len(a), _p(a, u64p), int(k), _p(s, u64p), len(s), _p(keep, u8p), threads)
        if r < 0:
            raise ValueError("bad graph")
    return keep.astype(bool)


# ---------------------------------------------------------------------------
# order-independent digests of a set of states
# ---------------------------------------------------------------------------

def _mix_a(x: np.ndarray) -> np.ndarray:
    # splitmix64 output function (Steele, Lea, Flood 2014)
    z = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def _mix_b(x: np.ndarray) -> np.ndarray:
    # MurmurHash3 fmix64 (Appleby)
    z = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(33)
        z *= np.uint64(0xFF51AFD7ED558CCD)
        z ^= z >> np.uint64(33)
        z *= np.uint64(0xC4CEB9FE1A85EC53)
        z ^= z >> np.uint64(33)
    return z


def set_hashes(states: np.ndarray) -> tuple[int, int, int]:
    """(count, sum of mix_a mod 2^64, xor of mix_b) — independent of order."""
    s = np.asarray(states, dtype=np.uint64)
    if len(s) == 0:
        return 0, 0, 0
    with np.errstate(over="ignore"):
        tot = int(np.add.reduce(_mix_a(s), dtype=np.uint64))
    x = int(np.bitwise_xor.reduce(_mix_b(s)))
    return len(s), tot, x


# ---------------------------------------------------------------------------
# tree decompositions (§1: the goal the treewidth search serves)
# ---------------------------------------------------------------------------

def is_tree_decomposition(rows, bags, parent) -> bool:
    """The three conditions of a tree decomposition, for bags (vertex masks)
    hung on the forest given by parent (-1 = root), checked as defined:
    every vertex and every edge lies in some bag, and for every vertex the
    bags holding it form one connected subtree (exactly one of them has a
    parent bag that does not hold it, or no parent)."""
    a = [int(r) for r in rows]
    n = len(a)
    m = len(bags)
    if len(parent) != m:
        return False
    # parent pointers must form a forest: walking up always reaches a root
    for b in range(m):
        seen = set()
        x = b
        while x != -1:
            if x in seen or not (-1 <= parent[x] < m):
                return False
            seen.add(x)
            x = parent[x]
    bag_sets = [{v for v in range(n) if (int(bags[b]) >> v) & 1} for b in range(m)]
    for v in range(n):
        holding = [b for b in range(m) if v in bag_sets[b]]
        if not holding:
            return False
        tops = [b for b in holding if parent[b] == -1 or v not in bag_sets[parent[b]]]
        if len(tops) != 1:
            return False
    for u in range(n):
        for v in range(u + 1, n):
            if (a[u] >> v) & 1 and not any(u in s and v in s for s in bag_sets):
                return False
    return True


def decomposition_width(bags) -> int:
    return max(bin(int(b)).count("1") for b in bags) - 1 if len(bags) else -1
