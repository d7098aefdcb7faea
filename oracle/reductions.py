"""Oracle for the two search-space reductions of §3.1 (test infrastructure only).

Only the tests import this module; it imports nothing from the product
package.  Plain Python, written for obviousness rather than speed.

§3.1 names three optimisations of the level search.  The third (stop after
n - k - 1 levels) is part of the plain oracle.  The first two are here:

* Clique skip.  For any clique C some optimal elimination order ends with the
  vertices of C, so the search never adds a vertex of a maximum clique to a
  state.  Reading taken where the paper is silent: C is the maximum clique
  whose ascending vertex list is lexicographically smallest, and decide(k) is
  NO without a search when k < |C| - 1 (a clique on |C| vertices already has
  treewidth |C| - 1).
* Disjoint-path edges.  If tw(G) <= k and u, v are joined by at least k + 1
  internally vertex-disjoint paths, adding the edge uv keeps tw <= k.  For the
  test "tw <= k" the search runs on G_k+ = G plus uv for every non-adjacent
  pair with at least k + 1 such paths, the counts taken once on G (the paper
  precomputes them once).  Adding edges one at a time never lowers a count, so
  all of them can be added together.

Functions:
    max_clique        Bron-Kerbosch enumeration of maximal cliques
    disjoint_paths    Menger counts by unit-capacity max flow on the split graph
    augmented_rows    G_k+
    decide_reduced    levels of Listing 1 on G_k+ with clique vertices skipped
    treewidth_reduced smallest k with decide_reduced YES
Pins (tests/test_oracle_pins.py): brute-force cliques and vertex separators
on small graphs, closed forms, and treewidth equal to the subset DP.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from . import oracle as O


def _adj_sets(rows) -> list[set[int]]:
    a = [int(r) for r in rows]
    n = len(a)
    return [{j for j in range(n) if (a[i] >> j) & 1} for i in range(n)]


def max_clique(rows) -> list[int]:
    """Maximum clique, lexicographically smallest ascending vertex list among
    the maximum ones.  Bron-Kerbosch (no pivot) lists every maximal clique."""
    adj = _adj_sets(rows)
    n = len(adj)
    best: list[int] = []

    def expand(r: list[int], p: list[int], x: list[int]):
        nonlocal best
        if not p and not x:
            c = sorted(r)
            if len(c) > len(best) or (len(c) == len(best) and c < best):
                best = c
            return
        for v in list(p):
            expand(r + [v], [u for u in p if u in adj[v]], [u for u in x if u in adj[v]])
            p.remove(v)
            x.append(v)

    expand([], list(range(n)), [])
    return best


def _max_flow_vertex_disjoint(adj: list[set[int]], s: int, t: int) -> int:
    """Number of internally vertex-disjoint s-t paths (s, t non-adjacent):
    max flow where every vertex w other than s, t is split into w_in -> w_out
    of capacity 1 and every edge {a, b} gives a_out -> b_in and b_out -> a_in."""
    n = len(adj)
    IN = lambda w: 2 * w  # noqa: E731
    OUT = lambda w: 2 * w + 1  # noqa: E731
    cap: dict[tuple[int, int], int] = {}
    nbr: list[set[int]] = [set() for _ in range(2 * n)]

    def add(a: int, b: int, c: int):
        cap[(a, b)] = cap.get((a, b), 0) + c
        cap.setdefault((b, a), 0)
        nbr[a].add(b)
        nbr[b].add(a)

    big = n + 1
    for w in range(n):
        add(IN(w), OUT(w), big if w in (s, t) else 1)
        for x in adj[w]:
            add(OUT(w), IN(x), big)
    src, snk = OUT(s), IN(t)
    flow = 0
    while True:
        prev = {src: None}
        q = deque([src])
        while q and snk not in prev:
            a = q.popleft()
            for b in nbr[a]:
                if b not in prev and cap[(a, b)] > 0:
                    prev[b] = a
                    q.append(b)
        if snk not in prev:
            return flow
        b = snk
        while prev[b] is not None:
            a = prev[b]
            cap[(a, b)] -= 1
            cap[(b, a)] += 1
            b = a
        flow += 1


def disjoint_paths(rows) -> np.ndarray:
    """P[u, v] = number of internally vertex-disjoint u-v paths for
    non-adjacent u != v; 0 on the diagonal and for adjacent pairs."""
    adj = _adj_sets(rows)
    n = len(adj)
    P = np.zeros((n, n), dtype=np.int32)
    for u in range(n):
        for v in range(u + 1, n):
            if v not in adj[u]:
                P[u, v] = P[v, u] = _max_flow_vertex_disjoint(adj, u, v)
    return P


def augmented_rows(rows, k: int, paths: np.ndarray | None = None) -> np.ndarray:
    """Rows of G_k+: G plus uv for non-adjacent u, v with >= k + 1 disjoint paths."""
    a = np.asarray(rows, dtype=np.uint64).copy()
    P = disjoint_paths(rows) if paths is None else paths
    n = len(a)
    for u in range(n):
        for v in range(n):
            if u != v and P[u, v] >= k + 1:
                a[u] |= np.uint64(1 << v)
    return a


def decide_reduced(rows, k: int, clique: list[int] | None = None, paths: np.ndarray | None = None,
                   threads: int = 0, prune_mmw: bool = False):
    """decide(k) of Listing 1 on G_k+ with the clique's vertices never added.

    Returns (yes, levels): levels F_0..F_L(k) (sorted arrays) over subsets of
    V minus C; ([F_0], NO) when k < |C| - 1.  With prune_mmw, states S whose
    eliminated graph in G_k+ has MMW > k are not expanded (O6 of the C oracle)."""
    n = len(rows)
    C = max_clique(rows) if clique is None else clique
    if k < len(C) - 1:
        return False, [np.zeros(1, dtype=np.uint64)]
    rk = augmented_rows(rows, k, paths)
    allowed = ((1 << n) - 1) & ~sum(1 << c for c in C)
    f = np.zeros(1, dtype=np.uint64)
    levels = [f]
    for _ in range(O.n_levels(n, k)):
        if prune_mmw:
            f = f[O.mmw_keep(rk, k, f, threads)]
        f, _, _ = O.bfs_level(rk, k, f, threads, allowed=allowed)
        levels.append(f)
        if len(f) == 0:
            break
    return len(levels) == O.n_levels(n, k) + 1 and len(levels[-1]) > 0, levels


def treewidth_reduced(rows, k0: int = 0, threads: int = 0) -> int:
    """Smallest k >= max(k0, |C| - 1) with decide_reduced YES."""
    C = max_clique(rows)
    P = disjoint_paths(rows)
    for k in range(max(k0, len(C) - 1, 0), len(rows)):
        yes, _ = decide_reduced(rows, k, C, P, threads)
        if yes:
            return k
    return len(rows) - 1
