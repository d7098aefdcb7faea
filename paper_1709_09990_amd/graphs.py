"""Seeded synthetic graph generators (inputs only; no treewidth arithmetic).

A graph is a ``numpy.ndarray`` of ``n`` unsigned 64-bit adjacency rows: bit
``j`` of ``rows[i]`` is set iff ``{i, j}`` is an edge.  Graphs are simple and
undirected (symmetric rows, no self-loops) with ``1 <= n <= 64``.

The paper evaluates on preprocessed PACE 2016 / libtw instances (§4.1), which
are not available here.  These families stand in for them at the sizes the
paper used (n 21..64): Erdos-Renyi G(n,p), random geometric graphs, random
partial k-trees, grids, plus families whose treewidth has a closed form.

Randomness comes from one counter-free generator written from its published
definition: splitmix64 (Steele, Lea, Flood 2014) seeds xoshiro256** (Blackman
and Vigna 2018).  Every random graph is relabelled by a uniformly random
permutation so that construction order never leaks an elimination order.

This module is shared by the tests, the benchmark and the oracle's callers.
It holds no part of the method (no degree, no reachability, no dedup).
"""
from __future__ import annotations

import math

import numpy as np

M64 = (1 << 64) - 1


class Rng:
    """xoshiro256** seeded through splitmix64."""

    def __init__(self, seed: int):
        x = seed & M64
        s = []
        for _ in range(4):
            x = (x + 0x9E3779B97F4A7C15) & M64
            z = x
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
            s.append(z ^ (z >> 31))
        self.s = s

    @staticmethod
    def _rotl(x: int, k: int) -> int:
        return ((x << k) | (x >> (64 - k))) & M64

    def next_u64(self) -> int:
        s = self.s
        result = (self._rotl((s[1] * 5) & M64, 7) * 9) & M64
        t = (s[1] << 17) & M64
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = self._rotl(s[3], 45)
        return result

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def below(self, m: int) -> int:
        """Uniform integer in [0, m) by rejection (no modulo bias)."""
        if m <= 0:
            raise ValueError("below(m) needs m > 0")
        limit = (1 << 64) - ((1 << 64) % m)
        while True:
            r = self.next_u64()
            if r < limit:
                return r % m

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + self.below(hi - lo + 1)

    def permutation(self, n: int) -> list[int]:
        p = list(range(n))
        for i in range(n - 1, 0, -1):
            j = self.below(i + 1)
            p[i], p[j] = p[j], p[i]
        return p

    def sample(self, population: list, k: int) -> list:
        """k distinct items, uniformly (partial Fisher-Yates)."""
        pool = list(population)
        for i in range(k):
            j = i + self.below(len(pool) - i)
            pool[i], pool[j] = pool[j], pool[i]
        return pool[:k]


# ----------------------------------------------------------------------------
# representation helpers
# ----------------------------------------------------------------------------

def from_edges(n: int, edges) -> np.ndarray:
    if not 1 <= n <= 64:
        raise ValueError(f"n={n} outside 1..64")
    rows = [0] * n
    for a, b in edges:
        a, b = int(a), int(b)
        if a == b:
            raise ValueError("self-loop")
        if not (0 <= a < n and 0 <= b < n):
            raise ValueError("vertex out of range")
        rows[a] |= 1 << b
        rows[b] |= 1 << a
    return np.array(rows, dtype=np.uint64)


def edges_of(rows: np.ndarray) -> list[tuple[int, int]]:
    n = len(rows)
    out = []
    for i in range(n):
        r = int(rows[i])
        for j in range(i + 1, n):
            if (r >> j) & 1:
                out.append((i, j))
    return out


def relabel(rows: np.ndarray, perm: list[int]) -> np.ndarray:
    """Vertex i of the input becomes vertex perm[i]."""
    return from_edges(len(rows), [(perm[a], perm[b]) for a, b in edges_of(rows)])


def random_relabel(rows: np.ndarray, rng: Rng) -> np.ndarray:
    return relabel(rows, rng.permutation(len(rows)))


def n_edges(rows: np.ndarray) -> int:
    return sum(bin(int(r)).count("1") for r in rows) // 2


# ----------------------------------------------------------------------------
# random families
# ----------------------------------------------------------------------------

def gnp(n: int, p: float, seed: int) -> np.ndarray:
    """Erdos-Renyi G(n, p), randomly relabelled."""
    rng = Rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.uniform() < p]
    return random_relabel(from_edges(n, edges), rng)


def rgg(n: int, mean_degree: float, seed: int) -> np.ndarray:
    """Random geometric graph on n uniform points of the unit square.

    Edge iff Euclidean distance <= r with r = sqrt(d / ((n-1) pi)), the radius
    for expected degree d ignoring boundary effects (the realised mean degree
    is lower; ``n_edges`` reports it)."""
    rng = Rng(seed)
    pts = [(rng.uniform(), rng.uniform()) for _ in range(n)]
    r2 = mean_degree / ((n - 1) * math.pi) if n > 1 else 0.0
    edges = []
    for i in range(n):
        for j in range(i + 1, n):
            dx = pts[i][0] - pts[j][0]
            dy = pts[i][1] - pts[j][1]
            if dx * dx + dy * dy <= r2:
                edges.append((i, j))
    return random_relabel(from_edges(n, edges), rng)


def ktree_edges(n: int, k: int, rng: Rng) -> list[tuple[int, int]]:
    """Random k-tree on n >= k+1 vertices: start from K_{k+1}; each new vertex
    joins a uniformly random k-subset of a uniformly random existing
    (k+1)-clique (which creates k new (k+1)-cliques)."""
    if n < k + 1:
        raise ValueError("a k-tree needs n >= k+1")
    edges = [(i, j) for i in range(k + 1) for j in range(i + 1, k + 1)]
    cliques = [list(range(k + 1))]
    for v in range(k + 1, n):
        base = cliques[rng.below(len(cliques))]
        sub = rng.sample(base, k)
        for u in sub:
            edges.append((u, v))
        cliques.append(sub + [v])
    return edges


def partial_ktree(n: int, k: int, drop_frac: float, seed: int) -> np.ndarray:
    """Random k-tree with exactly round(drop_frac * m) uniformly chosen edges
    removed (treewidth <= k), randomly relabelled."""
    rng = Rng(seed)
    edges = ktree_edges(n, k, rng)
    drop = int(round(drop_frac * len(edges)))
    removed = set(rng.sample(list(range(len(edges))), drop))
    kept = [e for t, e in enumerate(edges) if t not in removed]
    return random_relabel(from_edges(n, kept), rng)


def ktree(n: int, k: int, seed: int) -> np.ndarray:
    """Random complete k-tree (treewidth exactly k when n >= k+1)."""
    rng = Rng(seed)
    return random_relabel(from_edges(n, ktree_edges(n, k, rng)), rng)


def random_tree(n: int, seed: int) -> np.ndarray:
    """Uniform random labelled tree (each vertex v >= 1 attaches to a uniform
    earlier vertex, then random relabel); treewidth 1 for n >= 2."""
    rng = Rng(seed)
    edges = [(v, rng.below(v)) for v in range(1, n)]
    return random_relabel(from_edges(n, edges), rng)


# ----------------------------------------------------------------------------
# deterministic families with closed-form treewidth
# ----------------------------------------------------------------------------

def complete(n: int) -> np.ndarray:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def edgeless(n: int) -> np.ndarray:
    return np.zeros(n, dtype=np.uint64)


def path(n: int) -> np.ndarray:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n: int) -> np.ndarray:
    if n < 3:
        raise ValueError("cycle needs n >= 3")
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def grid(a: int, b: int) -> np.ndarray:
    """a x b grid, row-major labels (vertex r*b + c)."""
    edges = []
    for r in range(a):
        for c in range(b):
            v = r * b + c
            if c + 1 < b:
                edges.append((v, v + 1))
            if r + 1 < a:
                edges.append((v, v + b))
    return from_edges(a * b, edges)


def complete_bipartite(a: int, b: int) -> np.ndarray:
    return from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def complete_multipartite(parts: list[int]) -> np.ndarray:
    label = []
    for p, size in enumerate(parts):
        label += [p] * size
    n = len(label)
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n) if label[i] != label[j]])


def disjoint_cliques(c: int, copies: int) -> np.ndarray:
    edges = []
    for t in range(copies):
        base = t * c
        edges += [(base + i, base + j) for i in range(c) for j in range(i + 1, c)]
    return from_edges(c * copies, edges)


def petersen() -> np.ndarray:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return from_edges(10, outer + spokes + inner)


# ----------------------------------------------------------------------------
# the synthetic workloads
# ----------------------------------------------------------------------------

def workload_single_small(seed: int = 1001) -> np.ndarray:
    """G(20, 0.3) from one seed (32-bit masks)."""
    return gnp(20, 0.3, seed)


def workload_single_n40() -> dict[str, np.ndarray]:
    """The three single graphs at n = 40..42 (64-bit masks): G(40, 0.15),
    the 6x7 grid (treewidth 6) and a random 8-tree on 40 vertices with 30% of
    its edges dropped."""
    return {
        "gnp40_p015": gnp(40, 0.15, 2001),
        "grid6x7": grid(6, 7),
        "partial8tree40": partial_ktree(40, 8, 0.30, 2003),
    }


def workload_batch(count: int = 512, seed0: int = 3000, n_lo: int = 16, n_hi: int = 48) -> list[np.ndarray]:
    """Uneven batch: thirds of G(n,p) (p ~ U[0.1,0.4]), random geometric
    graphs (target mean degree ~ U[4,8]) and partial k-trees (k ~ U{4..10},
    30% edge drop), n ~ U{n_lo..n_hi}."""
    out = []
    for t in range(count):
        rng = Rng(seed0 + t)
        n = rng.randint(n_lo, n_hi)
        fam = t % 3
        if fam == 0:
            p = 0.1 + 0.3 * rng.uniform()
            out.append(gnp(n, p, rng.next_u64()))
        elif fam == 1:
            d = 4.0 + 4.0 * rng.uniform()
            out.append(rgg(n, d, rng.next_u64()))
        else:
            k = rng.randint(4, min(10, n - 1))
            out.append(partial_ktree(n, k, 0.30, rng.next_u64()))
    return out


def workload_large_n64(seed: int = 4001) -> np.ndarray:
    """Random 12-tree on 64 vertices keeping 80% of its edges (tw <= 12)."""
    return partial_ktree(64, 12, 0.20, seed)
