"""Oracle for graphs of more than 64 vertices (test infrastructure only).

Only the tests import this module; it imports nothing from the product
package.  Pure Python: vertex sets are Python integers of any width, so
states, rows and Q sets are not limited to one machine word.  The paper keeps
a state as a bitset and notes that wider bitsets extend the method (§3.1);
this module is the plain definition at any width, for graphs whose levels
stay small.

Functions (each follows the same passage as its 64-bit counterpart in the C
oracle, written again here, sharing no code with it):
    q_set        §2: the vertices outside S and other than v that v reaches
                 by paths whose internal vertices all lie in S
    bfs_level    one level of Listing 1 (§3.1) with exact duplicate removal
    decide       levels F_0..F_L for bound k, L = max(0, n - k - 1); YES iff
                 F_L is non-empty (third optimisation of §3.1)
    treewidth    smallest k with decide(k) YES
    order_from_levels  an elimination order of width <= k read back through
                 the levels (each state of F_{i+1} minus a vertex lies in F_i)
    order_width  width of an order by explicit fill-in (§2)
Pins: tests/test_oracle_wide.py (equality with the C oracle's levels for
n <= 64, closed forms beyond 64 vertices, invariance under relabelling, and a
planted 64-bit truncation that the pins catch).
"""
from __future__ import annotations


def rows_from_edges(n: int, edges) -> list[int]:
    rows = [0] * n
    for a, b in edges:
        if a == b:
            raise ValueError("self-loop")
        rows[a] |= 1 << b
        rows[b] |= 1 << a
    return rows


def q_set(rows: list[int], S: int, v: int) -> int:
    """Q(S, v) as a vertex set: search from v, continuing only through S."""
    seen = 1 << v
    stack = [v]
    q = 0
    while stack:
        u = stack.pop()
        new = rows[u] & ~seen
        seen |= new
        q |= new & ~S
        inside = new & S
        while inside:
            w = (inside & -inside).bit_length() - 1
            inside &= inside - 1
            stack.append(w)
    return q


def bfs_level(rows: list[int], k: int, frontier) -> list[int]:
    """All S + {v} with S in the frontier, v outside S and |Q(S, v)| <= k,
    each once, sorted."""
    n = len(rows)
    out = set()
    for S in frontier:
        for v in range(n):
            if not (S >> v) & 1 and bin(q_set(rows, S, v)).count("1") <= k:
                out.add(S | (1 << v))
    return sorted(out)


def decide(rows: list[int], k: int):
    """(yes, [F_0, ..., F_L]) for bound k; stops at the first empty level."""
    n = len(rows)
    L = max(0, n - k - 1)
    levels = [[0]]
    for _ in range(L):
        nxt = bfs_level(rows, k, levels[-1])
        levels.append(nxt)
        if not nxt:
            return False, levels
    return True, levels


def treewidth(rows: list[int], k0: int = 0) -> int:
    for k in range(max(0, k0), len(rows)):
        if decide(rows, k)[0]:
            return k
    return len(rows) - 1


def order_from_levels(rows: list[int], k: int, levels) -> list[int]:
    """Follow one state of the last level back to the empty set, choosing at
    each step a vertex v with S - {v} in the previous level and
    |Q(S - {v}, v)| <= k; the vertices outside the last state go last."""
    n = len(rows)
    S = levels[-1][0]
    last = S
    rev = []
    for i in range(len(levels) - 1, 0, -1):
        prev = set(levels[i - 1])
        for v in range(n):
            if (S >> v) & 1 and (S & ~(1 << v)) in prev and \
                    bin(q_set(rows, S & ~(1 << v), v)).count("1") <= k:
                rev.append(v)
                S &= ~(1 << v)
                break
        else:
            raise AssertionError("no predecessor")
    return rev[::-1] + [v for v in range(n) if not (last >> v) & 1]


def order_width(rows: list[int], order: list[int]) -> int:
    """Largest degree met when eliminating in this order with fill-in."""
    nb = list(rows)
    width = 0
    for v in order:
        N = nb[v]
        width = max(width, bin(N).count("1"))
        m = N
        while m:
            w = (m & -m).bit_length() - 1
            m &= m - 1
            nb[w] = (nb[w] | N) & ~(1 << w) & ~(1 << v)
        nb[v] = 0
    return width
