"""Write per-level oracle digests of one bound-k search on a named workload.

    python tests/golden/make_levels.py partial8tree40 8 [threads]

Calls only the oracle (Listing 1 with exact dedup, §3.1) and the seeded
generators.  Output: tests/golden/levels_<name>_k<k>.txt with one line per
level i: count, candidate pairs E_{i-1}, feasible pairs G_{i-1}, and the two
order-independent digests of the level's states (sum of one 64-bit mix and
xor of another).  A level whose successors would not fit the memory budget is
built in groups of successor keys (the oracle's grouped level step), and the
digests of the groups are combined (a sum mod 2^64 and a xor).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1709_09990_amd import graphs as G  # noqa: E402

BUDGET = float(os.environ.get("TW_ORACLE_BUDGET_GB", "20")) * 2**30
BYTES_PER_SUCCESSOR = 24  # per-thread buffers, the merged array and the sort's scratch


def groups_for(expected_successors: float) -> int:
    p = 1
    while p < 64 and expected_successors * BYTES_PER_SUCCESSOR > BUDGET * p:
        p *= 2
    return p


def main():
    name, k = sys.argv[1], int(sys.argv[2])
    threads = int(sys.argv[3]) if len(sys.argv) > 3 else 0
    rows = G.workload_single_n40()[name]
    n = len(rows)
    path = os.path.join(HERE, f"levels_{name}_k{k}.txt")
    t0 = time.time()
    lines = [f"# oracle levels of decide(k={k}) on {name} (n={n}); "
             f"written by: python tests/golden/make_levels.py {name} {k}",
             "# level count candidates feasible digest_sum digest_xor"]
    f = np.zeros(1, dtype=np.uint64)
    _, s, x = O.set_hashes(f)
    lines.append(f"0 1 0 0 {s} {x}")
    ratio = float(n)  # feasible pairs per state of the previous level
    for i in range(O.n_levels(n, k)):
        parts = groups_for(len(f) * ratio * 1.3)
        outs, gen, cand, hs, hx = [], 0, 0, 0, 0
        for p in range(parts):
            o, g, c = O.bfs_level(rows, k, f, threads, parts=parts, part=p)
            _, a, b = O.set_hashes(o)
            hs = (hs + a) % 2**64
            hx ^= b
            gen += g
            cand += c
            outs.append(o)
        nxt = np.concatenate(outs) if parts > 1 else outs[0]
        del outs
        ratio = gen / max(len(f), 1)
        lines.append(f"{i + 1} {len(nxt)} {cand} {gen} {hs} {hx}")
        print(f"level {i + 1} count {len(nxt)} feasible {gen} groups {parts} t={time.time() - t0:.1f}s",
              flush=True)
        f = nxt
        if len(f) == 0:
            break
    yes = len(f) > 0
    lines.append(f"# answer {'YES' if yes else 'NO'}")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(path, "YES" if yes else "NO", f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
