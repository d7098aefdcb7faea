"""Write per-level oracle digests of one bound-k search on a named workload.

    python tests/golden/make_levels.py partial8tree40 8

Calls only the oracle (Listing 1 with exact dedup, §3.1) and the seeded
generators.  Output: tests/golden/levels_<name>_k<k>.txt with one line per
level i: count, candidate pairs E_{i-1}, feasible pairs G_{i-1}, and the two
order-independent digests of the level's states (sum of one 64-bit mix and
xor of another).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1709_09990_amd import graphs as G  # noqa: E402


def main():
    name, k = sys.argv[1], int(sys.argv[2])
    rows = G.workload_single_n40()[name]
    path = os.path.join(HERE, f"levels_{name}_k{k}.txt")
    t0 = time.time()
    lines = [f"# oracle levels of decide(k={k}) on {name} (n={len(rows)}); "
             f"written by: python tests/golden/make_levels.py {name} {k}",
             "# level count candidates feasible digest_sum digest_xor"]
    c, s, x = O.set_hashes(__import__("numpy").zeros(1, dtype="uint64"))
    lines.append(f"0 1 0 0 {s} {x}")

    def on_level(i, f, cand, gen):
        cnt, hs, hx = O.set_hashes(f)
        lines.append(f"{i} {cnt} {cand} {gen} {hs} {hx}")
        print(f"level {i} count {cnt} t={time.time() - t0:.1f}s", flush=True)

    yes, _, _ = O.decide(rows, k, keep_levels=False, on_level=on_level)
    lines.append(f"# answer {'YES' if yes else 'NO'}")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(path, "YES" if yes else "NO", f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
