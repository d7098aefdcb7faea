"""Benchmark: exact treewidth of single n = 40 graphs on one MI355X.

One step solves each graph of the workload with tw_solve (minor-min-width
lower bound, ascending k, every level expanded and deduplicated on the GPU,
elimination order rebuilt and checked).  The metric is (S, v) expansions per
second over the whole job: sum over every level of |level| * (n - i), divided
by wall time.  Inputs are built on the host before the timed region; every
call returns after its outputs are written, so the timed region holds whole
solves and nothing else.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Prints one JSON line.  Fields beyond the driver's contract:
  batch         graphs solved per second on 512 held-out graphs (n 20..32),
                batched: plain ascending k, the learned start bound, and both
                with the clique skip and disjoint-path edges of §3.1
                (outside the timed region of `value`)
  reductions    the bench solves again with those reductions: time per step
                and expansions against the plain Listing 1 search
  roofline      the expansion kernel against HBM bandwidth, algorithmic bytes
                (key read per state, one compare-and-swap per feasible pair,
                key + creator byte written per new state) over the kernel time
                measured with HIP events on the launching stream; `traffic` is
                the counter-measured bytes per launch of the committed
                rocprofv3 summary (null once the kernel sources change), and
                `probe_reference` the machine's random-access rate for the
                insert's access pattern, measured in the same run
  cpu_baseline  the oracle (Listing 1 with exact dedup, plain C + OpenMP) on a
                bounded prefix of the same workload, on this host's cores
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


WORKLOADS = {
    # the single n = 40..42 graphs; the 6x7 grid's bound k = 6 needs levels of
    # ~10^10 states (k = 5 already peaks at 3.1e9), beyond one GPU's 288 GB
    "single_n40_one_gpu": "G(40, 0.15) seed 2001 and the random partial 8-tree on 40 vertices "
                          "(30% edges dropped, seed 2003): the n=40..42 single graphs whose exact "
                          "solve fits one MI355X (the 6x7 grid needs >288 GB at k=6)",
    "single_n40": "all three n=40..42 single graphs (includes the 6x7 grid; exceeds one GPU)",
    "single_n20": "G(20, 0.3) seed 1001",
}


def _workload(name: str):
    from paper_1709_09990_amd import graphs as G
    if name == "single_n40":
        return G.workload_single_n40()
    if name == "single_n40_one_gpu":
        w = G.workload_single_n40()
        return {k: w[k] for k in ("gnp40_p015", "partial8tree40")}
    if name == "single_n20":
        return {"gnp20_p03": G.workload_single_small(1001)}
    raise SystemExit(f"unknown workload {name}")


PROFILE = os.path.join(ROOT, "profiles", "expand_kernel_single_n40.md")
KERNEL_SOURCES = ("tw_kernels.hip", "tw_wave.h", "tw_internal.h")


def measured_traffic():
    """HBM bytes per expansion launch from the committed rocprofv3 counter
    summary, or None if the kernel sources changed since it was taken."""
    import hashlib
    if not os.path.exists(PROFILE):
        return None
    fields = {}
    for line in open(PROFILE):
        if "=" in line and line.startswith("    "):
            k, v = line.strip().split("=", 1)
            fields[k.strip()] = v.strip()
    src = b"".join(open(os.path.join(ROOT, "paper_1709_09990_amd", "csrc", f), "rb").read()
                   for f in KERNEL_SOURCES)
    if fields.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return float(fields["traffic_bytes_per_launch"])


def copy_probe(nbytes: int, reps: int = 5):
    """A plain device-to-device copy of known size (read nbytes, write nbytes),
    run only to scale the FETCH_SIZE / WRITE_SIZE counters of a profile."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


WEIGHTS = os.path.join(ROOT, "paper_1709_09990_amd", "weights", "mpnn_mixture_n16_30.bin")
# trained on labels of the search with the §3.1 reductions (their peak levels)
WEIGHTS_REDUCED = os.path.join(ROOT, "paper_1709_09990_amd", "weights", "mpnn_mixture_n16_30_reduced.bin")


def probe_reference(kernel_successors_per_s: float) -> dict:
    """The machine's rate for the insert's access pattern, measured now with
    tw_probe_rate on an 8 GiB buffer (far above the 256 MB Infinity Cache, as
    the large levels' tables are): random 16-byte loads with one in flight per
    lane (the probe), random 64-bit compare-and-swaps, and loads with eight in
    flight per lane.  The expansion kernel does one probe per feasible pair."""
    from paper_1709_09990_amd import tw as T
    nbytes, count = 8 << 30, 1 << 31
    r = {"buffer_bytes": nbytes, "operations": count}
    for mode, name in ((0, "random_16B_loads_per_s"), (1, "random_cas64_per_s"),
                       (2, "random_16B_loads_8_in_flight_per_s")):
        r[name] = T.probe_rate(nbytes, count, mode)
    r["kernel_probes_per_s"] = kernel_successors_per_s
    r["kernel_frac_of_random_loads"] = round(kernel_successors_per_s / r["random_16B_loads_per_s"], 4)
    return r


def batch_leg(count: int = 512):
    """Graphs solved per second, batched: plain ascending-k search vs the
    learned start bound and admission, on held-out graphs of the uneven
    mixture (n 20..32, seeds 600000+), same GPU, identical answers required."""
    from paper_1709_09990_amd import graphs as G
    from paper_1709_09990_amd import tw as T
    import numpy as np
    graphs = G.workload_batch(count, seed0=600000, n_lo=20, n_hi=32)
    out = {"graphs": count, "n": [20, 32], "weights": os.path.relpath(WEIGHTS, ROOT)}
    ref = None
    red = {"reductions": T.TW_REDUCE_CLIQUE_PATHS}
    learned = {"k_policy": T.TW_K_LEARNED, "weights_path": WEIGHTS}
    learned_red = {"k_policy": T.TW_K_LEARNED, "weights_path": WEIGHTS_REDUCED, **red}
    for name, kw in (("plain", {}), ("learned", learned), ("plain_reduced", red),
                     ("learned_reduced", learned_red)):
        with T.Context(device=0, **kw) as c:
            c.solve_batch(graphs[:16])
            t0 = time.perf_counter()
            tws, _, status, st = c.solve_batch(graphs)
            dt = time.perf_counter() - t0
        if np.any(status != 0):
            raise RuntimeError(f"batch leg: {name} failed on {int(np.sum(status != 0))} graphs")
        out[f"{name}_graphs_per_s"] = round(count / dt, 2)
        out[f"{name}_expansions"] = st["expansions"]
        out[f"{name}_bounds_tried"] = st["decisions"]
        if ref is None:
            ref = tws
        elif not np.array_equal(ref, tws):
            raise RuntimeError(f"batch leg: {name} changed an answer")
    out["identical"] = True
    out["learned_speedup"] = round(out["learned_graphs_per_s"] / out["plain_graphs_per_s"], 3)
    out["learned_reduced_speedup"] = round(out["learned_reduced_graphs_per_s"] /
                                           out["plain_reduced_graphs_per_s"], 3)
    out["weights_reduced"] = os.path.relpath(WEIGHTS_REDUCED, ROOT)
    return out


def reductions_leg(graphs: dict, steps: int = 2) -> dict:
    """The same single-graph solves with the clique skip and disjoint-path
    edges of §3.1 (TW_REDUCE_CLIQUE_PATHS): time per step and work, answers
    checked against the plain search's."""
    from paper_1709_09990_amd import tw as T
    out = {}
    with T.Context(device=0, timing=True, reductions=T.TW_REDUCE_CLIQUE_PATHS) as c:
        for nm in graphs:
            c.solve(graphs[nm])  # warm
        t0 = time.perf_counter()
        exp = 0
        tws = {}
        for _ in range(steps):
            for nm in graphs:
                tw, _, st = c.solve(graphs[nm])
                tws[nm] = tw
                exp += st["expansions"]
        dt = time.perf_counter() - t0
    out["ms_per_step"] = dt / steps * 1e3
    out["expansions_per_step"] = exp // steps
    out["treewidth"] = tws
    return out


def mmw_leg(graphs: dict, steps: int = 1) -> dict:
    """The same single-graph solves with per-state minor-min-width pruning
    (§3.3, TW_MMW_PRUNE): time per step, states expanded, answers checked
    against the plain search's."""
    from paper_1709_09990_amd import tw as T
    out = {}
    with T.Context(device=0, timing=True, mmw_prune=T.TW_MMW_PRUNE) as c:
        c.solve(graphs[min(graphs, key=lambda nm: len(graphs[nm]))])  # warm
        t0 = time.perf_counter()
        states = exp_kernel = 0
        tws = {}
        for _ in range(steps):
            for nm in graphs:
                tw, _, st = c.solve(graphs[nm])
                tws[nm] = tw
                states += st["states_expanded"]
                exp_kernel += st["kernel_seconds"]
        dt = time.perf_counter() - t0
    out["ms_per_step"] = dt / steps * 1e3
    out["states_expanded_per_step"] = states // steps
    out["expansion_kernel_ms_per_step"] = exp_kernel / steps * 1e3
    out["treewidth"] = tws
    return out


def cpu_baseline(budget_s: float = 15.0):
    """The oracle timed on a bounded prefix: levels of decide(8) on the random
    partial 8-tree (n=40) until the budget is spent."""
    from oracle import oracle as O
    from paper_1709_09990_amd import graphs as G

    rows = G.workload_single_n40()["partial8tree40"]
    k = 8
    threads = O.max_threads()
    try:
        threads = min(threads, len(os.sched_getaffinity(0)))
    except AttributeError:
        pass
    f = None
    import numpy as np
    f = np.zeros(1, dtype=np.uint64)
    cand_total = 0
    t0 = time.perf_counter()
    level = 0
    while time.perf_counter() - t0 < budget_s and len(f):
        f, gen, cand = O.bfs_level(rows, k, f, threads)
        cand_total += cand
        level += 1
    dt = time.perf_counter() - t0
    cpu = ""
    ram_gb = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram_gb = round(int(line.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    return {
        "value": cand_total / dt,
        "unit": "expansions/s",
        "cores": threads,
        "host": {"cpu": cpu, "ram_gb": ram_gb},
        "kind": "oracle",
        "sample": f"levels 1..{level} of decide(k={k}) on the random partial 8-tree (n=40), "
                  f"{cand_total} (S,v) pairs in {dt:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single_n40_one_gpu", choices=sorted(WORKLOADS))
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a device copy of this many bytes")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline leg")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched learned-vs-plain leg")
    ap.add_argument("--no-probe", action="store_true", help="skip the random-access reference measurement")
    ap.add_argument("--no-reduce", action="store_true", help="skip the single-graph leg with the section 3.1 reductions")
    ap.add_argument("--mmw", action="store_true", help="add a single-graph leg with per-state minor-min-width pruning")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the search over one graph "
              "is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    from paper_1709_09990_amd import tw as T

    graphs = _workload(args.workload)
    ctx = T.Context(device=0, timing=True)
    names = list(graphs)

    def step():
        agg = {"expansions": 0, "states_expanded": 0, "successors": 0, "unique": 0,
               "launches": 0, "kernel_seconds": 0.0, "retries": 0, "peak_frontier": 0}
        tws = {}
        for nm in names:
            tw, order, st = ctx.solve(graphs[nm])
            tws[nm] = tw
            for key in agg:
                if key == "peak_frontier":
                    agg[key] = max(agg[key], st[key])
                else:
                    agg[key] += st[key]
        return tws, agg

    for _ in range(args.warmup):
        step()
    t0 = time.perf_counter()
    total = None
    tws = None
    for _ in range(args.steps):
        tws, agg = step()
        if total is None:
            total = agg
        else:
            for key in total:
                total[key] = max(total[key], agg[key]) if key == "peak_frontier" else total[key] + agg[key]
    elapsed = time.perf_counter() - t0

    n_max = max(len(g) for g in graphs.values())
    w = 8 if n_max > 32 else 4
    alg_bytes = w * total["states_expanded"] + w * total["successors"] + (w + 1) * total["unique"]
    ks = total["kernel_seconds"]
    achieved = alg_bytes / ks / 1e9 if ks > 0 else 0.0
    traffic = measured_traffic()
    avg_launch_s = ks / max(1, total["launches"])
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": traffic,
        "kernel": "expand_kernel<uint%d>" % (8 * w),
        "launches": total["launches"],
        "avg_launch_us": round(avg_launch_s * 1e6, 2),
        "alg_bytes_per_launch": int(alg_bytes / max(1, total["launches"])),
    }
    if traffic and avg_launch_s > 0:
        # counter-measured bytes (committed profile) over this run's average launch
        roofline["traffic_GBps"] = round(traffic / avg_launch_s / 1e9, 1)
        roofline["traffic_frac"] = round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)
    if not args.no_probe and ks > 0:
        roofline["probe_reference"] = probe_reference(total["successors"] / ks)
    out = {
        "metric": "(S,v) expansions/sec + graphs solved/sec (learned-k batched vs plain), exact",
        "value": total["expansions"] / elapsed,
        "unit": "expansions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u%d" % (8 * w),
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "graphs": {nm: len(graphs[nm]) for nm in names},
                   "treewidth": tws, "dedup": "exact", "k_policy": "ascending from minor-min-width"},
        "states_per_s": total["states_expanded"] / elapsed,
        "graphs_per_s": len(names) * args.steps / elapsed,
        "successors": total["successors"],
        "peak_frontier": total["peak_frontier"],
        "retries": total["retries"],
        "kernel_fraction": round(ks / elapsed, 4),
        "roofline": roofline,
    }
    ctx.close()
    if not args.no_reduce:
        r = reductions_leg(graphs)
        if r["treewidth"] != tws:
            raise RuntimeError(f"reductions changed an answer: {r['treewidth']} vs {tws}")
        r["speedup_vs_plain_step"] = round(out["ms_per_step"] / r["ms_per_step"], 3)
        r["expansions_plain_per_step"] = total["expansions"] // args.steps
        out["reductions"] = r
    if args.mmw:
        m = mmw_leg(graphs)
        if m["treewidth"] != tws:
            raise RuntimeError(f"pruning changed an answer: {m['treewidth']} vs {tws}")
        m["slowdown_vs_plain_step"] = round(m["ms_per_step"] / out["ms_per_step"], 3)
        m["states_expanded_plain_per_step"] = total["states_expanded"] // args.steps
        out["mmw_prune"] = m
    if not args.no_batch:
        out["batch"] = batch_leg()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
