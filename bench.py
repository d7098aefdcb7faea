"""Benchmark: exact treewidth of single n = 40 graphs on one MI355X.

One step solves each graph of the workload with tw_solve (minor-min-width
lower bound, ascending k, every level expanded and deduplicated on the GPU,
elimination order rebuilt and checked).  The metric is (S, v) expansions per
second over the whole job: sum over every level of |level| * (n - i), divided
by wall time.  Inputs are built on the host before the timed region; every
call returns after its outputs are written, so the timed region holds whole
solves and nothing else.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Prints one JSON line on stdout (progress of the longer legs goes to
stderr).  Fields beyond the driver's contract:
  batch         graphs solved per second on 512 held-out graphs (n 20..32),
                batched: plain ascending k, the learned start bound, and both
                with the clique skip and disjoint-path edges of §3.1
                (outside the timed region of `value`)
  batch_n16_48  the 512-graph uneven batch with n 16..48 (seeds 3000+), each
                level capped at 2^26 states: graphs solved per second, plain
                against the learned start bound, with the unsolved graphs and
                the level each reached
  small_graphs  G(20, 0.3) solves, captured level loop against the
                host-driven loop, with the oracle timed on the same graphs
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


def probe_reference(kernel_successors_per_s: float, kernel_claims_per_s: float = 0.0) -> dict:
    """The machine's rate for the insert's access pattern, measured now with
    tw_probe_rate on an 8 GiB buffer (far above the 256 MB Infinity Cache, as
    the large levels' tables are): random 16-byte loads with one in flight per
    lane (the probe), random 64-bit compare-and-swaps, and loads with eight in
    flight per lane.  The expansion kernel does one probe per feasible pair,
    and one winning compare-and-swap per new state (claims: a lower bound on
    its compare-and-swap rate, since a lost race costs one more)."""
    from paper_1709_09990_amd import tw as T
    nbytes, count = 8 << 30, 1 << 31
    r = {"buffer_bytes": nbytes, "operations": count}
    for mode, name in ((0, "random_16B_loads_per_s"), (1, "random_cas64_per_s"),
                       (2, "random_16B_loads_8_in_flight_per_s")):
        r[name] = T.probe_rate(nbytes, count, mode)
    r["kernel_probes_per_s"] = kernel_successors_per_s
    r["kernel_frac_of_random_loads"] = round(kernel_successors_per_s / r["random_16B_loads_per_s"], 4)
    if kernel_claims_per_s:
        r["kernel_claims_per_s"] = kernel_claims_per_s
        r["kernel_claims_frac_of_random_cas"] = round(kernel_claims_per_s / r["random_cas64_per_s"], 4)
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


def config1_leg(count: int = 64, reps: int = 3, oracle_graphs: int = 8) -> dict:
    """Small single graphs: G(20, 0.3) with seeds 1001.., plain tw_solve
    (ascending bounds from the minor-min-width bound).  Time per solve with
    each bound's level loop replayed as one captured HIP graph, against the
    host-driven loop (a launch sequence and a host wait per level); answers
    must agree.  Beside it the oracle on the first graphs, on one core (the
    paper's CPU baseline is sequential) and on every core: the subset DP over
    all 2^20 sets, and the level search of Listing 1 from the same bound."""
    from oracle import oracle as O
    from paper_1709_09990_amd import graphs as G
    from paper_1709_09990_amd import tw as T
    import numpy as np
    graphs = [G.workload_single_small(1001 + t) for t in range(count)]
    out = {"graphs": count, "n": 20, "p": 0.3, "seeds": [1001, 1000 + count], "reps": reps}
    ref = None
    for name, cap in (("captured", T.TW_CAPTURE_AUTO), ("host_loop", T.TW_CAPTURE_OFF)):
        with T.Context(device=0, capture=cap) as c:
            for r in graphs[:4]:
                c.solve(r)
            exp = launches = levels = 0
            tws = []
            t0 = time.perf_counter()
            for _ in range(reps):
                tws = []
                for r in graphs:
                    tw, _, st = c.solve(r)
                    tws.append(tw)
                    exp += st["expansions"]
                    launches += st["launches"]
                    levels += st["levels"]
            dt = time.perf_counter() - t0
        solves = count * reps
        out[f"{name}_ms_per_solve"] = round(dt / solves * 1e3, 4)
        out[f"{name}_solves_per_s"] = round(solves / dt, 1)
        out[f"{name}_expansions_per_s"] = exp / dt
        out[f"{name}_launches_per_solve"] = round(launches / solves, 2)
        out[f"{name}_levels_per_solve"] = round(levels / solves, 2)
        if ref is None:
            ref = tws
        elif ref != tws:
            raise RuntimeError("config-1 leg: the captured loop changed an answer")
    out["capture_speedup"] = round(out["host_loop_ms_per_solve"] / out["captured_ms_per_solve"], 3)
    threads = O.max_threads()
    try:
        threads = min(threads, len(os.sched_getaffinity(0)))
    except AttributeError:
        pass
    sample = graphs[:oracle_graphs]
    for label, th in (("1_core", 1), (f"{threads}_cores", threads)):
        t0 = time.perf_counter()
        for r, tw in zip(sample, ref):
            got, _ = O.subset_dp(r, threads=th)
            if got != tw:
                raise RuntimeError("config-1 leg: the subset DP disagrees")
        dt = time.perf_counter() - t0
        out[f"oracle_subset_dp_{label}_ms_per_graph"] = round(dt / len(sample) * 1e3, 2)
        t0 = time.perf_counter()
        for r, tw in zip(sample, ref):
            if O.treewidth_bfs(r, O.mmw(r), threads=th) != tw:
                raise RuntimeError("config-1 leg: the oracle level search disagrees")
        dt = time.perf_counter() - t0
        out[f"oracle_level_search_{label}_ms_per_graph"] = round(dt / len(sample) * 1e3, 2)
    out["oracle_graphs"] = len(sample)
    out["oracle_cores"] = threads
    out["treewidths"] = sorted(set(int(x) for x in np.asarray(ref)))
    return out


WEIGHTS_N40_REDUCED = os.path.join(ROOT, "paper_1709_09990_amd", "weights", "mpnn_mixture_n16_40_reduced.bin")


def _outcomes(graphs, tws, status, per) -> dict:
    import numpy as np
    solved = [t for t in range(len(graphs)) if status[t] == 0]
    failed = [t for t in range(len(graphs)) if status[t] != 0]
    codes = {}
    for t in failed:
        codes[int(status[t])] = codes.get(int(status[t]), 0) + 1
    out = {"solved": len(solved), "unsolved": len(failed), "unsolved_status": codes}
    if failed:
        ns = [len(graphs[t]) for t in failed]
        peaks = [int(per[t]["peak_any"]) for t in failed]
        out["unsolved_n_range"] = [min(ns), max(ns)]
        out["unsolved_largest_level_min"] = min(peaks)
        out["unsolved_graphs"] = [[t, len(graphs[t]), int(per[t]["peak_any"])] for t in failed]
    out["paths"] = {str(p): sum(1 for t in range(len(graphs)) if per[t]["path"] == p) for p in (0, 1, 2)}
    return out


def _oracle_treewidth(rows):
    """One graph's treewidth by the oracle's level search (Listing 1), on one
    core: a worker of the process pool below."""
    import numpy as np
    from oracle import oracle as O
    r = np.asarray(rows, dtype=np.uint64)
    return O.treewidth_bfs(r, O.mmw(r), threads=1)


def _pool_ready(_):
    return 0


def oracle_batch_sample(graphs, base: dict, max_n: int = 26, count: int = 64) -> dict:
    """The oracle on a bounded sample of a batch: its first `count` graphs with
    n <= max_n, one graph per host core at a time (a process pool started
    before the timed region), against the GPU's batched solve of the same
    graphs with the leg's options.  Treewidths must agree."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    from paper_1709_09990_amd import tw as T
    sample = [g for g in graphs if len(g) <= max_n][:count]
    if not sample:
        return {}
    try:
        cores = min(16, len(os.sched_getaffinity(0)))
    except AttributeError:
        cores = min(16, os.cpu_count() or 1)
    rows = [[int(x) for x in g] for g in sample]
    # fresh interpreters (this process already holds the GPU); a worker that
    # cannot start raises here instead of leaving the map waiting
    with ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("spawn")) as ex:
        list(ex.map(_pool_ready, range(cores), timeout=120))
        t0 = time.perf_counter()
        want = list(ex.map(_oracle_treewidth, rows, timeout=300))
        cpu_s = time.perf_counter() - t0
    with T.Context(device=0, **base) as c:
        c.solve_batch(sample[:4])
        t0 = time.perf_counter()
        tws, _, status, _ = c.solve_batch(sample)
        gpu_s = time.perf_counter() - t0
    if list(status) != [0] * len(sample) or [int(x) for x in tws] != want:
        raise RuntimeError("oracle sample: the batched GPU solve disagrees with the oracle")
    return {"graphs": len(sample), "n_max": max(len(g) for g in sample), "cores": cores, "kind": "oracle",
            "oracle_seconds": round(cpu_s, 3), "oracle_graphs_per_s": round(len(sample) / cpu_s, 2),
            "gpu_seconds": round(gpu_s, 4), "gpu_graphs_per_s": round(len(sample) / gpu_s, 2),
            "sample": f"the first {len(sample)} graphs with n <= {max_n}, plain ascending search"}


def batch_config_leg(graphs, label: str, max_states: int, weights: str, reductions: bool,
                     ceiling: bool = False, per_call: int = 128, cpu: bool = False) -> dict:
    """Graphs solved per second, plain ascending bounds against the learned
    start bound, on one batch, each graph's levels capped at max_states
    states (a graph whose level would exceed the cap returns TW_ECAPACITY with
    the size it reached).  Task size, load factor and probe scheme from the
    autotuner (tuned on the batch's graphs of n <= 32); the schedule is the
    library's default (the persistent queue, level rounds with the
    reductions).  Answers must agree on every graph both
    policies solve.  With ceiling: the certifying work alone (decide(tw) and,
    when tw is above the lower bound, decide(tw - 1)) per solved graph, i.e.
    a start bound that is never wrong.  The graphs go in calls of per_call
    (one progress line each); the time is the sum over the calls."""
    import numpy as np
    from paper_1709_09990_amd import autotune
    from paper_1709_09990_amd import tw as T
    small = [g for g in graphs if len(g) <= 32][:48]
    tuned = autotune.tuned_options(small, sample=48) if small else {}
    base = dict(tuned)
    base["max_states"] = max_states
    if reductions:
        base["reductions"] = T.TW_REDUCE_CLIQUE_PATHS
    out = {"label": label, "graphs": len(graphs), "n": [min(len(g) for g in graphs), max(len(g) for g in graphs)],
           "max_states_per_level": max_states, "reductions": reductions, "tuned_options": tuned,
           "schedule": "level rounds" if reductions else "persistent queue",
           "weights": os.path.relpath(weights, ROOT)}
    res = {}
    out["graphs_per_call"] = per_call
    for name, kw in (("plain", {}), ("learned", {"k_policy": T.TW_K_LEARNED, "weights_path": weights})):
        tws, status, per = [], [], []
        exp = dec = 0
        dt = 0.0
        with T.Context(device=0, **base, **kw) as c:
            for lo in range(0, len(graphs), per_call):
                t0 = time.perf_counter()
                a, _, b, st, d = c.solve_batch(graphs[lo:lo + per_call], graph_stats=True)
                dt += time.perf_counter() - t0
                tws += [int(x) for x in a]
                status += [int(x) for x in b]
                per += d
                exp += st["expansions"]
                dec += st["decisions"]
                print(json.dumps({"leg": label, "policy": name, "graphs_done": lo + len(a),
                                  "seconds": round(dt, 1)}), file=sys.stderr, flush=True)
        res[name] = (tws, status, per)
        o = _outcomes(graphs, tws, status, per)
        o["seconds"] = round(dt, 2)
        o["graphs_solved_per_s"] = round(o["solved"] / dt, 2)
        o["expansions"] = exp
        o["bounds_tried"] = dec
        out[name] = o
    tp, sp, _ = res["plain"]
    tl, sl, _ = res["learned"]
    both = [t for t in range(len(graphs)) if sp[t] == 0 and sl[t] == 0]
    if any(tp[t] != tl[t] for t in both):
        raise RuntimeError(f"{label}: the learned start bound changed an answer")
    out["identical_on_both_solved"] = len(both)
    out["learned_speedup"] = round(out["learned"]["graphs_solved_per_s"] / out["plain"]["graphs_solved_per_s"], 3)
    if cpu:
        out["oracle_sample"] = oracle_batch_sample(graphs, base)
    if ceiling and len(both) < len(graphs):
        # the graphs both solve, again: graphs solved per second without the
        # time the capped graphs cost
        sub = [graphs[t] for t in both]
        for name, kw in (("plain", {}), ("learned", {"k_policy": T.TW_K_LEARNED, "weights_path": weights})):
            dt = 0.0
            exp = dec = 0
            with T.Context(device=0, **base, **kw) as c:
                for lo in range(0, len(sub), per_call):
                    t0 = time.perf_counter()
                    a, _, b, st = c.solve_batch(sub[lo:lo + per_call])
                    dt += time.perf_counter() - t0
                    exp += st["expansions"]
                    dec += st["decisions"]
                    if any(int(x) != 0 for x in b) or any(int(a[j]) != int(tp[both[lo + j]]) for j in range(len(a))):
                        raise RuntimeError(f"{label}: a solved graph changed on the second pass")
                    print(json.dumps({"leg": label, "solved_only": name, "graphs_done": lo + len(a),
                                      "seconds": round(dt, 1)}), file=sys.stderr, flush=True)
            out[f"solved_only_{name}"] = {"graphs": len(sub), "seconds": round(dt, 2),
                                          "graphs_per_s": round(len(sub) / dt, 2), "expansions": exp,
                                          "bounds_tried": dec}
        out["solved_only_learned_speedup"] = round(out["solved_only_learned"]["graphs_per_s"] /
                                                   out["solved_only_plain"]["graphs_per_s"], 3)
    if ceiling:
        kw = dict(base)
        kw.pop("max_states", None)
        exp = 0
        with T.Context(device=0, max_states=max_states, **{k: v for k, v in kw.items()
                                                           if k in ("reductions", "load_factor", "probe")}) as c:
            t0 = time.perf_counter()
            for q, t in enumerate(both):
                if q % 256 == 255:
                    print(json.dumps({"leg": label, "ceiling_graphs_done": q + 1}), file=sys.stderr, flush=True)
                lb = T.mmw(graphs[t])
                if reductions:
                    lb = max(lb, len(T.reductions(graphs[t])[0]) - 1)
                for k in ([int(tp[t])] + ([int(tp[t]) - 1] if tp[t] > lb else [])):
                    _, st = c.decide(graphs[t], k)
                    exp += st["expansions"]
            dt = time.perf_counter() - t0
        out["ceiling"] = {"graphs": len(both), "seconds": round(dt, 2), "graphs_per_s": round(len(both) / dt, 2),
                          "expansions": exp,
                          "note": "decide(tw) and decide(tw-1) one graph at a time on the single-graph path"}
    return out


def large_leg(cap_log2: int = 29) -> dict:
    """The large single instance: random partial 12-tree on 64 vertices, 80%
    of edges kept (seed 4001), decide(12) (its minor-min-width bound, so the
    bound that certifies tw = 12), exact table against the Bloom variant of
    §3.2, each level capped at 2^cap_log2 states: the levels up to the cap,
    their expansion kernel time and rate.  The full search outgrows one GPU's
    288 GB; the cap stops it with TW_ECAPACITY and the levels before it are
    reported."""
    from paper_1709_09990_amd import graphs as G
    from paper_1709_09990_amd import tw as T
    rows = G.workload_large_n64()
    out = {"graph": "partial 12-tree, n=64, 80% edges kept, seed 4001", "k": 12,
           "max_states_per_level": 1 << cap_log2}
    for name, dedup in (("exact", T.TW_DEDUP_EXACT), ("bloom", T.TW_DEDUP_BLOOM)):
        with T.Context(device=0, timing=True, dedup=dedup, max_states=1 << cap_log2) as c:
            st = {}
            t0 = time.perf_counter()
            status = "YES/NO"
            try:
                yes, st = c.decide(rows, 12, stats_on_error=st)
                status = "YES" if yes else "NO"
            except T.TwError as e:
                status = f"stopped: status {e.status}"
            dt = time.perf_counter() - t0
        ks = st.get("kernel_seconds", 0.0)
        out[name] = {"outcome": status, "seconds": round(dt, 2), "levels": st.get("levels"),
                     "peak_level": st.get("peak_frontier"), "expansions": st.get("expansions"),
                     "states_expanded": st.get("states_expanded"), "successors": st.get("successors"),
                     "unique": st.get("unique"), "launches": st.get("launches"),
                     "kernel_seconds": round(ks, 3),
                     "kernel_expansions_per_s": st.get("expansions", 0) / ks if ks else None}
        print(json.dumps({"leg": "large_n64", name: out[name]}), file=sys.stderr, flush=True)
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


def cpu_baseline(budget_s: float = 15.0, threads: int = 0):
    """The oracle timed on a bounded prefix: levels of decide(8) on the random
    partial 8-tree (n=40) until the budget is spent, on `threads` cores (0:
    every core this process may use).  The prefix holds the small early
    levels; later levels, whose per-pair search is longer, would give the
    oracle a lower rate."""
    from oracle import oracle as O
    from paper_1709_09990_amd import graphs as G

    rows = G.workload_single_n40()["partial8tree40"]
    k = 8
    if threads <= 0:
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
    ap.add_argument("--no-small", action="store_true", help="skip the G(20, 0.3) captured-loop leg")
    ap.add_argument("--batch-n16-48", action="store_true",
                    help="the 512-graph batch with n 16..48 (seeds 3000+), plain vs learned, per-level cap "
                         "(run by default; kept for older command lines)")
    ap.add_argument("--no-batch-n16-48", action="store_true", help="skip the n 16..48 batch leg")
    ap.add_argument("--learned-n20-56", action="store_true",
                    help="add the 2,048 held-out graphs with n 20..56 (seeds 600000+), plain vs learned vs ceiling")
    ap.add_argument("--cap", type=int, default=1 << 26, help="states per level for the two legs above")
    ap.add_argument("--reduce-batches", action="store_true", help="run the two legs above with the section 3.1 reductions")
    ap.add_argument("--large-n64", action="store_true", help="add the n=64 partial 12-tree leg (exact vs Bloom, capped levels)")
    ap.add_argument("--large-cap-log2", type=int, default=29, help="log2 of the states-per-level cap of that leg")
    ap.add_argument("--only-large", action="store_true",
                    help="run only the n=64 leg and print its result (for profiling that workload alone)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.only_large:
        print(json.dumps({"large_n64": large_leg(args.large_cap_log2)}), flush=True)
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
        roofline["probe_reference"] = probe_reference(total["successors"] / ks, total["unique"] / ks)
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
    if not args.no_small:
        out["small_graphs"] = config1_leg()
    if not args.no_batch:
        out["batch"] = batch_leg()
    if args.large_n64:
        out["large_n64"] = large_leg(args.large_cap_log2)
    run_n16_48 = not args.no_batch_n16_48
    if run_n16_48 or args.learned_n20_56:
        from paper_1709_09990_amd import graphs as G
        wts = WEIGHTS_N40_REDUCED if args.reduce_batches else WEIGHTS
        if run_n16_48:
            out["batch_n16_48"] = batch_config_leg(G.workload_batch(512, seed0=3000, n_lo=16, n_hi=48),
                                                   "batch_n16_48", args.cap, wts, args.reduce_batches,
                                                   cpu=not args.no_cpu)
        if args.learned_n20_56:
            out["learned_n20_56"] = batch_config_leg(G.workload_batch(2048, seed0=600000, n_lo=20, n_hi=56),
                                                     "learned_n20_56", args.cap, wts, args.reduce_batches,
                                                     ceiling=True, cpu=not args.no_cpu)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
        # the paper's CPU baseline is sequential: the same oracle on one core
        one = cpu_baseline(args.cpu_budget / 2, threads=1)
        out["cpu_baseline"]["one_core"] = {"value": one["value"], "unit": one["unit"], "cores": 1,
                                           "sample": one["sample"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
