"""Autotuner for the batched search: the persistent work queue's smallest task,
hash-table load factor and probe scheme, picked by timing candidates on a
sample.  The schedule itself is the library's choice (options.batch_schedule
left at TW_BATCH_AUTO): a sample of small graphs cannot show how large levels
favour the persistent queue.

    from paper_1709_09990_amd import autotune
    opts = autotune.tuned_options(graphs)          # cached per (n bucket, device)
    ctx = tw.Context(device=0, **opts)

Every candidate must return exactly the same treewidths as the first one
(the tuner raises otherwise); only the time differs.  The cache is a small
JSON file (default ``~/.cache/tw_mi355x/autotune.json``, or $TW_AUTOTUNE_CACHE).
"""
from __future__ import annotations

import itertools
import json
import os
import time

import numpy as np

from . import tw as T

# smallest persistent-queue task, in states (larger levels are cut into larger tasks)
CHUNKS = (64, 128, 256)
LOAD_FACTORS = (0.4, 0.5, 0.7)
PROBES = (1, 2)


def _cache_path() -> str:
    return os.environ.get("TW_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tw_mi355x", "autotune.json"))


def bucket_of(graphs) -> str:
    n = int(np.median([len(g) for g in graphs])) if len(graphs) else 0
    return f"n{(n // 8) * 8}-{(n // 8) * 8 + 7}"


def _device_name() -> str:
    try:
        import torch  # plumbing only: the device name for the cache key
        return torch.cuda.get_device_name(0)
    except Exception:  # noqa: BLE001 - no torch or no device: one shared key
        return "gfx950"


def _time(graphs, opts: dict, reps: int) -> tuple[float, np.ndarray]:
    with T.Context(device=0, **opts) as c:
        c.solve_batch(graphs[: max(1, len(graphs) // 8)])  # warm allocations
        best = float("inf")
        tws = None
        for _ in range(reps):
            t0 = time.perf_counter()
            tws, _, status, _ = c.solve_batch(graphs)
            best = min(best, time.perf_counter() - t0)
            if np.any(status != 0):
                raise RuntimeError("autotune candidate failed on a graph")
    return best, tws


def tune(graphs, reps: int = 2, log=None) -> dict:
    """Time every candidate on `graphs`; return the fastest option set."""
    results = []
    ref = None
    for chunk, lf, probe in itertools.product(CHUNKS, LOAD_FACTORS, PROBES):
        opts = {"batch_chunk": chunk, "load_factor": lf, "probe": probe}
        dt, tws = _time(graphs, opts, reps)
        if ref is None:
            ref = tws
        elif not np.array_equal(ref, tws):
            raise RuntimeError(f"autotune candidate {opts} changed an answer")
        results.append((dt, opts))
        if log:
            log(f"autotune {opts}: {dt * 1e3:.1f} ms")
    results.sort(key=lambda r: r[0])
    best = dict(results[0][1])
    best["_ms"] = results[0][0] * 1e3
    return best


def tuned_options(graphs, sample: int = 64, refresh: bool = False, log=None) -> dict:
    """Cached tuned options for graphs like these (tuning on a sample if needed)."""
    path = _cache_path()
    key = f"{_device_name()}|{bucket_of(graphs)}"
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if refresh or key not in cache:
        best = tune(list(graphs)[:sample], log=log)
        cache[key] = best
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return {k: v for k, v in cache[key].items() if not k.startswith("_")}
