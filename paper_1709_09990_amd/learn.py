"""Train the start-bound network on graphs labelled by the exact solver.

    python -m paper_1709_09990_amd.learn --train 20000 --out weights.bin

1. Training graphs: the uneven mixture (G(n,p) p~U[0.1,0.4], random geometric
   graphs with mean degree ~U[4,8], partial k-trees k~U{4..10} with 30% of
   edges dropped), n ~ U{16..30} by default, seeds 500000+.  (At n up to 40
   the mixture holds graphs needing 10^11 and more (S,v) pairs each, which
   makes 20,000 exact labels too costly; the range is an argument.)
2. Labels from exact runs of the batched solver: tw, and the largest level of
   the run that certified it (with --reductions, of the search with the
   clique skip and disjoint-path edges of §3.1).  Targets: tw/n and
   log2(peak+1)/32.
3. Training with the library's bf16 MFMA forward/backward kernels and AdamW.
4. Evaluation on held-out graphs (n ~ U{20..32} by default, seeds 600000+):
   the learned start bound against the plain ascending search, both batched,
   same GPU, identical answers required.

Labels are cached next to the weights (``<out>.labels.npz``) so a run can be
resumed.  Every step runs in libtw; this module only moves arrays.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

from . import graphs as G
from . import tw as T

def init_params(seed: int = 0) -> np.ndarray:
    """He-style random initialisation in the parameter order of tw.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for _ in range(3):
        parts.append(rng.normal(0, 1 / 8.0, 64 * 64))        # Ws
        parts.append(rng.normal(0, 1 / 32.0, 64 * 64))       # Wn
        parts.append(np.zeros(64))                           # b
    parts.append(rng.normal(0, 1 / (8.0 * np.sqrt(128)), 2 * 128))  # Wo
    parts.append(np.array([0.3, 0.5]))                       # bo: mean-ish targets
    return np.concatenate(parts).astype(np.float32)


def make_graphs(count: int, seed0: int, n_lo: int, n_hi: int) -> list[np.ndarray]:
    return G.workload_batch(count, seed0=seed0, n_lo=n_lo, n_hi=n_hi)


def label(graphs, ctx: T.Context, chunk: int = 512, log=print):
    """Exact labels; a graph the context cannot solve (its levels exceed the
    context's max_states) gets tw = -1 and is left out of training."""
    tws = np.zeros(len(graphs), dtype=np.int32)
    peaks = np.zeros(len(graphs), dtype=np.uint64)
    t0 = time.time()
    for b in range(0, len(graphs), chunk):
        part = graphs[b:b + chunk]
        tw, _, status, _, per = ctx.solve_batch(part, graph_stats=True)
        bad = status != 0
        tw = np.where(bad, -1, tw)
        tws[b:b + len(part)] = tw
        peaks[b:b + len(part)] = [q["peak_yes"] for q in per]
        log(f"labelled {b + len(part)}/{len(graphs)} graphs in {time.time() - t0:.1f}s"
            f" ({int(np.sum(tws[:b + len(part)] < 0))} beyond the state cap)")
    return tws, peaks


def targets_of(graphs, tws, peaks) -> np.ndarray:
    n = np.array([len(g) for g in graphs], dtype=np.float64)
    return np.stack([tws / n, np.log2(peaks.astype(np.float64) + 1.0) / 32.0], axis=1).astype(np.float32)


def train(net: T.Mpnn, graphs, targets, epochs: int, batch: int, lr: float, wd: float, seed: int, log=print):
    rng = np.random.default_rng(seed)
    idx = np.arange(len(graphs))
    history = []
    for ep in range(epochs):
        rng.shuffle(idx)
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / max(1, epochs)))  # cosine decay
        losses = []
        for b in range(0, len(idx), batch):
            sel = idx[b:b + batch]
            losses.append(net.train_step([graphs[i] for i in sel], targets[sel], lr=lr_ep, weight_decay=wd))
        history.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{epochs} loss {history[-1]:.5f} lr {lr_ep:.2e}")
    return history


def evaluate(graphs, weights_path: str, log=print, reductions: int = T.TW_REDUCE_NONE,
             max_states: int = 0) -> dict:
    """Plain ascending search vs learned start, both batched, same GPU."""
    out = {}
    for name, kw in (("plain", {}), ("learned", {"k_policy": T.TW_K_LEARNED, "weights_path": weights_path})):
        with T.Context(device=0, reductions=reductions, max_states=max_states, **kw) as c:
            c.solve_batch(graphs[:8])  # warm the context
            t0 = time.perf_counter()
            tws, orders, status, st, per = c.solve_batch(graphs, graph_stats=True)
            dt = time.perf_counter() - t0
        path = np.array([q["path"] for q in per])
        out[name] = {"tw": tws, "status": status, "seconds": dt, "graphs_per_s": len(graphs) / dt,
                     "expansions": st["expansions"], "decisions": st["decisions"],
                     "start_k": np.array([q["start_k"] for q in per]), "single_path": int(np.sum(path == 1))}
        log(f"{name}: {len(graphs) / dt:.1f} graphs/s, {st['expansions']:.3e} expansions, "
            f"{st['decisions']} bounds tried, {int(np.sum(path == 1))} graphs on the single-graph path, {dt:.2f}s")
    ok = (out["plain"]["status"] == 0) & (out["learned"]["status"] == 0)
    out["identical"] = bool(np.array_equal(out["plain"]["tw"][ok], out["learned"]["tw"][ok]))
    out["solved"] = int(np.sum(ok))
    if not np.all(ok):
        log(f"{int(np.sum(~ok))} graphs beyond the state cap in at least one policy")
    tw = out["plain"]["tw"][ok]
    d = out["learned"]["start_k"][ok] - tw
    log(f"held-out start bound: exact {np.mean(d == 0):.3f}, one below {np.mean(d == -1):.3f}, "
        f"above {np.mean(d > 0):.3f}; plain starts {np.mean(tw - out['plain']['start_k'][ok]):.2f} below tw on average")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--train-n", type=int, nargs=2, default=(16, 30))
    ap.add_argument("--eval", type=int, default=2048)
    ap.add_argument("--eval-n", type=int, nargs=2, default=(20, 32))
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--wd", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="weights.bin")
    ap.add_argument("--eval-only", action="store_true", help="skip labelling and training; evaluate --out")
    ap.add_argument("--max-states", type=int, default=0,
                    help="cap on states per level when labelling and evaluating (0 = none); graphs beyond it "
                         "are left out of training and counted apart in the evaluation")
    ap.add_argument("--reductions", action="store_true",
                    help="label, and evaluate, with the clique skip and disjoint-path edges of section 3.1 "
                         "(the peak label is then the reduced search's)")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    red = T.TW_REDUCE_CLIQUE_PATHS if args.reductions else T.TW_REDUCE_NONE

    if args.eval_only:
        ev = make_graphs(args.eval, 600000, *args.eval_n)
        res = evaluate(ev, args.out, log=log, reductions=red, max_states=args.max_states)
        log(f"identical answers: {res['identical']}; speedup "
            f"{res['learned']['graphs_per_s'] / res['plain']['graphs_per_s']:.3f}x")
        return 0

    graphs = make_graphs(args.train, 500000, *args.train_n)
    cache = args.out + ".labels.npz"
    if os.path.exists(cache):
        z = np.load(cache)
        tws, peaks = z["tw"], z["peak"]
        log(f"labels from {cache}")
    else:
        with T.Context(device=0, reductions=red, max_states=args.max_states) as ctx:
            tws, peaks = label(graphs, ctx, log=log)
        np.savez(cache, tw=tws, peak=peaks)
    keep = np.nonzero(tws >= 0)[0]
    if len(keep) < len(graphs):
        log(f"training on {len(keep)} of {len(graphs)} graphs (the rest exceed the state cap)")
    graphs = [graphs[i] for i in keep]
    tws, peaks = tws[keep], peaks[keep]
    targets = targets_of(graphs, tws, peaks)
    with T.Mpnn(init_params(args.seed)) as net:
        train(net, graphs, targets, args.epochs, args.batch, args.lr, args.wd, args.seed, log=log)
        T.write_weights(args.out, net.params())
        pred = net.predict(graphs)
    n = np.array([len(g) for g in graphs])
    err = np.abs(np.floor(pred[:, 0] * n) - tws)
    log(f"train: start bound exact for {np.mean(err == 0):.3f}, within 1 for {np.mean(err <= 1):.3f}")
    if args.eval:
        ev = make_graphs(args.eval, 600000, *args.eval_n)
        res = evaluate(ev, args.out, log=log, reductions=red, max_states=args.max_states)
        log(f"identical answers: {res['identical']}; speedup "
            f"{res['learned']['graphs_per_s'] / res['plain']['graphs_per_s']:.3f}x")
    return 0


if __name__ == "__main__":
    sys.exit(main())
