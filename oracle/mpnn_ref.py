"""CPU reference of the small message-passing network (test infrastructure only).

The network predicts, for one graph, its treewidth and the size of the
largest level of the certifying search; the solver uses the prediction to pick
its first bound k and to size per-graph memory.  Nothing in the paper fixes the
network, so this follows the design written for the build:

    node features  x_v = [1, deg(v)/8, core(v)/8, n/64, 0, ..., 0]   (64 wide)
    3 layers       H_{l+1} = ReLU(H_l Ws_l^T + (A H_l) Wn_l^T + b_l) * mask
    readout        r = [sum_v H3_v ; max_v H3_v]             (128)
    heads          y = Wo r + bo                             (2: tw/n, log2(peak+1)/32)
    loss           mean over graphs and heads of (y - t)^2

(core(v) is the core number: the largest c such that v lies in a subgraph of
minimum degree c.)  Every quantity is float64.  With ``bf16=True`` the
operands of every matrix product are first rounded to bfloat16
(round-to-nearest-even), at exactly the points where the GPU kernels hold them
in bfloat16: H_l, A H_l, the weights Ws/Wn, and in the backward pass the
gradients dZ_l and dZ_l Wn_l.  Accumulation stays float64, so the reference
differs from the GPU only by the GPU's float32 accumulation order.

The gradients in float64 mode (bf16=False) are pinned by central finite
differences (tests/test_mpnn_ref.py).
"""
from __future__ import annotations

import numpy as np

N = 64          # padded nodes per graph
HID = 64        # hidden width (and padded input width)
LAYERS = 3
OUT = 2


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    Goes through float32 first (the GPU rounds float32 values); NaN and inf do
    not occur here."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def core_numbers(rows) -> np.ndarray:
    """Core number of every vertex by repeatedly deleting a minimum-degree vertex."""
    n = len(rows)
    nb = [{j for j in range(n) if (int(rows[v]) >> j) & 1} for v in range(n)]
    alive = set(range(n))
    core = np.zeros(n, dtype=np.int64)
    cur = 0
    while alive:
        v = min(alive, key=lambda x: (len(nb[x] & alive), x))
        cur = max(cur, len(nb[v] & alive))
        core[v] = cur
        alive.remove(v)
    return core


def features(rows) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(X [64x64], A [64x64], mask [64]) for one graph, padded to 64 nodes."""
    n = len(rows)
    A = np.zeros((N, N))
    for v in range(n):
        for j in range(n):
            if (int(rows[v]) >> j) & 1:
                A[v, j] = 1.0
    deg = A.sum(axis=1)
    core = np.zeros(N)
    core[:n] = core_numbers(rows)
    X = np.zeros((N, HID))
    X[:n, 0] = 1.0
    X[:n, 1] = deg[:n] / 8.0
    X[:n, 2] = core[:n] / 8.0
    X[:n, 3] = n / 64.0
    mask = np.zeros(N)
    mask[:n] = 1.0
    return X, A, mask


def init_params(seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)
    p = {}
    for l in range(LAYERS):
        p[f"Ws{l}"] = rng.normal(0, 1 / np.sqrt(HID), (HID, HID))
        p[f"Wn{l}"] = rng.normal(0, 1 / np.sqrt(HID) / 4, (HID, HID))
        p[f"b{l}"] = np.zeros(HID)
    p["Wo"] = rng.normal(0, 1 / np.sqrt(2 * HID) / 8, (OUT, 2 * HID))
    p["bo"] = np.zeros(OUT)
    return p


def forward_one(p: dict, X, A, mask, bf16: bool = False):
    rb = bf16_round if bf16 else (lambda z: z)
    H = X
    cache = []
    for l in range(LAYERS):
        Hb = rb(H)
        M = A @ Hb
        Mb = rb(M)
        Ws, Wn = rb(p[f"Ws{l}"]), rb(p[f"Wn{l}"])
        Z = Hb @ Ws.T + Mb @ Wn.T + p[f"b{l}"]
        Hn = np.maximum(Z, 0.0) * mask[:, None]
        cache.append((Hb, Mb, Ws, Wn, Z))
        H = Hn
    valid = mask > 0
    rsum = H[valid].sum(axis=0)
    amax = np.argmax(np.where(valid[:, None], H, -np.inf), axis=0)  # first maximum
    rmax = H[amax, np.arange(HID)]
    r = np.concatenate([rsum, rmax])
    y = p["Wo"] @ r + p["bo"]
    return y, (cache, H, r, amax, valid)


def backward_one(p: dict, A, mask, fw, dy, bf16: bool = False) -> dict:
    rb = bf16_round if bf16 else (lambda z: z)
    cache, H3, r, amax, valid = fw
    g = {"Wo": np.outer(dy, r), "bo": dy.copy()}
    dr = p["Wo"].T @ dy
    dH = np.zeros((N, HID))
    dH[valid] += dr[:HID]
    dH[amax, np.arange(HID)] += dr[HID:]
    for l in reversed(range(LAYERS)):
        Hb, Mb, Ws, Wn, Z = cache[l]
        dZ = dH * (Z > 0) * mask[:, None]
        g[f"Ws{l}"] = dZ.T @ Hb
        g[f"Wn{l}"] = dZ.T @ Mb
        g[f"b{l}"] = dZ.sum(axis=0)
        if l > 0:
            dZb = rb(dZ)
            P = rb(dZb @ Wn)
            dH = dZb @ Ws + A @ P
    return g


def loss_and_grads(p: dict, batch, targets: np.ndarray, bf16: bool = False):
    """batch: list of (X, A, mask); targets: [B, 2].  Mean squared error."""
    B = len(batch)
    total = 0.0
    grads = {k: np.zeros_like(v) for k, v in p.items()}
    preds = np.zeros((B, OUT))
    for b, (X, A, mask) in enumerate(batch):
        y, fw = forward_one(p, X, A, mask, bf16)
        preds[b] = y
        diff = y - targets[b]
        total += float(diff @ diff)
        dy = 2.0 * diff / (B * OUT)
        gb = backward_one(p, A, mask, fw, dy, bf16)
        for k in grads:
            grads[k] += gb[k]
    return total / (B * OUT), grads, preds


def flatten(p: dict) -> np.ndarray:
    """Parameters in the order the GPU buffer uses: per layer Ws, Wn, b; then Wo, bo."""
    parts = []
    for l in range(LAYERS):
        parts += [p[f"Ws{l}"].ravel(), p[f"Wn{l}"].ravel(), p[f"b{l}"].ravel()]
    parts += [p["Wo"].ravel(), p["bo"].ravel()]
    return np.concatenate(parts)


def unflatten(v: np.ndarray) -> dict:
    p, o = {}, 0
    for l in range(LAYERS):
        for name, shape in ((f"Ws{l}", (HID, HID)), (f"Wn{l}", (HID, HID)), (f"b{l}", (HID,))):
            size = int(np.prod(shape))
            p[name] = np.asarray(v[o:o + size], dtype=np.float64).reshape(shape)
            o += size
    p["Wo"] = np.asarray(v[o:o + OUT * 2 * HID], dtype=np.float64).reshape(OUT, 2 * HID)
    o += OUT * 2 * HID
    p["bo"] = np.asarray(v[o:o + OUT], dtype=np.float64)
    return p


N_PARAMS = LAYERS * (2 * HID * HID + HID) + OUT * 2 * HID + OUT
