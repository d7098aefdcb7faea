"""The network's bf16 MFMA kernels against the CPU reference (oracle/mpnn_ref).

Product by product (test_every_product_within_its_bound): tw_mpnn_trace hands
back the kernels' float32 value of every product before its bfloat16 rounding.
Each product is recomputed in float64 from the GPU's own bfloat16 operands (the
bfloat16 rounding of the GPU's previous float32 value, which the reference
applies itself), so no earlier rounding difference can carry over, and the GPU
value must lie within the float32 accumulation bound of that one product:
|c_gpu - c_ref| <= K * 2^-24 * sum_k |a_k b_k| for K terms (each bf16 x bf16
product is exact in float32; each of the K additions rounds once).  A reference
that skips a rounding point (A H kept in float32, weights kept in float32, dZ
kept in float32) misses this bound by about 2^-9 / (K 2^-24), a factor of tens:
the planted variants below must fail.

End to end (predictions, summed gradients): the reference rounds at the same
points from its own values, so an intermediate within float32 noise of a
bfloat16 rounding boundary can land one bfloat16 step (2^-8 relative) apart and
carry over to later layers; there a relative bound of 1e-2 of each block's
largest value applies.
"""
import numpy as np
import pytest

from oracle import mpnn_ref as M
from paper_1709_09990_amd import graphs as G

pytestmark = pytest.mark.gpu


def _graphs(count, seed):
    return G.workload_batch(count, seed0=seed, n_lo=6, n_hi=56)


def _targets(count, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0.1, 0.5, count), rng.uniform(0.2, 0.8, count)], axis=1)


def test_predictions_match_reference():
    from paper_1709_09990_amd import tw as T
    p = M.init_params(11)
    graphs = _graphs(24, 41000)
    with T.Mpnn(M.flatten(p).astype(np.float32)) as net:
        # the device keeps float32 masters: compare against the reference on the same values
        p32 = M.unflatten(net.params().astype(np.float64))
        got = net.predict(graphs)
    for rows, y in zip(graphs, got):
        X, A, mask = M.features(rows)
        ref, _ = M.forward_one(p32, X, A, mask, bf16=True)
        assert np.all(np.abs(y - ref) <= 1e-2 * (np.abs(ref) + 0.05)), (y, ref)


def test_gradients_match_reference():
    from paper_1709_09990_amd import tw as T
    p = M.init_params(12)
    graphs = _graphs(16, 42000)
    t = _targets(16, 3)
    with T.Mpnn(M.flatten(p).astype(np.float32)) as net:
        p32 = M.unflatten(net.params().astype(np.float64))
        loss, g = net.gradients(graphs, t)
    batch = [M.features(r) for r in graphs]
    ref_loss, ref_g, _ = M.loss_and_grads(p32, batch, t, bf16=True)
    assert abs(loss - ref_loss) <= 1e-2 * abs(ref_loss) + 1e-5
    got = M.unflatten(g.astype(np.float64))
    for k in ref_g:
        scale = np.abs(ref_g[k]).max()
        assert np.abs(got[k] - ref_g[k]).max() <= 1e-2 * scale + 1e-7, k


def test_training_reduces_loss():
    from paper_1709_09990_amd import tw as T
    p = M.init_params(13)
    graphs = _graphs(64, 43000)
    t = _targets(64, 4)
    with T.Mpnn(M.flatten(p).astype(np.float32)) as net:
        first = net.train_step(graphs, t, lr=3e-3)
        for _ in range(60):
            last = net.train_step(graphs, t, lr=3e-3)
    assert last < 0.5 * first, (first, last)


U = 2.0 ** -24


def _check_trace(p, rows, target, tr, grads, plant=None):
    """Checks one graph's trace product by product; returns the name of the
    first product outside its bound (None if all hold).  plant names a
    rounding point the check skips on purpose: 'AH' (A H_l kept in float32),
    'W' (weights kept in float32), 'dZ' (dZ_l kept in float32)."""
    rb = M.bf16_round
    X, A, mask = M.features(rows)
    n = len(rows)

    def within(got, ref, absref, K):
        return bool(np.all(np.abs(got - ref) <= K * U * absref + 1e-30))

    Hb = rb(X)
    Hbs, Mbs, Ws_, Wn_ = [], [], [], []
    H = None
    for l in range(3):
        Ws = p[f"Ws{l}"] if plant == "W" else rb(p[f"Ws{l}"])
        Wn = p[f"Wn{l}"] if plant == "W" else rb(p[f"Wn{l}"])
        Mref = A @ Hb
        if not within(tr["M"][l], Mref, A @ np.abs(Hb), 64):
            return f"AH{l}"
        Mb = tr["M"][l] if plant == "AH" else rb(tr["M"][l])
        Zref = Hb @ Ws.T + Mb @ Wn.T + p[f"b{l}"]
        absZ = np.abs(Hb) @ np.abs(Ws).T + np.abs(Mb) @ np.abs(Wn).T + np.abs(p[f"b{l}"])
        if not within(tr["Z"][l], Zref, absZ, 129):
            return f"Z{l}"
        Hbs.append(Hb)
        Mbs.append(Mb)
        Ws_.append(Ws)
        Wn_.append(Wn)
        H = np.maximum(tr["Z"][l], 0.0) * mask[:, None]
        Hb = rb(H)
    # readout: sum in float32 over the n nodes, maximum exact
    rsum = H[:n].sum(axis=0)
    if not within(tr["r"][:64], rsum, np.abs(H[:n]).sum(axis=0), n):
        return "r_sum"
    if not np.array_equal(tr["r"][64:], H[:n].max(axis=0)):
        return "r_max"
    amax = np.argmax(H[:n], axis=0)
    y = p["Wo"] @ tr["r"] + p["bo"]
    if not within(tr["y"], y, np.abs(p["Wo"]) @ np.abs(tr["r"]) + np.abs(p["bo"]), 129):
        return "y"
    # dL/dy for the mean of two squares; the device holds the targets in float32
    d = tr["y"] - np.asarray(target, dtype=np.float32).astype(np.float64)
    dr = p["Wo"].T @ d
    dH = mask[:, None] * dr[None, :64]
    dH[amax, np.arange(64)] += dr[64:]
    absdH = mask[:, None] * (np.abs(p["Wo"][:, :64]).T @ np.abs(d))[None, :]
    absdH[amax, np.arange(64)] += np.abs(p["Wo"][:, 64:]).T @ np.abs(d)
    if not within(tr["dH3"], dH, absdH + np.abs(dH), 8):
        return "dH3"
    g = M.unflatten(grads.astype(np.float64))
    if not within(g["Wo"], np.outer(d, tr["r"]), np.abs(np.outer(d, tr["r"])), 4):
        return "gWo"
    dH = tr["dH3"]
    Hnext = [rb(np.maximum(tr["Z"][l], 0.0) * mask[:, None]) for l in range(3)]
    for l in (2, 1, 0):
        on = (Hnext[l] > 0).astype(np.float64)
        dZ = dH * on * mask[:, None]
        if not np.array_equal(tr["dZ"][l], dZ):
            return f"dZ{l}"
        dZb = tr["dZ"][l] if plant == "dZ" else rb(tr["dZ"][l])
        if not within(g[f"b{l}"], tr["dZ"][l].sum(axis=0), np.abs(tr["dZ"][l]).sum(axis=0), 64):
            return f"gb{l}"
        if not within(g[f"Ws{l}"], dZb.T @ Hbs[l], np.abs(dZb).T @ np.abs(Hbs[l]), 64):
            return f"gWs{l}"
        if not within(g[f"Wn{l}"], dZb.T @ Mbs[l], np.abs(dZb).T @ np.abs(Mbs[l]), 64):
            return f"gWn{l}"
        if l == 0:
            break
        P = dZb @ Wn_[l]
        if not within(tr["P"][l], P, np.abs(dZb) @ np.abs(Wn_[l]), 64):
            return f"P{l}"
        Pb = rb(tr["P"][l])
        dHref = dZb @ Ws_[l] + A @ Pb
        if not within(tr["dH"][l], dHref, np.abs(dZb) @ np.abs(Ws_[l]) + A @ np.abs(Pb), 128):
            return f"dH{l}"
        dH = tr["dH"][l]
    return None


def test_every_product_within_its_bound():
    """12 graphs (n 6..56), parameters from three seeds and after training
    steps: every product of the forward and backward pass is within the
    float32 accumulation bound of its own bfloat16 operands."""
    from paper_1709_09990_amd import tw as T
    graphs = _graphs(12, 47000)
    t = _targets(12, 5)
    checked = 0
    for seed in (21, 22, 23):
        with T.Mpnn(M.flatten(M.init_params(seed)).astype(np.float32)) as net:
            if seed == 23:
                for _ in range(5):
                    net.train_step(graphs, t, lr=3e-3)
            p = M.unflatten(net.params().astype(np.float64))
            for rows, target in zip(graphs, t):
                tr, g = net.trace(rows, target)
                assert _check_trace(p, rows, target, tr, g) is None
                checked += 1
    assert checked == 36


@pytest.mark.parametrize("plant", ["AH", "W", "dZ"])
def test_planted_rounding_mistakes_fail(plant):
    """A reference that skips one bfloat16 rounding point misses the bound."""
    from paper_1709_09990_amd import tw as T
    graphs = _graphs(4, 48000)
    t = _targets(4, 6)
    with T.Mpnn(M.flatten(M.init_params(31)).astype(np.float32)) as net:
        p = M.unflatten(net.params().astype(np.float64))
        fails = 0
        for rows, target in zip(graphs, t):
            tr, g = net.trace(rows, target)
            assert _check_trace(p, rows, target, tr, g) is None
            fails += _check_trace(p, rows, target, tr, g, plant=plant) is not None
    assert fails == len(graphs), (plant, fails)
