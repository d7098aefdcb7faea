"""The network's bf16 MFMA kernels against the CPU reference (oracle/mpnn_ref).

Tolerance: the reference rounds the same operands to bfloat16 and accumulates
in float64; the GPU accumulates in float32 (K = 64 terms, relative error about
64 * 2^-24 = 4e-6 before each bfloat16 rounding).  An intermediate value that
lands within that distance of a bfloat16 rounding boundary may round one
bfloat16 step (2^-8 relative) differently, which then propagates; a few such
flips per graph bound the difference by about 1e-2 of the largest value of
each block.  Both checks below use that bound.
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
