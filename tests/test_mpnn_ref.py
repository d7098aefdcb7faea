"""Pins of the CPU reference of the message-passing network.

* float64 gradients against central finite differences (every parameter
  block, several graphs, loss summed over a batch);
* bfloat16 rounding against hand-checked bit patterns;
* core numbers against closed forms (cliques, cycles, trees, grids).
"""
import numpy as np
import pytest

from oracle import mpnn_ref as M
from paper_1709_09990_amd import graphs as G


def _batch():
    gs = [G.gnp(12, 0.3, 1), G.partial_ktree(20, 4, 0.3, 2), G.rgg(30, 6.0, 3), G.grid(4, 5)]
    return [M.features(r) for r in gs]


def test_bf16_round_bits():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.0e-3])
    got = M.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 ** -7
    # 1 + 3*2^-8 is a tie between 1+2^-7 (odd) and 1+2^-6 (even)
    assert got[3] == 1.0 + 2 ** -6
    assert got[4] == -2.5 and got[5] == 0.0
    assert abs(got[6] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_core_numbers_closed_forms():
    assert list(M.core_numbers(G.complete(6))) == [5] * 6
    assert list(M.core_numbers(G.cycle(7))) == [2] * 7
    assert list(M.core_numbers(G.random_tree(9, 4))) == [1] * 9
    assert list(M.core_numbers(G.grid(3, 4))) == [2] * 12
    assert list(M.core_numbers(G.edgeless(3))) == [0] * 3
    # a triangle with a pendant vertex
    rows = G.from_edges(4, [(0, 1), (1, 2), (0, 2), (2, 3)])
    assert list(M.core_numbers(rows)) == [2, 2, 2, 1]


def test_gradients_match_finite_differences():
    p = M.init_params(7)
    batch = _batch()
    t = np.array([[0.3, 0.4], [0.2, 0.5], [0.25, 0.6], [0.2, 0.3]])
    loss, grads, _ = M.loss_and_grads(p, batch, t)
    rng = np.random.default_rng(3)
    eps = 1e-6
    for name in p:
        flat = p[name].ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            orig = flat[idx]
            flat[idx] = orig + eps
            lp, _, _ = M.loss_and_grads(p, batch, t)
            flat[idx] = orig - eps
            lm, _, _ = M.loss_and_grads(p, batch, t)
            flat[idx] = orig
            fd = (lp - lm) / (2 * eps)
            g = grads[name].ravel()[idx]
            assert abs(fd - g) <= 1e-6 + 1e-4 * abs(fd), (name, idx, fd, g)


def test_flatten_roundtrip():
    p = M.init_params(1)
    v = M.flatten(p)
    assert v.size == M.N_PARAMS
    q = M.unflatten(v)
    for k in p:
        assert np.array_equal(p[k], q[k])


def test_bf16_mode_close_to_float64():
    p = M.init_params(5)
    batch = _batch()
    t = np.array([[0.3, 0.4]] * 4)
    l64, g64, _ = M.loss_and_grads(p, batch, t, bf16=False)
    l16, g16, _ = M.loss_and_grads(p, batch, t, bf16=True)
    assert abs(l64 - l16) <= 0.05 * abs(l64) + 1e-4
    for k in g64:
        scale = np.abs(g64[k]).max() + 1e-12
        assert np.abs(g64[k] - g16[k]).max() <= 0.1 * scale, k
