"""Pins of the oracle's network (CPU only): BF16 rounding against an
independent implementation, FP64 gradients of the row-weighted loss against
central finite differences, the BF16 emulation against FP64, and the
features, targets, weights and preconditioned blocks on a case computed by
hand."""
import numpy as np
import pytest
import torch

from oracle import nn as onn


def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(onn.bf16(x), ref)
    one = np.float32(1.0)
    assert onn.bf16(np.float32(1 + 2.0 ** -8)) == one                      # tie -> even (1.0)
    assert onn.bf16(np.float32(1 + 3 * 2.0 ** -8)) == np.float32(1 + 2.0 ** -6)  # tie -> even (odd below)
    assert onn.bf16(np.float32(1 + 2.0 ** -8 + 2.0 ** -20)) == np.float32(1 + 2.0 ** -7)


def _small(seed, k1=40, hidden=32, o_pad=32, rows=7):
    rng = np.random.default_rng(seed)
    layers = [(rng.standard_normal((r, c)) * 0.3, rng.standard_normal(r) * 0.1)
              for r, c in onn.shapes(k1, hidden, o_pad)]
    X = rng.standard_normal((rows, k1))
    T = rng.standard_normal((rows, o_pad))
    return layers, X, T


@pytest.mark.parametrize("weighted", [False, True])
def test_grads64_against_central_differences(weighted):
    layers, X, T = _small(1)
    W = np.random.default_rng(5).uniform(0.1, 3.0, X.shape[0]) if weighted else None
    g = onn.pack(onn.grads64(layers, X, T, W))
    p = onn.pack(layers)
    shp = onn.shapes(X.shape[1], layers[0][0].shape[0], layers[2][0].shape[0])
    rng = np.random.default_rng(2)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp = onn.loss64(onn.unpack(pp, X.shape[1], shp[0][0], shp[2][0]), X, T, W)
        lm = onn.loss64(onn.unpack(pm, X.shape[1], shp[0][0], shp[2][0]), X, T, W)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_emulation_close_to_fp64():
    layers, X, T = _small(3, rows=64)
    W = np.random.default_rng(6).uniform(0.1, 3.0, 64)
    Xb = onn.bf16(X)
    g64 = onn.pack(onn.grads64(layers, Xb.astype(np.float64), T, W))
    gb, loss = onn.grads_bf16(layers, Xb, T, W)
    gb = onn.pack(gb)
    assert np.linalg.norm(gb - g64) <= 2e-2 * np.linalg.norm(g64)
    assert abs(loss - onn.loss64(layers, Xb.astype(np.float64), T, W)) <= 2e-2 * loss


def test_features_targets_weights_by_hand():
    """d = 2, three blocks worked out by hand: r_0 = [[3, 0], [0, 4i]]
    (|r_0| = 5), r_1 = 0 (a converged block), r_2 = [[0, 1], [0, 0]];
    decays 0, 2 + 1i, 4 - 2i (cs = |4 - 2i| = sqrt 20); levels (n, m) =
    (0, 0), (1, 0), (2, 1) with n_max = 2, m_max = 1; shift z = 0.5i."""
    r = np.zeros((3, 2, 2), complex)
    r[0] = [[3, 0], [0, 4j]]
    r[2] = [[0, 1], [0, 0]]
    decay = np.array([0, 2 + 1j, 4 - 2j])
    cs = np.sqrt(20.0)
    X, nu = onn.features(r, np.array([0, 1, 2]), np.array([0, 0, 1]), decay, 2, 1, k1=16, shift=0.5j)
    assert np.allclose(nu, [5.0, 0.0, 1.0])
    row0 = [0.6, 0, 0, 0,  0, 0, 0, 0.8,  0.0, 0.0,  0.0, 0.0,  0.0, 0.5 / cs,  0, 0]
    row1 = [0, 0, 0, 0,  0, 0, 0, 0,  0.5, 0.0,  2 / cs, 1 / cs,  0.0, 0.5 / cs,  0, 0]
    row2 = [0, 1, 0, 0,  0, 0, 0, 0,  1.0, 1.0,  4 / cs, -2 / cs,  0.0, 0.5 / cs,  0, 0]
    assert np.allclose(X, [row0, row1, row2])
    # error blocks: e = r + correction
    e = r.copy()
    e[0] += [[1, 0], [0, 0]]          # correction 1 on a block of norm 5 -> target 0.2
    e[1] += [[0, 0], [1j, 0]]         # zero residual: target 0 (not predictable), weight 0
    e[2] += [[0, -2], [0, 0]]         # correction -2 on a block of norm 1
    T, W = onn.targets(r, e)
    assert np.allclose(T[0], [0.2, 0, 0, 0, 0, 0, 0, 0])
    assert np.allclose(T[1], 0)
    assert np.allclose(T[2], [0, -2, 0, 0, 0, 0, 0, 0])
    assert np.allclose(W, np.array([25.0, 0.0, 1.0]) / (26.0 / 3.0))
    # the preconditioned blocks with the exact targets as outputs reproduce e
    # on every block that has a residual; the zero block stays zero
    z = onn.precondition(r, T)
    assert np.allclose(z[0], e[0]) and np.allclose(z[2], e[2]) and np.allclose(z[1], 0)
    # a zero network is the identity
    assert np.allclose(onn.precondition(r, np.zeros_like(T)), r)
