"""Pins of the oracle's network (CPU only): BF16 rounding against an
independent implementation, FP64 gradients against central finite
differences, and the BF16 emulation against FP64."""
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


def test_grads64_against_central_differences():
    layers, X, T = _small(1)
    g = onn.pack(onn.grads64(layers, X, T))
    p = onn.pack(layers)
    shp = onn.shapes(X.shape[1], layers[0][0].shape[0], layers[2][0].shape[0])
    rng = np.random.default_rng(2)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp = onn.loss64(onn.unpack(pp, X.shape[1], shp[0][0], shp[2][0]), X, T)
        lm = onn.loss64(onn.unpack(pm, X.shape[1], shp[0][0], shp[2][0]), X, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_emulation_close_to_fp64():
    layers, X, T = _small(3, rows=64)
    Xb = onn.bf16(X)
    g64 = onn.pack(onn.grads64(layers, Xb.astype(np.float64), T))
    gb, _ = onn.grads_bf16(layers, Xb, T)
    gb = onn.pack(gb)
    assert np.linalg.norm(gb - g64) <= 2e-2 * np.linalg.norm(g64)
