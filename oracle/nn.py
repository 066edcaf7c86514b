"""Learned block preconditioner's network -- oracle (test infrastructure only).

A multilayer perceptron X -> relu(X W1^T + b1) -> relu(. W2^T + b2) ->
. W3^T + b3 with the row-weighted loss L = sum_rows w (O - T)^2 / (2 rows)
(w = 1 when no weights are given), written out with numpy:

* ``forward64`` / ``grads64``: FP64, the mathematical definition (checked
  against central finite differences in the tests);
* ``forward_bf16`` / ``grads_bf16``: FP32 arithmetic with the operands that
  the GPU kernels round to BF16 rounded the same way (round to nearest
  even), for element-wise comparison with the GPU.

Parameters use the library's layout [W1, b1, W2, b2, W3, b3] (row-major,
W_l of shape (rows_l, cols_l)).
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    out = (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(nan, np.float32(np.nan), out).astype(np.float32)


def shapes(k1, hidden, o_pad):
    return [(hidden, k1), (hidden, hidden), (o_pad, hidden)]


def unpack(flat, k1, hidden, o_pad):
    out, off = [], 0
    for (r, c) in shapes(k1, hidden, o_pad):
        W = np.asarray(flat[off: off + r * c]).reshape(r, c)
        off += r * c
        b = np.asarray(flat[off: off + r])
        off += r
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def relu(z):
    return np.maximum(z, 0)


# ----------------------------------------------------------------- FP64
def forward64(layers, X):
    (W1, b1), (W2, b2), (W3, b3) = layers
    Z1 = X @ W1.T + b1
    A1 = relu(Z1)
    Z2 = A1 @ W2.T + b2
    A2 = relu(Z2)
    return A2 @ W3.T + b3, (Z1, A1, Z2, A2)


def _w(W, rows):
    return np.ones(rows) if W is None else np.asarray(W, dtype=np.float64)


def loss64(layers, X, T, W=None):
    O, _ = forward64(layers, X)
    return 0.5 * np.sum(_w(W, X.shape[0])[:, None] * (O - T) ** 2) / X.shape[0]


def grads64(layers, X, T, W=None):
    (W1, b1), (W2, b2), (W3, b3) = layers
    O, (Z1, A1, Z2, A2) = forward64(layers, X)
    dO = _w(W, X.shape[0])[:, None] * (O - T) / X.shape[0]
    gW3, gb3 = dO.T @ A2, dO.sum(0)
    dZ2 = (dO @ W3) * (Z2 > 0)
    gW2, gb2 = dZ2.T @ A1, dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0)
    gW1, gb1 = dZ1.T @ X, dZ1.sum(0)
    return [(gW1, gb1), (gW2, gb2), (gW3, gb3)]


# ----------------------------------------------------------------- BF16 emulation
def forward_bf16(layers, X):
    """X: BF16-valued float32 features.  Mirrors the GPU rounding points."""
    (W1, b1), (W2, b2), (W3, b3) = [(bf16(W), np.float32(b)) for W, b in layers]
    X = X.astype(np.float32)
    Z1 = (X.astype(np.float64) @ W1.T.astype(np.float64)).astype(np.float32) + b1
    A1 = bf16(relu(Z1))
    Z2 = (A1.astype(np.float64) @ W2.T.astype(np.float64)).astype(np.float32) + b2
    A2 = bf16(relu(Z2))
    O = (A2.astype(np.float64) @ W3.T.astype(np.float64)).astype(np.float32) + b3
    return O, (Z1, A1, Z2, A2)


def grads_bf16(layers, X, T, W=None):
    Wb = [bf16(W) for W, _ in layers]
    O, (Z1, A1, Z2, A2) = forward_bf16(layers, X)
    rows = X.shape[0]
    w32 = np.float32(_w(W, rows))[:, None]
    dO = bf16((O - T.astype(np.float32)) * np.float32(1.0 / rows) * w32)
    f64 = lambda a: a.astype(np.float64)
    gW3 = f64(dO).T @ f64(A2)
    gb3 = f64(dO).sum(0)
    dZ2 = bf16(np.where(Z2 > 0, (f64(dO) @ f64(Wb[2])).astype(np.float32), 0))
    gW2 = f64(dZ2).T @ f64(A1)
    gb2 = f64(dZ2).sum(0)
    dZ1 = bf16(np.where(Z1 > 0, (f64(dZ2) @ f64(Wb[1])).astype(np.float32), 0))
    gW1 = f64(dZ1).T @ f64(X)
    gb1 = f64(dZ1).sum(0)
    loss = 0.5 * float(np.sum(f64(w32) * (f64(O) - f64(T)) ** 2)) / rows
    return [(gW1, gb1), (gW2, gb2), (gW3, gb3)], loss


# ----------------------------------------------------------------- features
def features(r_blocks, level_n, level_m, decay, n_max, m_max, k1, shift=0.0):
    """Features of every block of the residual r (shape [N][d][d], complex):
    nu_a = |r_a|_2, then [Re r_a/nu_a, Im r_a/nu_a, n_a/n_max, m_a/m_max,
    Re c_a/cs, Im c_a/cs, Re z/cs, Im z/cs] padded to k1, with cs = max |c_a|
    and z the shift of the system; a zero block has zero block features.
    Returns (X float64, nu)."""
    r = np.asarray(r_blocks, dtype=np.complex128)
    N, d, _ = r.shape
    nu = np.sqrt(np.sum(np.abs(r) ** 2, axis=(1, 2)))
    inv = np.where(nu > 1e-300, 1.0 / np.where(nu > 1e-300, nu, 1.0), 0.0)
    cs = np.max(np.abs(decay))
    X = np.zeros((N, k1))
    X[:, : d * d] = (r.real * inv[:, None, None]).reshape(N, -1)
    X[:, d * d: 2 * d * d] = (r.imag * inv[:, None, None]).reshape(N, -1)
    X[:, 2 * d * d] = level_n / max(n_max, 1)
    X[:, 2 * d * d + 1] = level_m / max(m_max, 1)
    X[:, 2 * d * d + 2] = decay.real / cs
    X[:, 2 * d * d + 3] = decay.imag / cs
    X[:, 2 * d * d + 4] = complex(shift).real / cs
    X[:, 2 * d * d + 5] = complex(shift).imag / cs
    return X, nu


def targets(r_blocks, e_blocks):
    """Training targets (e_a - r_a)/nu_a (zero for a zero block) and row
    weights nu_a^2 / mean_b nu_b^2 of residual blocks r and error blocks e;
    targets as [Re, Im] rows of length 2 d^2."""
    r = np.asarray(r_blocks, dtype=np.complex128)
    e = np.asarray(e_blocks, dtype=np.complex128)
    N, d, _ = r.shape
    nu = np.sqrt(np.sum(np.abs(r) ** 2, axis=(1, 2)))
    inv = np.where(nu > 1e-300, 1.0 / np.where(nu > 1e-300, nu, 1.0), 0.0)
    t = (e - r) * inv[:, None, None]
    T = np.concatenate([t.real.reshape(N, -1), t.imag.reshape(N, -1)], axis=1)
    m = np.mean(nu ** 2)
    W = nu ** 2 / m if m > 0 else np.zeros(N)
    return T, W


def precondition(r_blocks, g_rows):
    """The preconditioned blocks z_a = r_a + nu_a (g_re + i g_im) for network
    outputs g (rows of length >= 2 d^2)."""
    r = np.asarray(r_blocks, dtype=np.complex128)
    N, d, _ = r.shape
    nu = np.sqrt(np.sum(np.abs(r) ** 2, axis=(1, 2)))
    g = np.asarray(g_rows, dtype=np.float64)
    corr = (g[:, : d * d] + 1j * g[:, d * d: 2 * d * d]).reshape(N, d, d)
    return r + nu[:, None, None] * corr
