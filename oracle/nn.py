"""Learned block preconditioner's network -- oracle (test infrastructure only).

A multilayer perceptron X -> relu(X W1^T + b1) -> relu(. W2^T + b2) ->
. W3^T + b3 with loss L = sum (O - T)^2 / (2 rows), written out with numpy:

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


def loss64(layers, X, T):
    O, _ = forward64(layers, X)
    return 0.5 * np.sum((O - T) ** 2) / X.shape[0]


def grads64(layers, X, T):
    (W1, b1), (W2, b2), (W3, b3) = layers
    O, (Z1, A1, Z2, A2) = forward64(layers, X)
    dO = (O - T) / X.shape[0]
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


def grads_bf16(layers, X, T):
    Wb = [bf16(W) for W, _ in layers]
    O, (Z1, A1, Z2, A2) = forward_bf16(layers, X)
    rows = X.shape[0]
    dO = bf16((O - T.astype(np.float32)) * np.float32(1.0 / rows))
    f64 = lambda a: a.astype(np.float64)
    gW3 = f64(dO).T @ f64(A2)
    gb3 = f64(dO).sum(0)
    dZ2 = bf16(np.where(Z2 > 0, (f64(dO) @ f64(Wb[2])).astype(np.float32), 0))
    gW2 = f64(dZ2).T @ f64(A1)
    gb2 = f64(dZ2).sum(0)
    dZ1 = bf16(np.where(Z1 > 0, (f64(dZ2) @ f64(Wb[1])).astype(np.float32), 0))
    gW1 = f64(dZ1).T @ f64(X)
    gb1 = f64(dZ1).sum(0)
    loss = 0.5 * float(np.sum((f64(O) - f64(T)) ** 2)) / rows
    return [(gW1, gb1), (gW2, gb2), (gW3, gb3)], loss


# ----------------------------------------------------------------- features
def features(r_blocks, diag_blocks, level_n, level_m, decay, n_max, m_max, k1, border=False):
    """Features of every block of r (shape [N][d][d], complex): Jacobi
    scaling jr = r / diag (diagonal of the system; the bordered element and
    exact zeros count as 1), nu = |jr_a|, then [Re jr/nu, Im jr/nu, n/n_max,
    m/m_max, Re c/cs, Im c/cs] padded to k1.  Returns (X float64, nu, jr)."""
    diag = np.array(diag_blocks, dtype=np.complex128, copy=True)
    if border:
        diag[0, 0, 0] = 1.0
    diag[diag == 0] = 1.0
    jr = r_blocks / diag
    N, d, _ = jr.shape
    nu = np.sqrt(np.sum(np.abs(jr) ** 2, axis=(1, 2)))
    nu[~(nu > 1e-300)] = 1.0
    cs = np.max(np.abs(decay))
    X = np.zeros((N, k1))
    X[:, : d * d] = (jr.real / nu[:, None, None]).reshape(N, -1)
    X[:, d * d: 2 * d * d] = (jr.imag / nu[:, None, None]).reshape(N, -1)
    X[:, 2 * d * d] = level_n / max(n_max, 1)
    X[:, 2 * d * d + 1] = level_m / max(m_max, 1)
    X[:, 2 * d * d + 2] = decay.real / cs
    X[:, 2 * d * d + 3] = decay.imag / cs
    return X, nu, jr
