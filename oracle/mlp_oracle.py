"""FP64 reference of the weight-window network (test infrastructure only).

A fully connected network 8 -> 64 -> 64 -> 64 -> 1 with tanh on the hidden
layers and a linear output, trained on a weighted mean-squared error with
Adam.  Written plainly in NumPy float64; the GPU library's FP32 MFMA training
kernels and BF16 MFMA inference kernel are checked against it.  Pinned by
central finite differences and Adam's closed-form first step
(tests/test_oracle_mlp.py).

Flat parameter layout (shared with the C ABI, which documents it):
    W1 [8][64], b1 [64], W2 [64][64], b2 [64], W3 [64][64], b3 [64],
    w4 [64], b4 [1]            (W[k][j]: input k to output j)
"""
from __future__ import annotations

import numpy as np

WIDTHS = (8, 64, 64, 64, 1)
SHAPES = [(8, 64), (64,), (64, 64), (64,), (64, 64), (64,), (64,), (1,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta, X):
    """Returns the output y [n] and the hidden activations."""
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(theta)
    H1 = np.tanh(X @ W1 + b1)
    H2 = np.tanh(H1 @ W2 + b2)
    H3 = np.tanh(H2 @ W3 + b3)
    y = H3 @ w4 + b4[0]
    return y, (H1, H2, H3)


def loss(theta, X, t, wts):
    y, _ = forward(theta, X)
    return float(np.sum(wts * (y - t) ** 2))


def loss_and_grad(theta, X, t, wts):
    """Weighted squared error L = sum_i w_i (y_i - t_i)^2 and dL/dtheta by
    the chain rule through the three tanh layers."""
    X = np.asarray(X, dtype=np.float64)
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(theta)
    y, (H1, H2, H3) = forward(theta, X)
    r = y - t
    L = float(np.sum(wts * r * r))
    dy = 2.0 * wts * r                        # dL/dy
    gw4 = H3.T @ dy
    gb4 = np.array([dy.sum()])
    dZ3 = np.outer(dy, w4) * (1.0 - H3 * H3)
    gW3 = H2.T @ dZ3
    gb3 = dZ3.sum(axis=0)
    dZ2 = (dZ3 @ W3.T) * (1.0 - H2 * H2)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * (1.0 - H1 * H1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3, gw4, gb4])


def adam(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015); step counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, X, t, wts, steps, lr):
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for s in range(1, steps + 1):
        L, g = loss_and_grad(theta, X, t, wts)
        losses.append(L)
        theta, m, v = adam(theta, g, m, v, s, lr)
    return theta, np.array(losses)


def bf16(a):
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    """Inference with weights and activations rounded to bfloat16, biases
    kept in float32, exact (FP64 here) accumulation, tanh on the accumulated
    value."""
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(theta)
    H = bf16(X)
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        H = bf16(np.tanh(H @ bf16(W) + b.astype(np.float32).astype(np.float64)))
    return H @ bf16(w4) + float(np.float32(b4[0]))
