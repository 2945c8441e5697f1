"""FP64 CPU oracle of the sample-count predictor network (test infrastructure only).

Only tests/, __graft_entry__.smoke() and the bench's CPU-baseline leg may import this
module; the product path never does. It shares no code with the HIP library.

Network (the predictor of the initial number of training states, which the paper leaves
open in Sec. 3 and Sec. 5): x [64] -> h1 = relu(W1 x + b1) [128] -> h2 = relu(W2 h1 + b2)
[128] -> y = W3 h2 + b3 [2]. The weights used by every pass are the bfloat16 roundings
(round to nearest, ties to even) of the FP32 master weights; arithmetic here is FP64.

Loss per row, mean over rows:
    [t0 finite] * (y0 - t0)^2 / 2  +  softplus(y1) - t1 * y1
(squared error on log2 M where a label exists, binary cross-entropy of the logit y1
against the success fraction t1).

Parameter vector layout (FP32): W1 [128][64], b1 [128], W2 [128][128], b2 [128],
W3 [2][128], b3 [2].
"""
from __future__ import annotations

import numpy as np

F, H, O = 64, 128, 2
SIZES = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (O, H)), ("b3", (O,))]
NUM_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def bf16_round(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    exp_all_ones = (u & 0x7F800000) == 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = exp_all_ones & ((u & 0x7FFFFF) != 0)
    r = np.where(exp_all_ones, (u >> 16) << 16, r)
    r = np.where(nan, r | (0x40 << 16), r)
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def unpack(theta):
    """Split a flat parameter vector into named arrays (FP64 copies)."""
    out, o = {}, 0
    theta = np.asarray(theta, dtype=np.float64)
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def forward(theta, X):
    """Outputs y [B][2] and the intermediate values, in FP64 from the given weights."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.maximum(z2, 0.0)
    y = a2 @ p["W3"].T + p["b3"]
    return y, dict(X=X, z1=z1, a1=a1, z2=z2, a2=a2)


def loss(theta, X, T):
    y, _ = forward(theta, X)
    T = np.asarray(T, dtype=np.float64)
    B = len(y)
    lab = np.isfinite(T[:, 0])
    d0 = np.where(lab, y[:, 0] - np.where(lab, T[:, 0], 0.0), 0.0)
    sp = np.logaddexp(0.0, y[:, 1])  # softplus
    return float((0.5 * d0 @ d0 + np.sum(sp - T[:, 1] * y[:, 1])) / B)


def gradient(theta, X, T):
    """Analytic gradient of `loss` by the chain rule, layer by layer."""
    p = unpack(theta)
    y, c = forward(theta, X)
    T = np.asarray(T, dtype=np.float64)
    B = len(y)
    lab = np.isfinite(T[:, 0])
    dy = np.zeros_like(y)
    dy[:, 0] = np.where(lab, y[:, 0] - np.where(lab, T[:, 0], 0.0), 0.0) / B
    dy[:, 1] = (1.0 / (1.0 + np.exp(-y[:, 1])) - T[:, 1]) / B
    g = {"W3": dy.T @ c["a2"], "b3": dy.sum(0)}
    dz2 = (dy @ p["W3"]) * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["a1"]
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["X"]
    g["b1"] = dz1.sum(0)
    return pack(g)


def effective(theta32):
    """The weights the passes use: bfloat16 roundings of the FP32 masters, as FP64."""
    return bf16_round(np.asarray(theta32, dtype=np.float32)).astype(np.float64)
