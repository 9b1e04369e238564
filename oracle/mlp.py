"""The learned-null threshold network in FP64 (test infrastructure only).

A 16 -> 64 -> 64 -> 2 multilayer perceptron with ReLU hidden activations maps
a step's feature vector to its predicted surrogate max-statistic thresholds
(tau_0.05 and tau_0.01, each scaled by sqrt(N)).  The paper does not describe
a learned null (it only says that surrogate null distributions gate parent
selection, Summary, network-inference paragraph); the network shape and the
BF16-weights / FP32-accumulate arithmetic are the library's own choices.
The oracle evaluates it in FP64 on the *same* BF16-rounded parameters that
the device uses.

Flat parameter layout (5,378 values):
  W1 [64][16] | b1 [64] | W2 [64][64] | b2 [64] | W3 [2][64] | b3 [2]
Loss: L = (1/B) sum_b sum_o 0.5 (out_bo - t_bo)^2.
Adam: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected (Kingma & Ba 2015).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 16, 64, 2
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 5378


def bf16_round(a) -> np.ndarray:
    """Round FP32 values to the nearest BF16 value (ties to even), returned as FP32."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (rounded & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = flat[off:off + n].reshape(shape)
        off += n
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SIZES])


def forward(flat, feats):
    """FP64 forward pass.  feats [B][16] -> (out [B][2], cache)."""
    p = unpack(flat)
    f = np.asarray(feats, dtype=np.float64)
    a1 = f @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    out = h2 @ p["W3"].T + p["b3"]
    return out, (f, a1, h1, a2, h2)


def loss(flat, feats, targets) -> float:
    out, _ = forward(flat, feats)
    t = np.asarray(targets, dtype=np.float64)
    return float(0.5 * np.sum((out - t) ** 2) / out.shape[0])


def backward(flat, feats, targets) -> np.ndarray:
    """Gradient of ``loss`` with respect to the flat parameter vector (FP64)."""
    p = unpack(flat)
    out, (f, a1, h1, a2, h2) = forward(flat, feats)
    B = out.shape[0]
    g_out = (out - np.asarray(targets, dtype=np.float64)) / B
    g = {}
    g["W3"] = g_out.T @ h2
    g["b3"] = g_out.sum(axis=0)
    g_h2 = g_out @ p["W3"]
    g_a2 = g_h2 * (a2 > 0)
    g["W2"] = g_a2.T @ h1
    g["b2"] = g_a2.sum(axis=0)
    g_h1 = g_a2 @ p["W2"]
    g_a1 = g_h1 * (a1 > 0)
    g["W1"] = g_a1.T @ f
    g["b1"] = g_a1.sum(axis=0)
    return pack(g)


def adam_step(master, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of FP64 copies; returns new (master, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v

