"""Cost-model reference in float64 -- TEST INFRASTRUCTURE ONLY.

The model is dense 64 -> 128 -> 128 -> 1 with ReLU on both hidden layers and a
linear output, trained with the mean squared error; its weight matrices are
used in bf16 (rounded to nearest even from the fp32 master copy), its biases
in fp32.  This module computes the forward pass, the exact gradients of the
mean squared error by backpropagation and one Adam step (Kingma and Ba,
"Adam: a method for stochastic optimization", ICLR 2015) in float64, on the
same bf16-valued weights and inputs the device uses.  Written with numpy only;
it shares nothing with the device code.

Flat parameter layout (24961 floats): W1[128][64], b1[128], W2[128][128],
b2[128], W3[128], b3.
"""
from __future__ import annotations

import numpy as np

NPARAMS = 24961
SLICES = {"W1": (0, (128, 64)), "b1": (8192, (128,)), "W2": (8320, (128, 128)),
          "b2": (24704, (128,)), "W3": (24832, (128,)), "b3": (24960, ())}


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bf16 value (ties to even), returned as float32."""
    u = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32).astype(np.uint64)
    bias = ((u >> 16) & 1) + 0x7FFF
    r = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def unpack(params) -> dict:
    p = np.asarray(params, np.float64)
    out = {}
    for k, (o, shape) in SLICES.items():
        size = int(np.prod(shape)) if shape else 1
        out[k] = p[o:o + size].reshape(shape) if shape else p[o]
    return out


def pack(d: dict) -> np.ndarray:
    p = np.zeros(NPARAMS, np.float64)
    for k, (o, shape) in SLICES.items():
        size = int(np.prod(shape)) if shape else 1
        p[o:o + size] = np.asarray(d[k], np.float64).reshape(-1)
    return p


def working_weights(master_fp32) -> dict:
    """The weights the device computes with: W's rounded to bf16, biases as is."""
    m = np.asarray(master_fp32, np.float32)
    d = unpack(m)
    for k in ("W1", "W2", "W3"):
        o, shape = SLICES[k]
        d[k] = bf16_round(m[o:o + int(np.prod(shape))]).astype(np.float64).reshape(shape)
    return d


def forward(w: dict, X):
    """y = W3 . relu(W2 relu(W1 x + b1) + b2) + b3 for each row x of X."""
    X = np.asarray(X, np.float64)
    z1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["W3"] + w["b3"]
    return y, (X, z1, h1, z2, h2)


def loss_and_grads(w: dict, X, t):
    """Mean squared error and its gradients with respect to every parameter."""
    y, (X, z1, h1, z2, h2) = forward(w, X)
    t = np.asarray(t, np.float64)
    n = y.shape[0]
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / n                       # dL/dy
    g = {"W3": h2.T @ dy, "b3": dy.sum()}
    dz2 = np.outer(dy, w["W3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ w["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(master, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of flat arrays; step counts from 1."""
    master, grad = np.asarray(master, np.float64), np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * grad
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v
