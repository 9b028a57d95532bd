"""FP64 reference of the learned proposal's network -- TEST INFRASTRUCTURE ONLY.

Network 6 -> 128 -> 128 -> 128 -> 4 with ReLU and a softmax over the outcome
classes (quench, r1, r2, dissociation), softmax cross-entropy loss averaged
over the batch, Adam (Kingma & Ba 2015).  Plain numpy, written as the
definitions read; the optional `bf16` flag rounds the operands of every matrix
product to bfloat16 (round to nearest even) at the points where the GPU
kernels round them, so that GPU results can be compared at FP32-accumulation
accuracy.

Flat parameter layout (float): W1[6][128], b1[128], W2[128][128], b2[128],
W3[128][128], b3[128], W4[128][4], b4[4] (W[i][o]: input-major).
"""
from __future__ import annotations

import numpy as np

SIZES = [(6, 128), (128, 128), (128, 128), (128, 4)]
NPARAM = sum(i * o + o for i, o in SIZES)   # 34,436


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for i, o in SIZES:
        W = theta[off:off + i * o].reshape(i, o)
        off += i * o
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16(a):
    """Round float values to bfloat16 (round to nearest, ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, x, use_bf16=False):
    """Returns (logits, probabilities, cache)."""
    L = unpack(theta)
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    h = r(x)
    cache = {"h": [h]}
    for k, (W, b) in enumerate(L):
        z = h @ r(W) + b
        if k < 3:
            h = r(np.maximum(z, 0.0))
            cache["h"].append(h)
            cache.setdefault("z", []).append(z)
        else:
            logits = z
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    p = e / e.sum(axis=1, keepdims=True)
    cache["p"] = p
    return logits, p, cache


def loss(theta, x, y, use_bf16=False):
    _, p, _ = forward(theta, x, use_bf16)
    return float(-np.mean(np.log(p[np.arange(len(y)), y])))


def backward(theta, x, y, use_bf16=False):
    """Gradient of the mean softmax cross-entropy; returns (loss, grad flat)."""
    L = unpack(theta)
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    _, p, c = forward(theta, x, use_bf16)
    n = len(y)
    onehot = np.zeros_like(p)
    onehot[np.arange(n), y] = 1.0
    lval = float(-np.mean(np.log(p[np.arange(n), y])))
    dz = (p - onehot) / n                 # d loss / d logits
    grads = [None] * 4
    for k in range(3, -1, -1):
        W, b = L[k]
        h = c["h"][k]
        dzr = r(dz)
        grads[k] = (h.T @ dzr, dz.sum(axis=0))
        if k > 0:
            dh = dzr @ r(W).T
            dz = dh * (c["z"][k - 1] > 0.0)
    return lval, pack(grads)


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def he_uniform(seed):
    """Reference initialisation: W ~ U(-sqrt(6/fan_in), sqrt(6/fan_in)), b = 0."""
    rng = np.random.default_rng(seed)
    layers = []
    for i, o in SIZES:
        lim = np.sqrt(6.0 / i)
        layers.append((rng.uniform(-lim, lim, size=(i, o)), np.zeros(o)))
    return pack(layers)
