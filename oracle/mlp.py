"""FP64 reference of the boundary-closure network (not in the paper).

TEST INFRASTRUCTURE: only tests, the package smoke check and the benchmark's CPU-baseline
leg may import this module.

The network maps a strip of post-collision populations (3 cells deep along the inward
normal, Q values each, in the canonical face frame) to the k populations that enter the box
through the face:  x -> s = rms(x),  z = x / s,
    h1 = relu(z W1 + b1),  h2 = relu(h1 W2 + b2),  y = h2 W3 + b3,  output = s * y.
The rms is taken as m sqrt(mean((x/m)^2)) with m = max |x| (no underflow for tiny strips);
an all-zero strip has s = 0, z = 0 and predicts 0 (the scheme is linear).
Training minimises the mean squared error between y and target / s over samples with s > 0
(Adam).

`quantize=True` rounds every GEMM input to bfloat16 with round-to-nearest-even, as the GPU
kernels do before their matrix-core products: weights, the normalised strip, the hidden
activations, and in the backward pass the output and pre-activation gradients (bias
gradients are sums of those rounded gradients).  Accumulation stays FP64 here.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(rng, n_in: int, n_out: int, hidden: int = 64) -> dict:
    """He-normal weights, zero biases."""
    return dict(
        W1=rng.standard_normal((n_in, hidden)) * np.sqrt(2.0 / n_in), b1=np.zeros(hidden),
        W2=rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden), b2=np.zeros(hidden),
        W3=rng.standard_normal((hidden, n_out)) * np.sqrt(1.0 / hidden), b3=np.zeros(n_out),
    )


def normalise(x):
    """(z, s): s = rms of each row (computed scaled by the row's max |x|), z = x / s (0 if s = 0)."""
    x = np.asarray(x, dtype=np.float64)
    m = np.abs(x).max(axis=1, keepdims=True)
    safe = np.where(m > 0, m, 1.0)
    s = np.where(m > 0, m * np.sqrt(np.mean((x / safe) ** 2, axis=1, keepdims=True)), 0.0)
    z = np.where(s > 0, x / np.where(s > 0, s, 1.0), 0.0)
    return z, s


def forward(p: dict, z, quantize: bool = False):
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    z = q(z)
    a1 = z @ q(p["W1"]) + p["b1"]
    h1 = np.maximum(a1, 0.0)
    h1q = q(h1)
    a2 = h1q @ q(p["W2"]) + p["b2"]
    h2 = np.maximum(a2, 0.0)
    h2q = q(h2)
    y = h2q @ q(p["W3"]) + p["b3"]
    return y, dict(z=z, a1=a1, h1=h1q, a2=a2, h2=h2q)


def mse(y, t, valid=None) -> float:
    """Mean of (y - t)^2 over the valid rows (all rows if valid is None) and all outputs."""
    if valid is None:
        return float(np.mean((y - t) ** 2))
    v = np.asarray(valid, dtype=bool).reshape(-1)
    return float(np.sum((y[v] - t[v]) ** 2) / (v.sum() * y.shape[1])) if v.any() else 0.0


def backward(p: dict, cache: dict, y, t, quantize: bool = False, valid=None) -> dict:
    """Gradients of mse(y, t, valid) by the chain rule."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    B, k = y.shape
    v = np.ones(B, dtype=bool) if valid is None else np.asarray(valid, dtype=bool).reshape(-1)
    nv = max(int(v.sum()), 1)
    dy = q(2.0 * (y - t) / (nv * k) * v[:, None])
    g = {}
    g["W3"] = cache["h2"].T @ dy
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ q(p["W3"]).T
    da2 = q(dh2 * (cache["a2"] > 0))
    g["W2"] = cache["h1"].T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ q(p["W2"]).T
    da1 = q(dh1 * (cache["a1"] > 0))
    g["W1"] = cache["z"].T @ da1
    g["b1"] = da1.sum(axis=0)
    return g


def flat(p: dict) -> np.ndarray:
    """Parameters in the library's order: W1 (n_in x 64, row-major), b1, W2, b2, W3 (64 x k), b3."""
    return np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unflat(v, n_in: int, n_out: int, hidden: int = 64) -> dict:
    shapes = [("W1", (n_in, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
              ("W3", (hidden, n_out)), ("b3", (n_out,))]
    out, o = {}, 0
    for key, shp in shapes:
        n = int(np.prod(shp))
        out[key] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    assert o == len(v)
    return out


def adam(p: dict, g: dict, m: dict, v: dict, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8) -> None:
    """One Adam update (Kingma & Ba) of every parameter, in place; t counts from 1."""
    for key in p:
        m[key] = b1 * m[key] + (1 - b1) * g[key]
        v[key] = b2 * v[key] + (1 - b2) * g[key] ** 2
        mh = m[key] / (1 - b1 ** t)
        vh = v[key] / (1 - b2 ** t)
        p[key] = p[key] - lr * mh / (np.sqrt(vh) + eps)


def predict(p: dict, strips, quantize: bool = False):
    """Incoming populations for raw strips (B, 3Q): network on the normalised strip, rescaled."""
    z, s = normalise(strips)
    y, _ = forward(p, z, quantize)
    return y * s
