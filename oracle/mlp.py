"""CPU FP64 reference of the pricing surrogate's network -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py may import this module. The HIP product
path never calls it and shares no code with it.

The surrogate is a project addition (the paper has no learned component). Its network maps
seven inputs (the five Heston parameters, the maturity T and the log-moneyness k) to the
call price divided by S0:

  xn = (x - shift) * scale                      (fixed affine normalisation)
  a1 = silu(W1 xn + b1)                         (7 -> 256)
  a2 = silu(W2 a1 + b2), a3, a4 likewise        (256 -> 256, three times)
  y  = W5 a4 + b5                               (256 -> 1)

with silu(z) = z / (1 + e^-z) (Elfwing, Uchibe and Doya 2018). Training minimises the
mean squared error L = (1/B) sum_b (y_b - t_b)^2 with Adam (Kingma and Ba 2015,
Algorithm 1, bias-corrected moments). Everything here is the plain textbook definition in
float64: a matrix product per layer, the chain rule written out layer by layer, and the
Adam update elementwise.

Parameter vector layout (shared with the HIP side as an interface, each side with its own
code): W1 [256][7], b1 [256], W2 [256][256], b2 [256], W3, b3, W4, b4 (as W2, b2),
W5 [1][256], b5 [1]; row-major, output index first. 199,681 values in all.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

N_IN, WIDTH, DEPTH, N_OUT = 7, 256, 4, 1

_SHAPES: List[Tuple[str, Tuple[int, ...]]] = [
    ("W1", (WIDTH, N_IN)), ("b1", (WIDTH,)),
    ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
    ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)),
    ("W4", (WIDTH, WIDTH)), ("b4", (WIDTH,)),
    ("W5", (N_OUT, WIDTH)), ("b5", (N_OUT,)),
]
N_PARAMS = sum(int(np.prod(s)) for _, s in _SHAPES)


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    """Splits the flat parameter vector into named float64 arrays (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,), theta.shape
    out, o = {}, 0
    for name, shape in _SHAPES:
        cnt = int(np.prod(shape))
        out[name] = theta[o:o + cnt].reshape(shape)
        o += cnt
    return out


def pack(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in _SHAPES])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    """d silu / dz = s (1 + z (1 - s)), s = 1 / (1 + e^-z)."""
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def normalise(x: np.ndarray, shift: np.ndarray, scale: np.ndarray) -> np.ndarray:
    return (np.asarray(x, dtype=np.float64) - shift) * scale


def forward(theta: np.ndarray, xn: np.ndarray):
    """xn: [B, 7] normalised inputs. Returns y [B] and the pre-activations z1..z4."""
    p = unpack(theta)
    a = np.asarray(xn, dtype=np.float64)
    zs = []
    for l in range(1, DEPTH + 1):
        z = a @ p[f"W{l}"].T + p[f"b{l}"]
        zs.append(z)
        a = silu(z)
    y = a @ p["W5"].T + p["b5"]
    return y[:, 0], zs


def backward(theta: np.ndarray, xn: np.ndarray, zs, dy: np.ndarray) -> np.ndarray:
    """Gradient of sum_b dy_b y_b with respect to every parameter (chain rule, layer by
    layer from the output). Returns the flat gradient in the parameter layout."""
    p = unpack(theta)
    g = {}
    dy = np.asarray(dy, dtype=np.float64).reshape(-1, 1)
    a4 = silu(zs[3])
    g["W5"] = dy.T @ a4
    g["b5"] = dy.sum(axis=0)
    delta = (dy @ p["W5"]) * silu_grad(zs[3])          # dL/dz4
    for l in range(DEPTH, 0, -1):
        a_prev = silu(zs[l - 2]) if l >= 2 else np.asarray(xn, dtype=np.float64)
        g[f"W{l}"] = delta.T @ a_prev
        g[f"b{l}"] = delta.sum(axis=0)
        if l >= 2:
            delta = (delta @ p[f"W{l}"]) * silu_grad(zs[l - 2])
    return pack(g)


def mse_loss_and_grad(theta: np.ndarray, xn: np.ndarray, target: np.ndarray):
    """L = mean((y - t)^2) and dL/dtheta."""
    y, zs = forward(theta, xn)
    r = y - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / r.size
    return loss, backward(theta, xn, zs, dy)


def adam_step(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step t >= 1). Returns the new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Rounds float values to the nearest bfloat16 (ties to even), returned as float64: the
    value a BF16 operand actually carries."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
