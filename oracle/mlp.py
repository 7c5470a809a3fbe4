"""FP64 reference of the warm-start network (test infrastructure only).

A multilayer perceptron y = W_L g(... g(W_1 x + b_1) ...) + b_L with the tanh form of
GELU, g(z) = z/2 (1 + tanh(sqrt(2/pi)(z + 0.044715 z^3))), the weighted mean-square loss
L = sum_{r,c} w_c (y - t)^2 / (R C), its gradients by reverse-mode differentiation, and
one Adam step.  Parameters are one flat vector ordered W_0 (out x in, row-major), b_0,
W_1, b_1, ...

`bf16=True` rounds, as the GPU kernels do, every operand of a matrix product to bfloat16
(inputs, weights, hidden activations, and the back-propagated dZ) while everything else
stays in FP64; it isolates the kernels' arithmetic from BF16's own rounding.
"""
from __future__ import annotations

import math

import numpy as np

C_GELU = math.sqrt(2.0 / math.pi)


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (IEEE round to nearest, ties to even, of the binary32 value)."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = b.view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(C_GELU * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C_GELU * (1.0 + 3 * 0.044715 * z * z)


def unpack(params, widths):
    out, off = [], 0
    for l in range(len(widths) - 1):
        n, k = widths[l + 1], widths[l]
        W = params[off: off + n * k].reshape(n, k)
        off += n * k
        b = params[off: off + n]
        off += n
        out.append((W, b))
    assert off == params.size
    return out


def num_params(widths):
    return sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1))


def forward(params, widths, x, bf16=False):
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    layers = unpack(np.asarray(params, np.float64), widths)
    a = rnd(x)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = a @ rnd(W).T + b
        cache.append((a, z))
        a = z if l == len(layers) - 1 else rnd(gelu(z))
    return a, cache


def loss_and_grad(params, widths, x, target, weight=None, bf16=False):
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    y, cache = forward(params, widths, x, bf16)
    R, C = y.shape
    w = np.ones(C) if weight is None else np.asarray(weight, np.float64)
    d = y - target
    loss = float(np.sum(w * d * d) / (R * C))
    dA = 2.0 * w * d / (R * C)
    layers = unpack(np.asarray(params, np.float64), widths)
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a, z = cache[l]
        dZ = dA if l == len(layers) - 1 else dA * gelu_grad(z)
        dZr = rnd(dZ)
        gW = dZr.T @ a
        gb = dZ.sum(0)
        grads.append((gW, gb))
        dA = dZr @ rnd(W)
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
