"""Reference of the learned closure network: TEST INFRASTRUCTURE ONLY.

A multilayer perceptron 45 -> 128 -> 128 -> 128 -> 4 with GELU (erf form)
between layers, mean-squared-error loss, and Adam.  The paper leaves the
stress term of the momentum equation unclosed in coarse variables (Sec. 2.3)
and closes it through the fine-scale DEM; this network is the learned closure
of the benchmark configuration, trained on the method's own DEM output.

Everything is numpy FP64.  With ``bf16_mode=True`` the operands of every
matrix product (weights, network input, hidden activations and the
back-propagated errors) are rounded to bfloat16 (nearest, ties to even), as
the configuration stores them, while all arithmetic stays FP64: the parity
reference for the MFMA kernels.  ``bf16_mode=False`` is plain FP64 (used by
the finite-difference pins).

Parameter layout (one flat FP32/FP64 vector, 39,428 entries):
W1 [128 x 45], b1 [128], W2 [128 x 128], b2 [128], W3 [128 x 128], b3 [128],
W4 [4 x 128], b4 [4]; W_l[o, i] multiplies input i into output o.
"""
from __future__ import annotations

import math

import numpy as np

SIZES = [45, 128, 128, 128, 4]
SHAPES = []
for _i in range(4):
    SHAPES.append(("W%d" % (_i + 1), (SIZES[_i + 1], SIZES[_i])))
    SHAPES.append(("b%d" % (_i + 1), (SIZES[_i + 1],)))
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out = {}
    o = 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], np.float64).reshape(shp)
        o += k
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[n], np.float64).reshape(-1) for n, _ in SHAPES])


def bf16(x):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, x, bf16_mode=False, keep=False):
    """y = W4 g(W3 g(W2 g(W1 x + b1) + b2) + b3) + b4, rows of x are samples."""
    p = unpack(theta)
    r = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    a = r(x)
    acts, zs = [a], []
    for l in range(1, 5):
        z = a @ r(p["W%d" % l]).T + p["b%d" % l]
        zs.append(z)
        if l < 4:
            a = r(gelu(z))
            acts.append(a)
        else:
            a = z
    return (a, acts, zs) if keep else a


def loss(theta, x, t, bf16_mode=False):
    y = forward(theta, x, bf16_mode)
    return float(np.mean((y - t) ** 2))


def grad(theta, x, t, bf16_mode=False):
    """Gradient of the mean squared error over all samples and outputs."""
    p = unpack(theta)
    r = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    y, acts, zs = forward(theta, x, bf16_mode, keep=True)
    B = x.shape[0]
    d = 2.0 * (y - t) / (B * y.shape[1])
    g = {}
    for l in range(4, 0, -1):
        dr = r(d)               # operand of the products (bfloat16 in that mode)
        g["W%d" % l] = dr.T @ acts[l - 1]
        g["b%d" % l] = d.sum(axis=0)
        if l > 1:
            da = dr @ r(p["W%d" % l])
            d = da * gelu_grad(zs[l - 2])
    return pack(g)


def adam(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), bias-corrected; step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
