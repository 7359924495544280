"""FP64 numpy reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

Same architecture, input normalisation, targets and loss as the GPU kernels
declared in include/kerrhip_mlp.h, written plainly: a loop over five dense
layers, SiLU on the hidden ones, and reverse-mode differentiation by hand.
Only tests and the benchmark's CPU leg may import it.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(4, 256), (256, 256), (256, 256), (256, 256), (256, 4)]  # (in, out)
NPARAMS = sum(i * o + o for i, o in LAYERS)


def unpack(params):
    """[(W [out][in], b [out])] views of the flat parameter vector."""
    out, off = [], 0
    for nin, nout in LAYERS:
        W = params[off:off + nin * nout].reshape(nout, nin)
        off += nin * nout
        b = params[off:off + nout]
        off += nout
        out.append((W, b))
    return out


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    parts = []
    for nin, nout in LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / nin), (nout, nin)).ravel())
        parts.append(np.zeros(nout))
    return np.concatenate(parts)


def features(x):
    """x [n][4] = (alpha, beta, a, incl_radians) -> normalised inputs."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([x[:, 0] / 12.0, x[:, 1] / 12.0, (x[:, 2] - 0.5) * 2.0,
                     (np.degrees(x[:, 3]) - 45.0) / 40.0], axis=1)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, x, bf16_storage=False):
    """Network outputs.  bf16_storage=True rounds the weights and every hidden
    activation to BF16 and the inputs to a sum of two BF16 numbers (the storage
    format of the GPU's matrix products), keeping FP64 arithmetic otherwise."""
    h = features(x)
    layers = unpack(params)
    if bf16_storage:
        # the inputs enter as two BF16 terms each (leading term and the
        # rounded remainder), the other activations as one
        hi = round_bf16(h)
        h = hi + round_bf16(h - hi)
        layers = [(round_bf16(W), b) for W, b in layers]
    cache = [h]
    zs = []
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if l < len(layers) - 1:
            zs.append(z)
            h = z * sigmoid(z)
            if bf16_storage:
                h = round_bf16(h)
            cache.append(h)
        else:
            h = z
    return h, (cache, zs)


def loss_and_grad(params, x, t, mask, bf16_storage=False, weights=(1.0, 1.0, 1.0, 1.0)):
    """Mean over the batch of mask0 (w0 (y0-t0)^2 + w1 (y1-t1)^2) + mask1 w2 (y2-t2)^2 +
    w3 BCE(sigmoid(y3), t3), and its gradient (flat, like params).  With
    bf16_storage the forward pass stores weights and activations as BF16."""
    y, (hs, zs) = forward(params, x, bf16_storage)
    if bf16_storage:
        params = np.concatenate([np.concatenate([round_bf16(W).ravel(), b]) for W, b in unpack(params)])
    n = len(y)
    m0 = (np.asarray(mask) & 1).astype(np.float64)
    m1 = ((np.asarray(mask) >> 1) & 1).astype(np.float64)
    e0, e1, e2 = (y[:, 0] - t[:, 0]) * m0, (y[:, 1] - t[:, 1]) * m0, (y[:, 2] - t[:, 2]) * m1
    y3, t3 = y[:, 3], t[:, 3]
    bce = np.maximum(y3, 0) - y3 * t3 + np.log1p(np.exp(-np.abs(y3)))
    w0, w1, w2, w3 = (float(v) for v in weights)
    loss = np.mean(w0 * e0 ** 2 + w1 * e1 ** 2 + w2 * e2 ** 2 + w3 * bce)
    dy = np.stack([2 * w0 * e0, 2 * w1 * e1, 2 * w2 * e2, w3 * (sigmoid(y3) - t3)], axis=1) / n
    layers = unpack(params)
    grads = [None] * len(layers)
    d = dy
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (d.T @ hs[l], d.sum(axis=0))
        if l > 0:
            dh = d @ W
            z = zs[l - 1]
            s = sigmoid(z)
            d = dh * s * (1 + z * (1 - s))
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return loss, flat


def round_bf16(a):
    """Round FP32/FP64 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
