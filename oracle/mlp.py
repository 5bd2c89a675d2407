"""FP64 reference of the solve surrogate's network (test infrastructure only).

Plain numpy, one layer at a time: z = W a + b, a' = SiLU(z) = z / (1 + e^-z)
for the four hidden layers, a linear output layer; the loss of the C header
(masked squared error of 8 regression outputs plus the binary cross-entropy of
2 existence and 2 several-roots logits, averaged over the batch);
backpropagation written out by the chain rule; Adam (Kingma & Ba 2015) with
bias correction.

The GPU computes its matrix products from BF16-rounded weights and inputs;
``forward``/``gradients`` take ``bf16=True`` to evaluate the network at those
rounded values (everything else stays FP64), so that a comparison isolates
the GPU's own rounding (BF16 activations, FP32 accumulation).
Only the tests, the smoke check and the benchmark's CPU baseline use it.
"""
from __future__ import annotations

import numpy as np

N_IN, WIDTH, HIDDEN, N_OUT, N_TGT, N_LAB = 5, 256, 4, 12, 8, 4
DIMS = [(N_IN, WIDTH)] + [(WIDTH, WIDTH)] * (HIDDEN - 1) + [(WIDTH, N_OUT)]


def layout():
    """[(offset of W, offset of b, n_in, n_out)] and the total size."""
    out, off = [], 0
    for n_in, n_out in DIMS:
        out.append((off, off + n_in * n_out, n_in, n_out))
        off += n_in * n_out + n_out
    return out, off


def param_count() -> int:
    return layout()[1]


def unpack(params):
    lay, _ = layout()
    return [(params[w:w + ni * no].reshape(no, ni), params[b:b + no]) for w, b, ni, no in lay]


def round_bf16(x):
    """Round FP32 values to BF16 (round to nearest, ties to even), as FP64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, bf16=True, act_bf16=False):
    """Outputs [B][12] and the cache for backpropagation.  act_bf16 rounds
    the hidden activations to BF16 as the GPU stores them between layers."""
    layers = unpack(np.asarray(params, dtype=np.float64) if not bf16 else
                    np.asarray(params, dtype=np.float32))
    a = np.asarray(x, dtype=np.float64)
    if bf16:
        a = round_bf16(a)
    cache = []
    for l, (W, b) in enumerate(layers):
        Wd = round_bf16(W) if bf16 else W.astype(np.float64)
        z = a @ Wd.T + b.astype(np.float64)
        cache.append((a, z, Wd))
        a = silu(z) if l < len(layers) - 1 else z
        if act_bf16 and l < len(layers) - 1:
            a = round_bf16(a)
    return a, cache


def loss(y, t, m):
    """Loss of the C header for outputs y [B][12], targets t [B][8] and
    labels m [B][4] (existence of families 0, 1; several roots in 0, 1)."""
    B = y.shape[0]
    L = 0.0
    for f in range(2):
        e = y[:, 4 * f:4 * f + 4] - t[:, 4 * f:4 * f + 4]
        L += np.sum(m[:, f:f + 1] * e * e)
        z = y[:, 8 + f]
        L += np.sum(np.logaddexp(0.0, z) - m[:, f] * z)
        z = y[:, 10 + f]
        L += np.sum(np.logaddexp(0.0, z) - m[:, 2 + f] * z)
    return L / B


def loss_grad_y(y, t, m):
    B = y.shape[0]
    d = np.zeros_like(y)
    for f in range(2):
        e = y[:, 4 * f:4 * f + 4] - t[:, 4 * f:4 * f + 4]
        d[:, 4 * f:4 * f + 4] = 2.0 * m[:, f:f + 1] * e / B
        d[:, 8 + f] = (1.0 / (1.0 + np.exp(-y[:, 8 + f])) - m[:, f]) / B
        d[:, 10 + f] = (1.0 / (1.0 + np.exp(-y[:, 10 + f])) - m[:, 2 + f]) / B
    return d


def gradients(params, x, t, m, bf16=True, emulate=False):
    """(loss, dL/dparams as a flat FP64 array in the parameter layout).
    emulate rounds what the GPU stores in BF16 -- hidden activations and the
    gradients w.r.t. every layer's pre-activation -- at the same points."""
    t = np.asarray(t, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    y, cache = forward(params, x, bf16=bf16, act_bf16=emulate)
    lay, total = layout()
    g = np.zeros(total)
    d = loss_grad_y(y, t, m)  # dL/dz of the output layer
    for l in range(len(cache) - 1, -1, -1):
        a, z, Wd = cache[l]
        if l < len(cache) - 1:
            d = d * silu_grad(z)
        if emulate:
            d = round_bf16(d)
        w_off, b_off, ni, no = lay[l]
        g[w_off:w_off + ni * no] = (d.T @ a).ravel()
        g[b_off:b_off + no] = d.sum(axis=0)
        d = d @ Wd  # dL/da of the layer below
    return loss(y, t, m), g


def adam(params, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v

