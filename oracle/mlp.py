"""FP64 oracle of the learned flow-map surrogate -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the bench's CPU-baseline leg may import it.

The network maps a position to a 16-step displacement:
    xhat    = 2 * (x mod L) / L - 1                  (L = period of the block, per axis)
    h_0     = xhat                                   [3]
    z_l     = W_l h_l + b_l,  h_{l+1} = SiLU(z_l)    l = 0..3, widths 3 -> 256 -> 256 -> 256 -> 256
    out     = sigma * (W_4 h_4 + b_4)                [3]
    SiLU(z) = z * s(z),  s = logistic,  SiLU'(z) = s(z) (1 + z (1 - s(z)))
Loss on a batch: mean over samples and components of ((out - target) / sigma)^2.
Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps).

None of this is in the paper (the surrogate is one of the three forms the
project adds to the method); it is written from the definitions above, with
numpy matrix products as the only library primitive.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (3, 256, 256, 256, 256, 3)


def n_params(widths=WIDTHS) -> int:
    return sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1))


def normalise(x, period):
    x = np.asarray(x, np.float64)
    return 2.0 * (np.mod(x, period) / period) - 1.0


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, xhat, sigma, round_act=None):
    """params: list of (W [out, in], b [out]); xhat [B, 3]. Returns out [B, 3] and the
    per-layer inputs/pre-activations for backprop.

    round_act: None (plain FP64), or a rounding applied to every hidden activation
    h_{l+1} = SiLU(z_l) before the next layer uses it -- the precision in which the
    matrix cores take their operands (BF16), so that a decision taken on the output
    is taken in the same precision on both sides."""
    h = np.asarray(xhat, np.float64)
    hs, zs = [h], []
    for l, (W, b) in enumerate(params):
        z = h @ W.T + b
        zs.append(z)
        if l < len(params) - 1:
            h = silu(z)
            if round_act is not None:
                h = round_act(h)
            hs.append(h)
    out = zs[-1] * sigma
    return out, (hs, zs)


def loss(out, target, sigma):
    d = (out - target) / sigma
    return float(np.mean(d * d))


def backward(params, cache, out, target, sigma, round_grad=None):
    """Gradients of loss() with respect to every W_l and b_l.

    round_grad: None (plain FP64), or a rounding applied to every dL/dz_l before it
    enters a product (the precision of the matrix-core operands)."""
    hs, zs = cache
    B = out.shape[0]
    rg = (lambda a: a) if round_grad is None else round_grad
    # dL/dout = 2 (out - target) / sigma^2 / (B*3); out = sigma * z_last
    dz = rg(2.0 * (out - target) / (sigma * sigma) / (B * out.shape[1]) * sigma)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = (dz.T @ hs[l], dz.sum(axis=0))
        if l > 0:
            dh = dz @ W
            dz = rg(dh * dsilu(zs[l - 1]))
    return grads


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; t is the 1-based step count."""
    for l in range(len(params)):
        for k in range(2):
            g = grads[l][k]
            m[l][k] = b1 * m[l][k] + (1 - b1) * g
            v[l][k] = b2 * v[l][k] + (1 - b2) * g * g
            mhat = m[l][k] / (1 - b1 ** t)
            vhat = v[l][k] / (1 - b2 ** t)
            p = params[l][k] - lr * mhat / (np.sqrt(vhat) + eps)
            params[l] = (p, params[l][1]) if k == 0 else (params[l][0], p)


def zeros_like(params):
    return [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]


def round_bf16(a):
    """Round FP64 values to BF16 (round to nearest even), returned as FP64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
