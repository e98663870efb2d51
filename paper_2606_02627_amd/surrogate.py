"""Training and use of the learned flow-map surrogate (16-step displacement).

Everything numerical runs in the library: training windows come from the
GPU RK4 integrator (streami_advect over 16 steps), and each training step is
one streami_mlp_train_step (BF16 MFMA forward/backward, Adam).  This module
only sequences those calls.
"""
from __future__ import annotations

import math
import time


from . import (F32, Field, streami_advect, advect_params, streami_fetch_lines, streami_mlp_create,
               streami_mlp_train_step, streami_mlp_forward)

JUMP = 16


def flow_map_windows(block, starts, h, jump=JUMP, stream=None):
    """Start points and their `jump`-step displacements from the GPU integrator.

    Returns device tensors (x0 [n, 3], d [n, 3]) of FP32.  The lines are fetched
    straight into device memory (vertex 0 = start, vertex 1 = after `jump` steps).
    """
    import torch
    f = Field([block], block.fmt)
    d_starts = torch.as_tensor(starts, dtype=torch.float32, device="cuda").contiguous()
    n = d_starts.shape[0]
    f.seed(0, d_starts, default_max_steps=jump, record_stride=jump)
    f.advect(h)
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    xyz = torch.empty((2 * n, 3), dtype=torch.float32, device="cuda")
    _, need = streami_fetch_lines(f.h, 0, 0, n, off, xyz, 2 * n)
    f.close()
    if need != 2 * n or not bool(torch.all(off[1:] - off[:-1] == 2)):
        raise RuntimeError(f"a training window ended before {jump} steps")
    v = xyz.view(n, 2, 3)
    return v[:, 0].contiguous(), (v[:, 1] - v[:, 0]).contiguous()


def train(x0, d, init_params, period, epochs=8, batch=8192, lr=2e-3, log=None, seed=0):
    """Train a new network on (x0, d); returns (network handle, sigma, history).

    sigma = per-component standard deviation of the targets (output scale);
    Adam with a cosine learning-rate decay from lr to 0 over all steps; the
    windows are visited in a new random order (seeded) every epoch.
    """
    import torch
    sigma = d.to(torch.float64).std(dim=0, unbiased=False).cpu().numpy()
    gen = torch.Generator(device=x0.device)
    gen.manual_seed(seed)
    net = streami_mlp_create(init_params, sigma, period)
    n = x0.shape[0]
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    hist = []
    t0 = time.perf_counter()
    k = 0
    for e in range(epochs):
        perm = torch.randperm(n, device=x0.device, generator=gen)
        xs, ds = x0[perm], d[perm]
        for s in range(steps_per_epoch):
            lr_k = 0.5 * lr * (1.0 + math.cos(math.pi * k / total))
            sl = slice(s * batch, (s + 1) * batch)
            want = s == steps_per_epoch - 1
            loss, _ = streami_mlp_train_step(net, xs[sl], ds[sl], lr_k, want_loss=want)
            k += 1
        hist.append(dict(epoch=e, loss=loss, seconds=time.perf_counter() - t0))
        if log:
            log(f"epoch {e}: loss {loss:.3e} ({time.perf_counter() - t0:.1f}s)")
    torch.cuda.synchronize()
    return net, sigma, hist


def predict(net, x):
    """Network displacement for device positions x [n, 3] (FP32)."""
    import torch
    out = torch.zeros_like(x)
    streami_mlp_forward(net, x, out)
    return out
