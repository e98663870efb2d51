"""Seeded synthetic inputs evaluated with torch (on a GPU, or on the CPU for checking).

This module produces INPUTS only, like the rest of `fieldgen`: the random
Fourier-mode turbulence of `turbulence_values` (same modes, same phases, same
normalisation) and the streakline particle sets of `streakline_particles`, at
sizes where the host generator would take minutes (96 blocks x 16 time slices
x 512 modes is about 1.3e12 mode evaluations).  It holds no part of the
advection method.

The mode sum is separable: with phasors X[i,m] = exp(i (kappa_m u_m,x x_i + phi_m)),
Y[j,m] = exp(i kappa_m u_m,y y_j) and Z[k,m] = exp(i kappa_m u_m,z z_k),
    v_c(x_i, y_j, z_k) = sum_m a_m e_m,c Re(X[i,m] Y[j,m] Z[k,m]),
so each component of a block is one FP64 matrix product over the modes:
    V_c[(k,j), i] = [Re(YZ) a e_c | -Im(YZ) a e_c] . [Re X | Im X]^T.
Results agree with the host generator to FP64 rounding (summation order), and
the stored values are rounded to nearest even straight from FP64 to the storage
format (no intermediate rounding), as `quantize` does.
"""
from __future__ import annotations

import numpy as np

from . import (BF16, BOUNDARY_BLOCK, F16, F32, P_BLOCKSHAPE, P_MAXSTEPS, P_MODES, P_NSEEDS, Block, _load, _ptr,
               int_uniform, stream, uniform, uniform_seeds)

# (stored fraction bits, smallest normal exponent) of the 16-bit storage formats
_FORMAT = {F16: (10, -14), BF16: (7, -126)}


def rne_torch(d, fmt):
    """Round FP64 tensor d to nearest even in fmt.  F32: a float32 tensor; F16/BF16: the
    16-bit patterns as an int16 tensor.  Finite inputs within the format's range only."""
    import torch
    assert d.dtype == torch.float64
    if fmt == F32:
        return d.to(torch.float32)  # one correctly rounded conversion
    mant, emin = _FORMAT[fmt]
    _, e = torch.frexp(d)  # |d| = m 2^e, m in [0.5, 1): the leading bit has weight 2^(e-1)
    ex = torch.clamp(e.to(torch.int32) - 1, min=emin)
    ulp = torch.ldexp(torch.ones_like(d), (ex - mant).to(torch.float64))
    q = torch.round(d / ulp) * ulp  # torch.round is half-to-even; both operations are exact
    if fmt == F16:
        return q.to(torch.float32).to(torch.float16).view(torch.int16)  # q is exact in both
    return q.to(torch.float32).to(torch.bfloat16).view(torch.int16)


def turbulence_stored(config, dims, sub=0, n_modes=512, kmin=1.0, kmax=32.0, n_slices=1, fmt=F16,
                      device="cuda", want_values=False):
    """The field of `turbulence_values(config, dims, sub, n_modes, kmin, kmax, n_slices)`
    stored in `fmt`: a tensor [S][nz+2][ny+2][nx+2][3] on `device` (float32, or int16 bit
    patterns for FP16/BF16).  With want_values, also the FP64 values (same shape)."""
    import torch
    nx, ny, nz = (int(v) for v in dims)
    L = float(max(dims))
    M = int(n_modes)
    kappa, amp, phi, drift = (np.empty(M) for _ in range(4))
    u, e = np.empty(3 * M), np.empty(3 * M)
    _load().fg_turb_modes(stream(config, P_MODES, sub), M, kmin, kmax, L, _ptr(kappa), _ptr(u), _ptr(e),
                          _ptr(amp), _ptr(phi), _ptr(drift))
    f64 = dict(dtype=torch.float64, device=device)
    kap = torch.as_tensor(kappa, **f64)
    U = torch.as_tensor(u.reshape(M, 3), **f64)
    AE = torch.as_tensor(amp[:, None] * e.reshape(M, 3), **f64)  # a_m e_m  [M, 3]
    xs = torch.arange(nx + 2, **f64) - 0.5  # stored node coordinates (cell units), ghost at -0.5
    ys = torch.arange(ny + 2, **f64) - 0.5
    zs = torch.arange(nz + 2, **f64) - 0.5
    ay = ys[:, None] * (kap * U[:, 1])[None, :]
    az = zs[:, None] * (kap * U[:, 2])[None, :]
    yr, yi = torch.cos(ay), torch.sin(ay)
    zr, zi = torch.cos(az), torch.sin(az)
    # YZ[(k,j), m] = Y[j,m] Z[k,m]
    qr = (zr[:, None, :] * yr[None, :, :] - zi[:, None, :] * yi[None, :, :]).reshape(-1, M)
    qi = (zr[:, None, :] * yi[None, :, :] + zi[:, None, :] * yr[None, :, :]).reshape(-1, M)
    vals = torch.empty((n_slices, nz + 2, ny + 2, nx + 2, 3), **f64)
    vmax = torch.zeros((), **f64)
    for s in range(n_slices):
        ph = torch.as_tensor(phi + (2 * np.pi * drift * s / (n_slices - 1) if n_slices > 1 else 0.0), **f64)
        ax = xs[:, None] * (kap * U[:, 0])[None, :] + ph[None, :]
        B = torch.cat([torch.cos(ax), torch.sin(ax)], dim=1)  # [nx+2, 2M]
        for c in range(3):
            A = torch.cat([qr * AE[:, c], -qi * AE[:, c]], dim=1)  # [(nz+2)(ny+2), 2M]
            vals[s, ..., c] = (A @ B.T).reshape(nz + 2, ny + 2, nx + 2)
        vmax = torch.maximum(vmax, torch.sqrt((vals[s] * vals[s]).sum(dim=-1).max()))
    vals /= vmax
    stored = rne_torch(vals, fmt)
    return (stored, vals) if want_values else stored


def block_meta(dims, n_slices=1, slice_dt=1.0, fmt=F16):
    """Description of one batched turbulence block (cell units, its own owned box, no
    neighbours), without node values."""
    dims = tuple(int(v) for v in dims)
    return Block(dims=dims, ghost=1, origin=(0.5, 0.5, 0.5), spacing=(1.0, 1.0, 1.0), lo=(0.0, 0.0, 0.0),
                 hi=tuple(float(v) for v in dims), boundary=BOUNDARY_BLOCK, rank_grid=(1, 1, 1),
                 rank_coord=(0, 0, 0), n_slices=n_slices, t0=0.0, slice_dt=slice_dt, fmt=fmt)


def batched_blocks(config=4, n_blocks=96, edge_lo=32, edge_hi=192, fmt=F16, n_slices=1, n_modes=512, h=0.5,
                   m_lo=100, m_hi=5000, seeds_lo=1024, seeds_hi=65536, device="cuda", log=None):
    """The blocks, seeds and step limits of `fieldgen.batched_blocks` with the same arguments,
    the node values generated on `device`: (block descriptions, stored node tensors, seeds
    per block [host float32], step limits per block [host int32])."""
    edges = int_uniform(config, P_BLOCKSHAPE, n_blocks * 3, edge_lo, edge_hi).reshape(n_blocks, 3)
    counts = np.round(np.exp(np.log(seeds_lo) + uniform(stream(config, P_NSEEDS), n_blocks)
                             * (np.log(seeds_hi) - np.log(seeds_lo)))).astype(np.int64)
    counts = np.maximum(counts, 1)
    slice_dt = m_hi * h / (n_slices - 1) if n_slices > 1 else 1.0
    blocks, nodes, seeds, limits = [], [], [], []
    for b in range(n_blocks):
        dims = tuple(int(v) for v in edges[b])
        blocks.append(block_meta(dims, n_slices, slice_dt, fmt))
        nodes.append(turbulence_stored(config, dims, sub=b, n_modes=n_modes, n_slices=n_slices, fmt=fmt,
                                       device=device))
        seeds.append(uniform_seeds(config, int(counts[b]), (0, 0, 0), dims, sub=10 + b))
        limits.append(int_uniform(config, P_MAXSTEPS, int(counts[b]), m_lo, m_hi, sub=b).astype(np.int32))
        if log and (b + 1) % 16 == 0:
            log(f"generated {b + 1} of {n_blocks} blocks")
    return blocks, nodes, seeds, limits


def streakline_particles(emitters, limits, every, h):
    """`fieldgen.streakline_particles` for torch tensors (emitters [E,3] float32, limits [E]
    int32, on any device): emitter e releases a particle at steps 0, every, 2 every, ...
    < limits[e]; the particle born at step b starts at time b*h with step limit
    limits[e] - b.  Emitter-major, birth-minor: (positions, birth times, limits, emitter)."""
    import torch
    lim = limits.to(torch.int64)
    counts = (lim + every - 1) // every
    E = emitters.shape[0]
    emi = torch.repeat_interleave(torch.arange(E, device=emitters.device), counts)
    first = torch.cumsum(counts, 0) - counts
    bsteps = (torch.arange(emi.shape[0], device=emitters.device) - first[emi]) * every
    pos = emitters[emi].contiguous()
    tb = (bsteps.to(torch.float64) * h).to(torch.float32)
    lp = (lim[emi] - bsteps).to(torch.int32)
    return pos, tb, lp, emi
