"""Comparison helpers for GPU-vs-oracle parity (test side only).

Contract (floating point; FP32 kernel vs FP64 oracle on the same stored nodes):
  * local: every recorded GPU vertex equals one FP64 RK4 step of the oracle
    from the GPU's previous vertex, within  LOCAL_REL * extent + 4 ulp_f32(|P|);
    this pins the arithmetic of every step regardless of chaos;
  * global: on non-chaotic cases every vertex is within GLOBAL_REL * extent of
    the oracle's own trajectory (1e-4 for FP32 fields, 2e-3 for 16-bit);
  * discrete: step counts and termination codes are identical for every
    particle whose termination event is not boundary-sensitive.
The bound for the local check: one FP32 step rounds the position (<= 1 ulp),
evaluates the stage coordinates with <= 1 ulp(s) error (a relative 6e-8 of
the block edge) and the trilinear sums with ~1e-7 relative error; 1e-6 of the
extent covers these with a margin of > 10x at every configuration used.
"""
from __future__ import annotations

import numpy as np

LOCAL_REL = 1e-6


def ulp32(x):
    x = np.abs(np.asarray(x, np.float32))
    return np.spacing(x).astype(np.float64)


def split_lines(lines):
    off = lines["offsets"]
    return [lines["xyz"][off[i]:off[i + 1]].astype(np.float64) for i in range(len(off) - 1)]


def local_check(field, lines, h, extent, eps=1e-6, t_birth=None, stride=1):
    """Max violation ratio (<= 1 passes) of the per-step check over all consecutive vertex
    pairs that are one step apart (stride 1)."""
    assert stride == 1
    segs = split_lines(lines)
    p0, p1, t0 = [], [], []
    for i, s in enumerate(segs):
        if len(s) < 2:
            continue
        n = len(s) - 1
        # with stride 1 every step appends a vertex, except that a stagnant/halo/non-finite
        # stop appends nothing new; vertices j and j+1 are one step apart
        p0.append(s[:-1])
        p1.append(s[1:])
        tb = 0.0 if t_birth is None else float(np.asarray(t_birth).reshape(-1)[i] if np.ndim(t_birth) else t_birth)
        t0.append(tb + np.arange(n) * float(np.float32(h)))
    if not p0:
        return 0.0, 0
    p0 = np.concatenate(p0)
    p1 = np.concatenate(p1)
    tt = np.concatenate(t0)
    ref, st = field.step(p0, float(np.float32(h)), eps=0.0, t=tt)
    ok = st == 0
    err = np.abs(p1[ok] - ref[ok]).max(axis=1)
    tol = LOCAL_REL * extent + 4 * ulp32(p1[ok]).max(axis=1)
    return float((err / tol).max(initial=0.0)), int(ok.sum())


def global_compare(gpu_lines, orc, n_particles):
    """Per-particle max deviation over common vertices, plus vertex-count agreement."""
    segs = split_lines(gpu_lines)
    dev = np.zeros(n_particles)
    same_len = np.zeros(n_particles, bool)
    for i, s in enumerate(segs):
        nv = int(orc["n_verts"][i])
        k = min(len(s), nv, orc["verts"].shape[1])
        dev[i] = np.abs(s[:k] - orc["verts"][i, :k]).max(initial=0.0)
        same_len[i] = len(s) == nv
    return dev, same_len


def boundary_sensitive(orc, gpu_lines, dev, lo, hi, eps=1e-6, field=None):
    """Particles whose termination could legitimately differ between FP32 and FP64:
    the oracle's or the GPU's final position lies within 10*dev + 1e-5 of a face of the
    owned bounds, or |v| at the final position is within a factor 2 of eps."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    segs = split_lines(gpu_lines)
    gl = np.stack([s[-1] for s in segs])
    margin = 10 * dev[:, None] + 1e-5
    sens = np.zeros(len(segs), bool)
    for P in (orc["final_pos"], gl):
        d = np.minimum(np.abs(P - lo), np.abs(P - hi))
        sens |= np.any(d <= margin, axis=1)
    if field is not None:
        v, ok = field.sample(orc["final_pos"])
        speed = np.linalg.norm(v, axis=1)
        sens |= ok & (speed < 2 * eps) & (speed > eps / 2)
    return sens


def restart_check(field, lines, h, lo, hi, max_steps, stride=1, back=16, t_birth=None, eps=1e-6):
    """Discrete results from a late restart.  For each particle the oracle starts from the
    GPU's own recorded vertex at least `back` steps before the particle's last step (vertex j
    is step j*stride; the final vertex is the last step), at that vertex's time and with the
    steps its limit leaves, and must end with the same termination code at the same step count.
    Over so few steps the two sides differ by rounding only, so only terminations within
    10x that difference (plus 1e-5) of a face of the owned bounds, or with |v| within a factor
    2 of eps, are exempt -- unlike the whole-trajectory comparison, whose exemption margin grows
    with chaotic drift.  Returns (compared fraction, indices of mismatches)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    off = lines["offsets"]
    n = lines["steps"].astype(np.int64)
    k = len(n)
    nv = np.diff(off)
    m = np.broadcast_to(np.asarray(max_steps, np.int64), (k,))
    tb = np.zeros(k) if t_birth is None else np.broadcast_to(np.asarray(t_birth, np.float64), (k,))
    # restart vertex: the last recorded vertex at or before step n - back (never the final one
    # unless it is the only one)
    j = np.clip((n - back) // stride, 0, None)
    j = np.minimum(j, np.maximum(nv - 2, 0))
    start = lines["xyz"][off[:-1] + j].astype(np.float64)
    done = j * stride
    hf = float(np.float32(h))
    ref = field.trace(start, hf, (m - done).astype(np.int32), eps=eps, t_birth=tb + done * hf, keep_verts=False)
    final = lines["xyz"][off[1:] - 1].astype(np.float64)
    d = np.abs(final - ref["final_pos"]).max(axis=1)
    margin = 10 * d[:, None] + 1e-5
    sens = np.zeros(k, bool)
    for P in (ref["final_pos"], final):
        sens |= np.any(np.minimum(np.abs(P - lo), np.abs(P - hi)) <= margin, axis=1)
    v, ok = field.sample(ref["final_pos"])
    speed = np.linalg.norm(v, axis=1)
    sens |= ok & (speed < 2 * eps) & (speed > eps / 2)
    bad = ~sens & ((ref["steps"] + done != n) | (ref["code"] != lines["codes"]))
    return float((~sens).mean()), np.nonzero(bad)[0]
