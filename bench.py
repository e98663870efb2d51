#!/usr/bin/env python3
"""Throughput benchmark of the RK4 field-line advection path on one MI355X.

One step = one pass of the hot path over one batch of synthetic input, with
the field and the seed set already resident in HBM: clear the handle, seed
every particle (device-to-device), advect every particle to termination
(trilinear gathers, RK4, exit/stagnation tests, vertex and outbox appends).
Field ingest and line fetch are one-time costs, reported separately.

Default workload: one rank's block of synthetic turbulence, 256^3 interior
nodes + 1 ghost layer, FP32 vec3, 1M uniform seeds, h = 0.5 cell, at most 2000
steps, exits to the outbox (rank grid 4^3, block at (1,1,1)).

Prints ONE JSON line (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
LAYOUT_NAMES = {1: "linear", 2: "brick4", 3: "cell", 5: "brick8"}
CLOCK_GHZ = 2.4  # MI355X peak engine clock
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak, published
# one network evaluation: 2 * (3*256 + 3*256*256 + 256*3) multiply-adds
MLP_FLOPS_PER_EVAL = 2 * (3 * 256 + 3 * 256 * 256 + 256 * 3)
MLP_SILU_PER_EVAL = 4 * 256  # a SiLU after each of the four 256-wide layers


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


WORKLOADS = {
    # name: (edge, dtype, n_seeds, max_steps, h, seed kind, record stride)
    "turb256-f32": (256, "f32", 1 << 20, 2000, 0.5, "uniform", 1),
    "turb512-bf16": (512, "bf16", 1 << 22, 4000, 0.5, "blobs", 8),
    "turb512-f16": (512, "f16", 1 << 22, 4000, 0.5, "blobs", 8),
    "turb512-f32": (512, "f32", 1 << 22, 4000, 0.5, "blobs", 8),
    "abc32-f32": (32, "f32", 1024, 200, 0.01, "abc", 1),
}


def code_text(src: str) -> str:
    """Source text without comments and whitespace: what the compiler sees of it."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return re.sub(r"\s+", "", src)


def kernel_source_hash() -> str:
    """Hash of the advection kernel's code (comments and whitespace ignored): a traffic
    measurement stays attached to the kernel it was taken on."""
    h = hashlib.sha1()
    for f in ("advect_impl.h", "device.h"):
        with open(os.path.join(ROOT, "paper_2606_02627_amd", "csrc", f)) as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:12]


def build_inputs(name):
    import fieldgen as fg
    edge, dt, n, m, h, kind, stride = WORKLOADS[name]
    fmt = {"f32": fg.F32, "f16": fg.F16, "bf16": fg.BF16}[dt]
    if kind == "abc":
        blk = fg.abc_block(edge, fmt)
        seeds = fg.uniform_seeds(1, n, (0, 0, 0), (2 * np.pi,) * 3)
    else:
        cfg = 2 if edge == 256 else 3
        blk = fg.turbulence_block(cfg, edge=edge, fmt=fmt)
        if kind == "uniform":
            seeds = fg.uniform_seeds(cfg, n, (0, 0, 0), (edge,) * 3)
        else:
            seeds = fg.blob_seeds(cfg, 64, n // 64, float(edge), 24.0, 8.0)
    return blk, seeds, fmt, m, h, stride


def host_cores():
    """(cores this process may run on, host's logical cores, the cgroup CPU quota or None):
    the CPU affinity mask, capped by a cgroup v2 `cpu.max` quota when one is set."""
    host = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = host
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, per = fh.read().split()[:2]
        if q != "max":
            quota = float(q) / float(per)
            avail = max(1, min(avail, int(quota)))
    except (OSError, ValueError):
        pass
    return avail, host, quota


def cpu_baseline(blk, seeds, h, m, budget_s=12.0):
    """The FP64 oracle as it stands, on a bounded sample of the same workload, with one
    thread per core this process may use."""
    import oracle
    F = oracle.Field.from_block(blk)
    threads, host, quota = host_cores()
    n = 256
    total_steps, total_t = 0, 0.0
    used = 0
    # grow the sample until ~budget_s of CPU wall time is spent
    while total_t < budget_s and used < len(seeds):
        k = min(n, len(seeds) - used)
        t0 = time.perf_counter()
        r = F.trace(seeds[used:used + k], h, m, threads=threads, keep_verts=False)
        total_t += time.perf_counter() - t0
        total_steps += int(r["steps"].sum())
        used += k
        n *= 2
    # one thread, on the first seeds only (about a second)
    k1 = min(len(seeds), 4096)
    t0 = time.perf_counter()
    r1 = F.trace(seeds[:k1], h, m, threads=1, keep_verts=False)
    one = int(r1["steps"].sum()) / (time.perf_counter() - t0)
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return dict(value=total_steps / total_t, unit="particle-steps/s", cores=threads, kind="oracle",
                host_logical_cores=host, cgroup_cpu_quota=quota,
                sample=f"first {used} of the {len(seeds)} seeds, full trajectories "
                       f"(<= {m} steps each, {total_steps} steps) on the same stored field, FP64",
                seconds=round(total_t, 2), one_thread_value=one, one_thread_sample=f"first {k1} seeds",
                cpu_model=model)


PARTICLE_BYTES = 80  # per particle and launch: pos, meta, meta2 read (48 B); pos, meta written (32 B)
OUTBOX_BYTES = 40    # per outbox record: the 32-byte record written plus the 8-byte id read


def compulsory_bytes(gathers, refill_bytes, vertices, particles, outbox, vertex_bytes=12):
    """HBM bytes one advect launch cannot avoid with the register cell cache: every refill
    reads the cell's stored corners (or its record) once, every recorded vertex writes its
    x, y, z, and every particle's state is read and written once."""
    d = {"refills": gathers * refill_bytes, "vertices": vertices * vertex_bytes,
         "particles": particles * PARTICLE_BYTES, "outbox": outbox * OUTBOX_BYTES,
         "refill_bytes": refill_bytes}
    d["total"] = d["refills"] + d["vertices"] + d["particles"] + d["outbox"]
    return d


def surrogate_bench(args):
    """Learned flow-map form on the ABC field: train on GPU-generated 16-step windows, then
    advect seeds for 2000 steps with plain RK4, with the surrogate (both residual kinds) and
    with one RK4 step of 16h per jump (the surrogate's gather budget without the network).
    Plain RK4 is the yardstick: every run's endpoints are compared with the plain run's (its own
    error against the FP64 oracle is a test's business, not the benchmark's)."""
    import torch
    import fieldgen as fg
    import paper_2606_02627_amd as S
    from paper_2606_02627_amd import surrogate

    h, steps = 0.01, 2000
    n_train = int(os.environ.get("STREAMI_SURR_TRAIN", 1 << 23))
    n_inf = int(os.environ.get("STREAMI_SURR_SEEDS", 1 << 22))
    epochs = int(os.environ.get("STREAMI_SURR_EPOCHS", 12))
    blk = fg.abc_block(32)
    ext = 2 * np.pi
    log(f"training windows: {n_train}")
    t0 = time.perf_counter()
    x0, d = surrogate.flow_map_windows(blk, fg.training_starts(5, n_train, ext), h)
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, sigma, hist = surrogate.train(x0, d, fg.mlp_init(5), ext, epochs=epochs, batch=8192, lr=2e-3, log=log)
    t_train = time.perf_counter() - t0
    del x0, d
    seeds = fg.uniform_seeds(5, n_inf, (0, 0, 0), (ext,) * 3, sub=21)
    d_seeds = torch.from_numpy(seeds).cuda()
    sample = 4096
    ref = {}

    def run(label, hh, m, **kw):
        f = S.Field([blk], S.F32)
        best = None
        for _ in range(max(1, args.steps)):
            f.clear()
            f.seed(0, d_seeds, default_max_steps=m, record_stride=16 if m >= 16 else 1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = S.streami_advect(f.h, S.advect_params(hh, **kw))
            wall = time.perf_counter() - t
            best = wall if best is None else min(best, wall)
        L = f.lines(0, 0, sample)
        f.close()
        end = L["xyz"][L["offsets"][1:] - 1].astype(np.float64)
        ref.setdefault("plain", end)  # the first run is plain RK4
        err = np.abs(end - ref["plain"]).max(axis=1) / ext
        acc = st.surrogate_accepted / max(1, st.surrogate_accepted + st.surrogate_fallback)
        r = dict(label=label, seconds=best, equiv_steps_per_s=n_inf * steps / best, device_ms=st.device_ms,
                 acceptance=acc if kw.get("mode") == S.MODE_SURROGATE else None,
                 endpoint_dev_from_plain_over_extent=dict(
                     median=float(np.median(err)), p90=float(np.quantile(err, 0.9)), max=float(err.max()),
                     frac_within_2e_3=float((err <= 2e-3).mean())))
        log(json.dumps(r))
        return r

    res = [run("plain-rk4", h, steps),
           run("rk4-16h-per-jump", 16 * h, steps // 16),
           run("surrogate-kind1-bigstep-residual", h, steps, mode=S.MODE_SURROGATE, mlp=net,
               residual_tol_cells=1e-3, residual_kind=1),
           run("surrogate-kind0-commutation-residual", h, steps, mode=S.MODE_SURROGATE, mlp=net,
               residual_tol_cells=1e-3, residual_kind=0)]
    # the fused network kernel alone (k_mlp_infer), on the surrogate's input size
    outn = torch.empty_like(d_seeds)
    S.streami_mlp_forward(net, d_seeds, outn)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        S.streami_mlp_forward(net, d_seeds, outn)
    e1.record()
    torch.cuda.synchronize()
    mlp_ms = e0.elapsed_time(e1) / reps
    flops = n_inf * MLP_FLOPS_PER_EVAL
    roof = {"bound": "mfma", "achieved": flops / mlp_ms / 1e9, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": flops / mlp_ms / 1e9 / MFMA_BF16_PEAK_TFLOPS, "traffic": None, "kernel": "k_mlp_infer",
            "flops_per_eval": MLP_FLOPS_PER_EVAL, "evals_per_launch": n_inf, "mean_launch_ms": mlp_ms}
    log(f"k_mlp_infer: {mlp_ms:.3f} ms for {n_inf} evaluations, {roof['achieved']:.1f} TFLOP/s")
    # the SiLU epilogue's own floor: per hidden output one exp, one rcp, three VOP2 instructions
    # (multiply, add, multiply) and half a packed BF16 conversion (VOP3), at the issue costs the
    # VALU probe measures on this chip, spread over every SIMD
    n_simd = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    cyc = {}
    for kind, name in ((0, "fma_f32"), (1, "add_u32"), (2, "exp_f32"), (3, "rcp_f32")):
        ms, n = S.streami_probe_valu(kind, 32)
        cyc[name] = n_simd * CLOCK_GHZ * 1e9 * ms * 1e-3 / n
    per64 = cyc["exp_f32"] + cyc["rcp_f32"] + 3 * cyc["add_u32"] + 0.5 * cyc["fma_f32"]
    silu_per_eval = MLP_SILU_PER_EVAL
    valu_ms = n_inf * silu_per_eval / 64 * per64 / (n_simd * CLOCK_GHZ * 1e9) * 1e3
    roof["epilogue_valu"] = {"cycles_per_wave64_instruction": cyc, "cycles_per_64_outputs": per64,
                             "silu_outputs_per_eval": silu_per_eval, "floor_ms": valu_ms,
                             "floor_over_launch": valu_ms / mlp_ms}
    log(f"SiLU epilogue VALU floor {valu_ms:.3f} ms ({per64:.1f} cycles per 64 outputs)")
    S.streami_mlp_destroy(net)
    plain = res[0]
    best_sur = max(res[2:], key=lambda r: r["equiv_steps_per_s"])
    out = {
        "metric": "RK4 particle-steps/s + HBM GB/s; surrogate vs plain at fixed endpoint error",
        "value": best_sur["equiv_steps_per_s"], "unit": "equivalent particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 0, "ms_per_step": best_sur["seconds"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 MFMA (fp32 accumulate) + f32 RK4", "data": "synthetic",
        "config": {"workload": "surrogate-abc", "field": "ABC 32^3 periodic f32", "train_windows": n_train,
                   "epochs": epochs, "seeds": n_inf, "steps": steps, "h": h, "residual_tol_cells": 1e-3},
        "roofline": roof,
        "speedup_vs_plain": best_sur["equiv_steps_per_s"] / plain["equiv_steps_per_s"],
        "runs": res, "train_seconds": t_train, "data_seconds": t_data,
        "final_loss": hist[-1]["loss"] if hist else None, "sigma": [float(v) for v in sigma],
    }
    print(json.dumps(out), flush=True)


def batched_bench(args, unsteady=False):
    """96 uneven FP16 blocks with uneven seed sets and trajectory lengths in one persistent
    launch (hipGraph replay, autotuned launch shape); unsteady: 16 time slices of the
    512-mode generator with drifting phases, every seed a streakline emitter releasing a
    particle every 10 steps, in one launch or, with --window-steps, in global-time windows
    (bit-identical results)."""
    import torch
    import fieldgen as fg
    import paper_2606_02627_amd as S
    from paper_2606_02627_amd import autotune

    h = 0.5
    t0 = time.perf_counter()
    window = 0
    nodes = None
    emit_every = 10
    if unsteady:
        # the node values of 96 blocks x 16 slices x 512 modes are generated on the GPU
        from fieldgen import device as fgd
        blocks, nodes, emitters, elim = fgd.batched_blocks(n_blocks=96, fmt=fg.F16, n_slices=16, n_modes=512,
                                                           log=log)
        n_emitters = sum(len(e) for e in emitters)
        dseeds, dlim, dtb = [], [], []
        for e, m in zip(emitters, elim):
            pos, tb, lim, _ = fgd.streakline_particles(torch.from_numpy(e).cuda(), torch.from_numpy(m).cuda(),
                                                       emit_every, h)
            dseeds.append(pos), dlim.append(lim), dtb.append(tb)
        stride = 1 << 20  # a streakline is the emitters' particles' final positions: keep seed + last vertex
        window = args.window_steps
        t_last = max(float((tb.double() + lim.double() * h).max()) for tb, lim in zip(dtb, dlim))
        t_ends = [k * window * h for k in range(1, int(np.ceil(t_last / (window * h))) + 1)] if window else []
        cands = [dict(waves_per_cu=w, refill_threshold=1, work_order=o) for w in (16, 32) for o in (0, 1)]
    else:
        blocks, seeds, limits = fg.batched_blocks(n_blocks=96, fmt=fg.F16)
        n_emitters = 0
        dseeds = [torch.from_numpy(x).cuda() for x in seeds]
        dlim = [torch.from_numpy(x).cuda() for x in limits]
        dtb = None
        stride = 1
        t_ends = []
        cands = None
    n_part = sum(int(x.shape[0]) for x in dseeds)
    torch.cuda.synchronize()
    log(f"inputs: {len(blocks)} blocks, {n_part} particles, {len(t_ends)} time windows, "
        f"generated in {time.perf_counter() - t0:.1f}s")

    def one_pass(f, cfg, stats=False):
        """Seed every block, then advect everything: one launch, or one per time window.
        With stats: the last call's stats and the sums over the pass's advect calls of
        steps, vertices and device time."""
        f.clear()
        f.seed_batches([dict(block=b, xyz=dseeds[b], max_steps=dlim[b], t_births=dtb[b] if dtb else None)
                        for b in range(len(blocks))], record_stride=stride)
        tot = dict(steps=0, vertices=0, dev_ms=0.0, gathers=0)
        for te in (t_ends or [None]):
            kw = dict(use_graph=1) if te is None else dict(t_end=te)
            st = S.streami_advect(f.h, S.advect_params(h, **kw, **cfg), want_stats=stats)
            if stats:
                tot["steps"] += int(st.steps)
                tot["vertices"] += int(st.vertices)
                tot["gathers"] += int(st.gathers)
                tot["dev_ms"] += st.device_ms
        return st, tot

    sig = dict(seeds=[int(x.shape[0]) for x in dseeds], h=h, stride=stride, windows=len(t_ends), unsteady=unsteady,
               n_modes=512, emit_every=emit_every if unsteady else 0)
    tuned = autotune.load(blocks, fg.F16, sig)
    if tuned is None:
        tuned = autotune.tune(blocks, fg.F16, one_pass, sig, log=log, repeats=1 if unsteady else 2, nodes=nodes,
                              candidates=cands)
    cfg = {k: tuned[k] for k in ("waves_per_cu", "refill_threshold", "work_order")}
    f = S.Field(blocks, fg.F16, layout=tuned["layout"], nodes=nodes)
    st0, tot = one_pass(f, cfg, stats=True)
    assert st0.active == 0, "particles left after the last call"
    for _ in range(max(0, args.warmup - 1)):
        one_pass(f, cfg)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        one_pass(f, cfg)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / args.steps
    steps_per_pass = tot["steps"]
    dev_ms = tot["dev_ms"]
    outbox_per_pass = int(st0.outbox)
    f.close()  # the baseline below holds the same particles again
    # baseline: the same work as one launch per block (one unbounded launch each)
    fields = [S.Field([b], fg.F16, layout=tuned["layout"], nodes=None if nodes is None else [nodes[k]])
              for k, b in enumerate(blocks)]

    def per_block_pass():
        for k, fb in enumerate(fields):
            fb.clear()
            fb.seed(0, dseeds[k], max_steps=dlim[k], record_stride=stride, t_births=dtb[k] if dtb else None)
            S.streami_advect(fb.h, S.advect_params(h), want_stats=False)

    per_block_pass()
    torch.cuda.synchronize()
    t = time.perf_counter()
    per_block_pass()
    torch.cuda.synchronize()
    wall_pb = time.perf_counter() - t
    for fb in fields:
        fb.close()
    value = steps_per_pass / wall
    vals = 192 if unsteady else 96
    alg = steps_per_pass * vals * 2 + tot["vertices"] * 12
    # a refill of a time-sliced field reads the cell in both bracketing slices
    refill = (96 if tuned["layout"] == S.LAYOUT_CELL else 8 * 8) * (2 if unsteady else 1)
    comp = compulsory_bytes(tot["gathers"], refill, tot["vertices"], n_part, outbox_per_pass)
    achieved = comp["total"] / (dev_ms * 1e-3) / 1e9
    out = {
        "metric": "RK4 particle-steps/s + HBM GB/s; surrogate vs plain at fixed endpoint error",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16 storage, f32 math", "data": "synthetic",
        "config": {"workload": "batched96-f16" + ("-streaklines" if unsteady else ""), "blocks": len(blocks),
                   "particles": n_part, "emitters": n_emitters, "emit_every_steps": emit_every if unsteady else None,
                   "fourier_modes": 512, "particle_steps_per_step": steps_per_pass, "slices": 16 if unsteady else 1,
                   "window_steps": window, "time_windows": len(t_ends),
                   "tuned": {k: tuned[k] for k in ("layout", "waves_per_cu", "refill_threshold", "work_order")},
                   "graph": not t_ends},
        # the advect calls' device time (HIP events on the handle's stream around the
        # work-order kernels and k_advect), summed over the pass's windows
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_advect (batched)", "advect_ms_per_step": dev_ms,
                     "compulsory_bytes_per_launch": comp, "kernel_hash": kernel_source_hash(),
                     "reuse": {"alg_bytes_per_launch": alg, "alg_over_compulsory": alg / comp["total"]}},
        "one_block_per_launch_steps_per_s": steps_per_pass / wall_pb,
        "batching_speedup": wall_pb / wall,
        "terminated": list(st0.terminated),
    }
    print(json.dumps(out), flush=True)


def hex_bench(args):
    """The default workload's block converted to hexahedra (every cell of its stored grid, as
    the paper converts voxels for its unstructured field): 257^3 cells located through the
    BVH, the same 1M seeds and limits, each pass clear -> seed -> advect; the structured
    field's pass on the same seeds is timed alongside for the ratio."""
    import torch
    import fieldgen as fg
    import paper_2606_02627_amd as S
    blk, seeds, fmt, m, h, stride = build_inputs("turb256-f32")
    mesh = fg.hex_mesh_from_block(blk)
    t0 = time.perf_counter()
    f = S.Field.hex(mesh)
    build_s = time.perf_counter() - t0
    field_bytes = S.streami_field_info(f.h)[1]
    log(f"hex field: {len(mesh['cells'])} cells, BVH + records built and uploaded in {build_s:.1f}s, "
        f"{field_bytes / 1e9:.2f} GB")
    d_seeds = torch.from_numpy(seeds).cuda()
    stream = torch.cuda.current_stream()

    def passes(fld, k, stats=False):
        out, ms = None, []
        for _ in range(k):
            fld.clear()
            fld.seed(0, d_seeds, default_max_steps=m, record_stride=stride)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st = S.streami_advect(fld.h, S.advect_params(h), want_stats=stats)
            e1.record(stream)
            out = out or st
            ms.append((e0, e1))
        return out, ms

    st0, _ = passes(f, max(1, args.warmup), stats=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, ev = passes(f, args.steps)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / args.steps
    adv_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    f.close()
    g = S.Field([blk], fmt)
    stg, _ = passes(g, 1, stats=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, evg = passes(g, args.steps)
    torch.cuda.synchronize()
    wall_g = (time.perf_counter() - t) / args.steps
    g.close()
    steps = int(st0.steps)
    # a BVH walk ends by reading the found cell's 192-byte record; every sample re-reads the
    # lane's current record (from the caches); compulsory: each walk's record once
    comp = compulsory_bytes(int(st0.gathers), 192, int(st0.vertices), len(seeds), int(st0.outbox))
    achieved = comp["total"] / (adv_ms * 1e-3) / 1e9
    out = {
        "metric": "RK4 particle-steps/s + HBM GB/s; surrogate vs plain at fixed endpoint error",
        "value": steps / wall, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "hex256-f32", "field": "256^3 + ghost turbulence block, every cell a hexahedron",
                   "cells": int(len(mesh["cells"])), "vertices": int(len(mesh["vertices"])), "seeds": len(seeds),
                   "max_steps": m, "h": h, "particle_steps_per_step": steps, "field_bytes": field_bytes},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_advect (hexahedra)",
                     "mean_launch_ms": adv_ms, "compulsory_bytes_per_launch": comp,
                     "kernel_hash": kernel_source_hash(),
                     "reuse": {"alg_bytes_per_launch": steps * 4 * 192 + int(st0.vertices) * 12}},
        "bvh_walks_per_step": int(st0.gathers) / steps,
        "build_seconds": build_s,
        "structured_steps_per_s": int(stg.steps) / wall_g,
        "hex_over_structured": (steps / wall) / (int(stg.steps) / wall_g),
        "same_step_count_as_structured": steps == int(stg.steps),
    }
    print(json.dumps(out), flush=True)


def forward_bench(args):
    """The default workload's field split into a 2 x 2 x 2 rank grid of 128^3 blocks in one handle,
    the same 1M seeds (each seeded in the block that owns it) and limits, traced with loopback
    forwarding (streami_trace): every exit routed on the device into the neighbouring block,
    rounds until nothing is active.  Timed with an exchange every --exchange-steps steps (256, the
    fastest measured for this field); one pass each with run-to-exit rounds and with an exchange
    every 512 ... 1 steps (the last is the paper's one exchange per step) shows what the exchange
    granularity costs on one GPU.  Every granularity gives the same lines."""
    import torch
    import fieldgen as fg
    import paper_2606_02627_amd as S
    edge, m, h = 256, 2000, 0.5
    whole = fg.turbulence_block(2, edge=edge, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
    parts = fg.partition(whole, (2, 2, 2))
    seeds = fg.uniform_seeds(2, 1 << 20, (0, 0, 0), (edge,) * 3)
    owner = (np.floor(seeds / (edge // 2)).astype(int) * np.array([1, 2, 4])).sum(axis=1)
    f = S.Field(parts, S.F32)
    layout = S.streami_field_info(f.h)[0]
    batches = [dict(block=b, xyz=torch.from_numpy(np.ascontiguousarray(seeds[owner == b])).cuda(),
                    ids=torch.from_numpy(np.nonzero(owner == b)[0].astype(np.uint64)).cuda()) for b in range(8)]

    def one(budget, stats=False):
        f.clear()
        f.seed_batches(batches, default_max_steps=m)
        return S.streami_trace(f.h, S.advect_params(h, step_budget=budget), want_stats=stats)

    k = max(0, args.exchange_steps)
    r0, st0 = one(k, stats=True)
    assert st0.active == 0
    for _ in range(max(0, args.warmup - 1)):
        one(k)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        one(k)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / args.steps
    steps = int(st0.steps)
    gran = []
    for budget in (0, 512, 256, 128, 64, 8, 1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        rk, stk = one(budget, stats=True)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        assert int(stk.steps) == steps and stk.active == 0
        gran.append(dict(steps_per_exchange=budget or "run to exit", rounds=rk, seconds=sec, steps_per_s=steps / sec,
                         advect_device_ms=stk.device_ms))
        log(f"exchange every {budget} steps: {rk} rounds, {sec * 1e3:.1f} ms, {steps / sec:.3g} steps/s")
    f.close()
    comp = compulsory_bytes(int(st0.gathers), 96 if layout == S.LAYOUT_CELL else 96, int(st0.vertices), len(seeds),
                            int(st0.outbox))
    achieved = comp["total"] / (st0.device_ms * 1e-3) / 1e9
    out = {
        "metric": "RK4 particle-steps/s + HBM GB/s; surrogate vs plain at fixed endpoint error",
        "value": steps / wall, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "forward256-f32", "field": "256^3 turbulence split into 2x2x2 blocks of 128^3 + ghost",
                   "seeds": len(seeds), "max_steps": m, "h": h, "steps_per_exchange": k or "run to exit",
                   "rounds": r0, "particle_steps_per_step": steps,
                   "layout": LAYOUT_NAMES[layout]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_advect (8 blocks, forwarding)",
                     "advect_device_ms_per_step": st0.device_ms, "compulsory_bytes_per_launch": comp,
                     "kernel_hash": kernel_source_hash()},
        "exchange_granularity": gran,
    }
    print(json.dumps(out), flush=True)


def memory_probe(S, field_bytes, record_bytes):
    """Measured peaks of the memory levels for the kernel's access: a plain device copy (HBM
    stream rate) and random record reads (streami_probe_gather) over footprints that live in
    the L2 (384 KB), the Infinity Cache (192 MB), at the stored field's own size, and in HBM
    (8 GiB).  Each read rate is the best over waves per CU (8-64) and records in flight per
    lane (1-8)."""
    import torch
    dev = torch.device("cuda:0")
    big = max(8 << 30, field_bytes)
    buf = torch.empty(big, dtype=torch.uint8, device=dev)
    buf[: 1 << 30].fill_(7)
    out = {"copy_GBps": None, "record_bytes": record_bytes, "read_GBps": {}}
    a = buf[: 1 << 30]
    b = buf[1 << 30: 2 << 30]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    e0.record()
    for _ in range(4):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    out["copy_GBps"] = 4 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    for name, fb in (("384KB", 384 << 10), ("192MB", 192 << 20), ("field", field_bytes), ("8GiB", 8 << 30)):
        best = 0.0
        for wpc in (8, 16, 32, 64):
            for inf in (1, 2, 4, 8):
                ms, n = S.streami_probe_gather(buf[:fb], record_bytes, 64, inf, wpc)
                best = max(best, n * record_bytes / (ms * 1e-3) / 1e9)
        out["read_GBps"][name] = best
    del buf, a, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="turb256-f32",
                    choices=sorted(WORKLOADS) + ["surrogate-abc", "batched96-f16", "batched96-f16-streaklines",
                                                 "hex256-f32", "forward256-f32"])
    ap.add_argument("--window-steps", type=int, default=0,
                    help="streaklines: advance in global-time windows of this many steps (0: one launch)")
    ap.add_argument("--layout", type=int, default=0, help="0 auto, 1 linear, 2 brick4, 5 brick8, 3 cell records (FP32)")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--no-cell-cache", action="store_true")
    ap.add_argument("--lds-cell-cache", action="store_true",
                    help="keep each lane's cached cell record in LDS instead of registers (cell records)")
    ap.add_argument("--graph", action="store_true")
    ap.add_argument("--exchange-steps", type=int, default=256,
                    help="forward256: steps each block runs between two exchanges (0: until every local particle "
                         "has terminated or left)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (scale for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on exactly one GPU (the multi-GPU exchange of the outbox is "
              "designed but not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2606_02627_amd as S

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.workload == "surrogate-abc":
        return surrogate_bench(args)
    if args.workload.startswith("batched96"):
        return batched_bench(args, unsteady=args.workload.endswith("streaklines"))
    if args.workload == "hex256-f32":
        return hex_bench(args)
    if args.workload == "forward256-f32":
        return forward_bench(args)
    dev = torch.device("cuda:0")
    log("building inputs", args.workload)
    t0 = time.perf_counter()
    blk, seeds, fmt, m, h, stride = build_inputs(args.workload)
    log(f"inputs ready in {time.perf_counter() - t0:.1f}s: field {blk.stored.nbytes / 1e6:.1f} MB, "
        f"{len(seeds)} seeds")

    stream = torch.cuda.current_stream()
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 3 x 1 GiB device-to-device")
    t0 = time.perf_counter()
    f = S.Field([blk], fmt, layout=args.layout)
    torch.cuda.synchronize()
    ingest_s = time.perf_counter() - t0
    layout, field_bytes = S.streami_field_info(f.h)
    log(f"layout {LAYOUT_NAMES[layout]} ({field_bytes / 1e9:.2f} GB stored)")
    d_seeds = torch.from_numpy(seeds).to(dev)
    torch.cuda.synchronize()

    kw = dict(waves_per_cu=args.waves_per_cu, refill_threshold=args.refill,
              no_cell_cache=int(args.no_cell_cache), use_graph=int(args.graph),
              lds_cell_cache=int(args.lds_cell_cache))

    def one_step(stats=False):
        f.clear()
        f.seed(0, d_seeds, default_max_steps=m, record_stride=stride)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        p = S.advect_params(h, **kw)
        st = S.streami_advect(f.h, p, want_stats=stats)
        e1.record(stream)
        return st, e0, e1

    # warmup (the first also provides the deterministic per-step counts)
    st0 = None
    for w in range(max(1, args.warmup)):
        st, _, _ = one_step(stats=True)
        st0 = st0 or st
        log(f"warmup {w}: {st.steps} particle-steps in {st.device_ms:.2f} ms "
            f"({st.steps / st.device_ms / 1e6:.3f} G steps/s), exits {st.terminated[2]}, "
            f"max-steps {st.terminated[1]}")
    steps_per_pass = int(st0.steps)
    verts_per_pass = int(st0.vertices)

    torch.cuda.synchronize()
    events = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        _, e0, e1 = one_step(stats=False)
        events.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    adv_ms = [e0.elapsed_time(e1) for e0, e1 in events]
    log(f"timed {args.steps} steps: wall {wall * 1e3:.1f} ms, advect "
        f"{np.mean(adv_ms):.3f} ms mean ({min(adv_ms):.3f} min)")

    # one-time costs outside the timed region
    t0 = time.perf_counter()
    n_lines = min(len(seeds), 65536)
    L = f.lines(0, 0, n_lines)
    fetch_s = time.perf_counter() - t0
    ob = f.outbox(cap=len(seeds))

    value = steps_per_pass * args.steps / wall
    mean_adv_s = float(np.mean(adv_ms)) / 1e3
    gathers = int(st0.gathers)
    node_bytes = 4 if fmt == S.F32 else 2
    # the method's own count (every sample gathers its 8 corners): an upper bound that ignores
    # the reuse of a cell across samples, kept only as the reuse ratio below
    alg_bytes = steps_per_pass * 96 * node_bytes + verts_per_pass * 12
    refill_bytes = 96 if layout == S.LAYOUT_CELL else 8 * (12 if fmt == S.F32 else 8)
    comp = compulsory_bytes(gathers, refill_bytes, verts_per_pass, len(seeds), int(st0.outbox))
    achieved = comp["total"] / mean_adv_s / 1e9
    traffic = None
    counters = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_advect_{args.workload}.json")
    if os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
            if tj.get("kernel_hash") == kernel_source_hash() and tj.get("layout", 0) == layout:
                traffic = tj.get("hbm_bytes_per_launch")
                if "valu_instructions" in tj:
                    # what bounds the kernel, from the same profiled revision's counters
                    counters = {"valu_instructions": tj["valu_instructions"], "l2_hit_rate": tj.get("l2_hit"),
                                "clock_ghz": tj.get("clock_ghz"), "source": os.path.relpath(tfile, ROOT)}
        except Exception:
            traffic = counters = None
    out = {
        "metric": "RK4 particle-steps/s + HBM GB/s; surrogate vs plain at fixed endpoint error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {S.F32: "f32", S.F16: "f16 storage, f32 math", S.BF16: "bf16 storage, f32 math"}[fmt],
        "data": "synthetic",
        "config": {"workload": args.workload, "field": f"{WORKLOADS[args.workload][0]}^3 + ghost",
                   "seeds": len(seeds), "max_steps": m, "h": h, "record_stride": stride,
                   "particle_steps_per_step": steps_per_pass, "vertices_per_step": verts_per_pass,
                   "layout": LAYOUT_NAMES[layout] + (" (auto)" if args.layout == 0 else ""),
                   "field_bytes": field_bytes, "waves_per_cu": args.waves_per_cu,
                   "cell_cache": ("off" if args.no_cell_cache else "lds" if args.lds_cell_cache else "registers"),
                   "graph": args.graph},
        # compulsory bytes of the cached kernel per launch (cell refills x stored refill bytes,
        # 12 B per recorded vertex, particle state and outbox records) over k_advect's mean
        # launch time, against the published HBM peak; `traffic` is the counted HBM bytes
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_frac": None if traffic is None else traffic / mean_adv_s / 1e9 / HBM_PEAK_GBS,
                     "kernel": "k_advect", "compulsory_bytes_per_launch": comp,
                     "mean_launch_ms": mean_adv_s * 1e3, "kernel_hash": kernel_source_hash(),
                     "counters": counters,
                     "reuse": {"alg_bytes_per_launch": alg_bytes, "alg_over_compulsory": alg_bytes / comp["total"]}},
        "advect_only_steps_per_s": steps_per_pass / mean_adv_s,
        "cell_refills_per_step": gathers / steps_per_pass,
        "ingest_ms": ingest_s * 1e3,
        "fetch_lines_ms_per_65536": fetch_s * 1e3,
        "outbox_records": int(len(ob)),
    }
    if counters is not None:
        # VALU busy fraction: the profiled instruction count at the measured issue cost of a
        # VOP2 add (lower bound) and of a VOP3 FMA (upper bound) per wave64 instruction
        n_simd = 4 * torch.cuda.get_device_properties(0).multi_processor_count
        cyc = {}
        for kind, name in ((0, "fma_f32"), (1, "add_u32")):
            ms, n = S.streami_probe_valu(kind, 32)
            cyc[name] = n_simd * CLOCK_GHZ * 1e9 * ms * 1e-3 / n
        slots = n_simd * CLOCK_GHZ * 1e9 * mean_adv_s
        counters["valu_cycles_per_instruction"] = cyc
        counters["valu_busy_range"] = [counters["valu_instructions"] * cyc["add_u32"] / slots,
                                       counters["valu_instructions"] * cyc["fma_f32"] / slots]
        log(f"VALU busy between {counters['valu_busy_range'][0]:.2f} and {counters['valu_busy_range'][1]:.2f} "
            f"(fma {cyc['fma_f32']:.2f}, add {cyc['add_u32']:.2f} cycles per wave64 instruction)")
    if layout == S.LAYOUT_CELL:
        # gather roofline: the lanes' cell-cache misses are random 96-byte record reads from
        # the stored field; set their rate against the measured rate of such reads
        probe = memory_probe(S, field_bytes, 96)
        g_rate = gathers * 96 / mean_adv_s / 1e9
        peak = probe["read_GBps"]["field"]
        out["gather_roofline"] = {
            "bound": "random 96-B record reads over the stored field (measured peak)", "achieved": g_rate,
            "peak": peak, "unit": "GB/s", "frac": g_rate / peak, "gathers_per_launch": gathers,
            "gathers_per_particle_step": gathers / steps_per_pass, "probe": probe}
        log(f"gathers {gathers / steps_per_pass:.3f} per step: {g_rate:.0f} GB/s of records against "
            f"{peak:.0f} GB/s measured for random record reads at {field_bytes / 1e9:.2f} GB "
            f"(copy {probe['copy_GBps']:.0f} GB/s)")
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(blk, seeds, h, m)
        log(f"cpu baseline {out['cpu_baseline']['value']:.3g} steps/s on {out['cpu_baseline']['cores']} threads")
    f.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
