"""Launch-configuration autotuner for the batched advection launch.

Times the caller's whole pass (seeding plus every advect call of it) under each
candidate -- node layout (x-fastest rows, 4x4x4 or 8x8x8 bricks: the brick size, and
for steady FP32 fields per-cell coefficient records), waves per CU,
refill threshold, work order -- through the C-ABI, and caches the fastest per
(device, dtype, block shapes, caller's signature) in a JSON file
(STREAMI_TUNE_CACHE, default ~/.cache/streami/autotune.json).  Results are
bit-identical under every candidate; only the time differs.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

CANDIDATES = [dict(waves_per_cu=w, refill_threshold=r, work_order=o)
              for w in (16, 24, 32) for r in (1, 16) for o in (0, 1)]


def _layouts(blocks, fmt):
    steady_f32 = fmt == 0 and all(int(b.n_slices) == 1 for b in blocks)
    return (1, 2, 5, 3) if steady_f32 else (1, 2, 5)


def _cache_path():
    return os.environ.get("STREAMI_TUNE_CACHE", os.path.expanduser("~/.cache/streami/autotune.json"))


def _key(blocks, fmt, sig):
    import torch
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    h = hashlib.sha1(json.dumps([[list(b.dims), int(b.n_slices)] for b in blocks] + [fmt, sig]).encode())
    return f"{dev}|{fmt}|{len(blocks)}|{h.hexdigest()[:16]}"


def load(blocks, fmt, sig):
    """The cached configuration for this workload, or None."""
    try:
        return json.load(open(_cache_path())).get(_key(blocks, fmt, sig))
    except (OSError, ValueError):
        return None


def tune(blocks, fmt, pass_fn, sig, log=None, repeats=2, nodes=None, candidates=None):
    """Return the fastest configuration {layout, waves_per_cu, refill_threshold, work_order, ms}.

    pass_fn(field, cfg) runs one whole pass on `field` (a Field over `blocks` with the
    candidate's layout) with advect keyword arguments `cfg`; it is timed by wall clock
    between two device synchronisations.  `sig` (JSON-able) names everything else the
    pass depends on (seed counts, step, windows) for the cache key.  `nodes` (optional)
    are the blocks' stored nodes when the blocks do not carry them; `candidates` (optional)
    replaces the launch shapes tried under each layout (a pass of seconds cannot afford all).
    """
    cands = CANDIDATES if candidates is None else list(candidates)
    from . import Field
    import torch
    best = None
    trials = []
    from . import StreamiError, E_UNSUPPORTED
    for layout in _layouts(blocks, fmt):
        try:
            f = Field(blocks, fmt, layout=layout, nodes=nodes)
        except StreamiError as e:  # a layout the blocks' shapes do not fit (32-bit plane offsets)
            if e.code != E_UNSUPPORTED:
                raise
            if log:
                log(f"tune layout={layout}: not possible for these blocks ({e})")
            continue

        def one(cfg):
            torch.cuda.synchronize()
            t = time.perf_counter()
            pass_fn(f, cfg)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) * 1e3

        one(cands[0])  # warm-up
        for cfg in cands:
            ms = min(one(cfg) for _ in range(repeats))
            trials.append(dict(layout=layout, ms=ms, **cfg))
            if log:
                log(f"tune layout={layout} {cfg}: {ms:.3f} ms")
            if best is None or ms < best["ms"]:
                best = dict(layout=layout, ms=ms, **cfg)
        f.close()
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        cache[_key(blocks, fmt, sig)] = best
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    best = dict(best)
    best["trials"] = trials
    return best
