"""Launch-configuration autotuner for the batched advection launch.

Times the real workload under each candidate (node layout: x-fastest rows or
4x4x4 bricks; waves per CU; refill threshold; work order) through the C-ABI
and caches the fastest per (device, dtype, block shapes, seed counts) in a
JSON file (STREAMI_TUNE_CACHE, default ~/.cache/streami/autotune.json).
Results are bit-identical under every candidate; only the time differs.
"""
from __future__ import annotations

import hashlib
import json
import os

CANDIDATES = [dict(waves_per_cu=w, refill_threshold=r, work_order=o)
              for w in (16, 24, 32) for r in (1, 16) for o in (0, 1)]
LAYOUTS = (1, 2)


def _cache_path():
    return os.environ.get("STREAMI_TUNE_CACHE", os.path.expanduser("~/.cache/streami/autotune.json"))


def _key(blocks, seeds, fmt, h):
    import torch
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    sig = hashlib.sha1(json.dumps([[list(b.dims), int(b.n_slices)] for b in blocks] + [[len(s) for s in seeds]]
                                  + [fmt, h]).encode()).hexdigest()[:16]
    return f"{dev}|{fmt}|{len(blocks)}|{sig}"


def load(blocks, seeds, fmt, h):
    try:
        return json.load(open(_cache_path())).get(_key(blocks, seeds, fmt, h))
    except (OSError, ValueError):
        return None


def tune(blocks, seeds, limits, fmt, h, record_stride=1, run_fn=None, log=None, repeats=2):
    """Return the fastest configuration {layout, waves_per_cu, refill_threshold, work_order, ms}.

    run_fn(field, params) -> device ms may replace the default seed+advect pass."""
    from . import Field, streami_advect, advect_params
    import torch
    best = None
    trials = []
    for layout in LAYOUTS:
        f = Field(blocks, fmt, layout=layout)
        dseeds = [torch.from_numpy(s).cuda() for s in seeds]
        dlim = [torch.from_numpy(m).cuda() for m in limits]

        def one(cfg):
            f.clear()
            for b in range(len(blocks)):
                f.seed(b, dseeds[b], max_steps=dlim[b], record_stride=record_stride)
            st = streami_advect(f.h, advect_params(h, **cfg))
            return st.device_ms

        one(CANDIDATES[0])  # warm-up
        for cfg in CANDIDATES:
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
        cache[_key(blocks, seeds, fmt, h)] = best
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    best = dict(best)
    best["trials"] = trials
    return best
