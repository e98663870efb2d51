"""16-bit node storage (BF16/FP16, FP32 interpolation and accumulation).

Parity: each format against the FP64 oracle on the same stored (dequantised)
nodes, by the per-step check.  Accuracy: the endpoint error against the FP64
oracle on the unrounded field, per format, stated and bounded (a run over
Gaussian seed blobs, as in the 512^3 workload, at reduced size).
"""
import sys

import numpy as np
import pytest

import fieldgen as fg
import oracle
from tests import parity

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_02627_amd as S
    S._load()
    return S


def test_precision_table(S):
    edge, steps, h = 96, 300, 0.5
    seeds = fg.blob_seeds(31, 8, 512, float(edge), 12.0, 4.0)
    acc_field = None
    errs = {}
    for fmt in (fg.F32, fg.BF16, fg.F16):
        note("precision", fg.DTYPE_NAMES[fmt])
        blk = fg.turbulence_block(3, edge=edge, fmt=fmt, rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
        f = S.Field([blk], fmt)
        f.seed(0, seeds, default_max_steps=steps)
        f.advect(h)
        L = f.lines(0)
        f.close()
        F = oracle.Field.from_block(blk)
        ratio, _ = parity.local_check(F, L, h, float(edge))
        assert ratio <= 1.0, (fmt, ratio)
        if acc_field is None:
            acc_field = oracle.Field.from_block(blk, use_values=True)
            ref = acc_field.trace(seeds, h, steps, keep_verts=False)
        end = L["xyz"][L["offsets"][1:] - 1].astype(np.float64)
        err = np.abs(end - ref["final_pos"]).max(axis=1) / edge
        errs[fg.DTYPE_NAMES[fmt]] = (float(np.median(err)), float(np.quantile(err, 0.9)), float((err <= 2e-3).mean()))
    note("endpoint error / extent vs the FP64 field (median, p90, frac <= 2e-3):", errs)
    assert errs["f32"][0] <= 1e-4
    assert errs["bf16"][0] <= 2e-3 and errs["f16"][0] <= 2e-3
    assert errs["f16"][0] <= errs["bf16"][0]  # 11-bit vs 8-bit significand


def test_full_size_512_accuracy_vs_fp64(S):
    """The 512^3 workload as benchmarked (4M seeds in 64 blobs, h = 0.5, up to 4000 steps,
    every 8th vertex kept), stored in FP32, BF16 and FP16: the endpoint error of the first
    2048 seeds against the FP64 oracle on the unrounded field, per format."""
    seeds = fg.blob_seeds(3, 64, 65536, 512.0, 24.0, 8.0)
    k, h, m = 2048, 0.5, 4000
    acc = None
    rows = {}
    for fmt in (fg.F32, fg.BF16, fg.F16):
        name = fg.DTYPE_NAMES[fmt]
        note("512^3 accuracy", name)
        blk = fg.turbulence_block(3, edge=512, fmt=fmt)
        f = S.Field([blk], fmt)
        f.seed(0, seeds, default_max_steps=m, record_stride=8)
        st = f.advect(h)
        assert st.active == 0
        L = f.lines(0, 0, k)
        f.close()
        if acc is None:
            acc = oracle.Field.from_block(blk, use_values=True).trace(seeds[:k], h, m, keep_verts=False)
        del blk
        end = L["xyz"][L["offsets"][1:] - 1].astype(np.float64)
        err = np.abs(end - acc["final_pos"]).max(axis=1) / 512.0
        same = (acc["code"] == L["codes"]) & (acc["steps"] == L["steps"])
        rows[name] = dict(median=float(np.median(err)), p90=float(np.quantile(err, 0.9)), max=float(err.max()),
                          within_2e3=float((err <= 2e-3).mean()), within_1e4=float((err <= 1e-4).mean()),
                          same_code_and_steps=float(same.mean()))
        note(name, rows[name])
    assert rows["f32"]["median"] <= 1e-4 and rows["f32"]["within_2e3"] >= 0.95
    assert rows["bf16"]["median"] <= 2e-3 and rows["f16"]["median"] <= 2e-3
    assert rows["f32"]["median"] <= rows["f16"]["median"] <= rows["bf16"]["median"]
