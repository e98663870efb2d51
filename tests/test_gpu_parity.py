"""GPU (gfx950) parity of the advection path against the FP64 oracle.

Every test calls the HIP library through its C-ABI binding and compares with
the oracle on the same stored node values; see tests/parity.py for the
contract.  Sizes span several tiles of the launch (many waves and workgroups)
with ragged tails; the full-size turbulence case runs the exact launch
configuration the benchmark times.
"""
import sys

import numpy as np
import pytest

import fieldgen as fg
import oracle
from tests import parity

pytestmark = pytest.mark.gpu

FMT_TO_ORC = {fg.F32: oracle.FMT_F32, fg.F16: oracle.FMT_F16, fg.BF16: oracle.FMT_BF16}


def note(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2606_02627_amd as S
    S._load()
    return S


def run(S, blocks, seeds_per_block, h, max_steps, dtype, layout=0, eps=1e-6, stride=1, **adv):
    """Seed every block, advect to completion, return (field, lines per block, outbox, stats)."""
    f = S.Field(blocks, dtype, layout=layout)
    for b, sd in enumerate(seeds_per_block):
        ms = max_steps[b] if isinstance(max_steps, list) else max_steps
        if isinstance(ms, np.ndarray):
            tbs = adv.pop("t_births", None) if b == 0 else None
            f.seed(b, np.ascontiguousarray(sd, np.float32), max_steps=ms.astype(np.int32),
                   record_stride=stride, t_birth=adv.pop("t_birth", 0.0) if b == 0 else 0.0,
                   t_births=None if tbs is None else np.ascontiguousarray(tbs, np.float32))
        else:
            f.seed(b, np.ascontiguousarray(sd, np.float32), default_max_steps=int(ms),
                   record_stride=stride)
    budget = adv.pop("chunk", 0)
    if budget:
        while True:
            st = f.advect(h, step_budget=budget, eps=eps, **adv)
            if st.active == 0:
                break
    else:
        st = f.advect(h, eps=eps, **adv)
    lines = [f.lines(b) for b in range(len(blocks))]
    ob = f.outbox()
    return f, lines, ob, st


def orc_field(blk):
    return oracle.Field.from_block(blk)


# ---------------------------------------------------------------- closed forms
def test_uniform_flow_bit_exact(S):
    """Dyadic uniform flow: the FP32 kernel reproduces P0 + n h c exactly, and the exit step,
    outbox position and destination rank exactly."""
    note("uniform flow")
    c = (0.375, -0.25, 0.125)
    blk = fg.closed_form_block(lambda x, y, z: (0 * x + c[0], 0 * x + c[1], 0 * x + c[2]),
                               (9, 9, 9), ghost=1, origin=(0.5, 0.5, 0.5), lo=(0, 0, 0),
                               hi=(9, 9, 9), rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    rng = np.random.default_rng(1)
    seeds = (rng.integers(0, 9 * 64, size=(777, 3)) / 64.0).astype(np.float32)
    for layout in (S.LAYOUT_LINEAR, S.LAYOUT_BRICK4, S.LAYOUT_BRICK8, S.LAYOUT_CELL):
        f, lines, ob, st = run(S, [blk], [seeds], 0.5, 1000, fg.F32, layout=layout)
        segs = parity.split_lines(lines[0])
        for i, s in enumerate(segs):
            n = len(s) - 1
            path = seeds[i].astype(np.float64) + np.arange(n + 1)[:, None] * 0.5 * np.array(c)
            np.testing.assert_array_equal(s, path)
            k = np.arange(1, 1000)
            pos = seeds[i] + k[:, None] * 0.5 * np.array(c)
            assert n == k[np.any((pos < 0) | (pos >= 9), axis=1)][0]
        assert (lines[0]["codes"] == S.EXIT).all()
        ref = orc_field(blk).trace(seeds, 0.5, 1000)
        srt = np.sort(ob, order="id")
        assert len(srt) == len(seeds)
        np.testing.assert_array_equal(srt["dest"], ref["out_dest"])
        np.testing.assert_array_equal(srt["pos"].astype(np.float64), ref["out_pos"])
        np.testing.assert_array_equal(srt["steps"], ref["steps"])


def test_gather_counts(S):
    """streami_stats.gathers counts the lanes' cell-cache misses: on a dyadic uniform flow the
    stage points are exact, so the count equals the number of cell changes along each
    particle's sample sequence (k1, k2, k3, k4 of every step), the same for node rows and cell
    records; without the cache every sample is a gather."""
    note("gather counts")
    c = (0.375, -0.25, 0.125)
    blk = fg.closed_form_block(lambda x, y, z: (0 * x + c[0], 0 * x + c[1], 0 * x + c[2]),
                               (9, 9, 9), ghost=1, origin=(0.5, 0.5, 0.5), lo=(0, 0, 0),
                               hi=(9, 9, 9), rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    rng = np.random.default_rng(3)
    seeds = (rng.integers(0, 9 * 64, size=(301, 3)) / 64.0).astype(np.float32)
    h, cv = 0.5, np.array(c)
    expect, total_steps = 0, 0
    for p0 in seeds.astype(np.float64):
        key, p = None, p0.copy()
        while True:
            for q in (p, p + 0.5 * h * cv, p + 0.5 * h * cv, p + h * cv):
                cell = tuple(int(min(max(np.floor(v + 0.5), 0), 9)) for v in q)
                if cell != key:
                    expect, key = expect + 1, cell
            p = p + h * cv
            total_steps += 1
            if ((p < 0) | (p >= 9)).any():
                break
    for layout in (S.LAYOUT_LINEAR, S.LAYOUT_CELL):
        f, lines, ob, st = run(S, [blk], [seeds], h, 1000, fg.F32, layout=layout)
        assert st.steps == total_steps and st.gathers == expect, (layout, st.steps, st.gathers, expect)
        f, lines, ob, st = run(S, [blk], [seeds], h, 1000, fg.F32, layout=layout, no_cell_cache=1)
        assert st.gathers == 4 * total_steps, (layout, st.gathers)


def test_memory_probe_reads_what_it_reports(S):
    """The probes (random record reads over a device buffer; VALU issue rate) run for every
    record size and instruction kind and report the work they did and a positive time."""
    import torch
    buf = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    for rec in (16, 96, 128):
        ms, n = S.streami_probe_gather(buf, rec, 8, 2, 4)  # 4 waves per CU: one workgroup per CU
        assert ms > 0 and n == n_cu * 256 * 8, (rec, ms, n)
        note(f"probe {rec} B: {n} records in {ms:.3f} ms")
    with pytest.raises(S.StreamiError):
        S.streami_probe_gather(buf[:8], 16, 8, 2, 4)
    for kind in (0, 1, 2, 3):
        ms, n = S.streami_probe_valu(kind, 4)
        assert ms > 0 and n == n_cu * 4 * 1024 * 128, (kind, ms, n)
        note(f"valu probe kind {kind}: {4 * n_cu * 2.4e6 * ms / n:.2f} cycles per wave64 instruction at 2.4 GHz")


def test_time_blend_closed_form(S):
    """Two slices of a uniform flow, V1 = 2 V0, slice_dt = 8: the velocity grows linearly in
    time, RK4 integrates it exactly (Simpson's rule), and with dyadic data every vertex equals
    P0 + c (t + t^2 / 16) bit for bit -- for FP32 node rows and cell records and FP16 nodes."""
    import dataclasses
    note("time blend closed form")
    c = np.array([0.375, -0.25, 0.125])
    base = fg.closed_form_block(lambda x, y, z: (0 * x + c[0], 0 * x + c[1], 0 * x + c[2]), (16, 16, 16),
                                ghost=1, origin=(0.5, 0.5, 0.5), lo=(0, 0, 0), hi=(16, 16, 16))
    vals = np.concatenate([base.values, 2.0 * base.values])
    rng = np.random.default_rng(8)
    seeds = (4.0 + rng.integers(0, 6 * 32, size=(300, 3)) / 32.0).astype(np.float32)  # stay inside
    h, steps, dt = 0.5, 16, 8.0
    t = np.arange(steps + 1) * h
    for fmt, layout in ((fg.F32, S.LAYOUT_LINEAR), (fg.F32, S.LAYOUT_CELL), (fg.F16, S.LAYOUT_LINEAR)):
        blk = dataclasses.replace(base, values=vals, n_slices=2, slice_dt=dt, t0=0.0).quantise(fmt)
        f, lines, ob, st = run(S, [blk], [seeds], h, steps, fmt, layout=layout)
        assert st.steps == len(seeds) * steps and (lines[0]["codes"] == S.MAX_STEPS).all()
        for i, seg in enumerate(parity.split_lines(lines[0])):
            want = seeds[i].astype(np.float64) + (t + t * t / (2 * dt))[:, None] * c
            np.testing.assert_array_equal(seg, want, err_msg=f"{fg.DTYPE_NAMES[fmt]} layout {layout}")



def test_time_clamped_at_both_ends(S):
    """Slices c, 2c, 3c at t0 = 0.5, slice_dt = 4: particles born at t = 10 (past the last
    slice, 8.5) move on straight lines at 3c, and particles that live in t < t0 at c -- the
    blend is clamped to the end slices, as in the oracle."""
    import dataclasses
    note("time clamp")
    c = np.array([0.375, -0.25, 0.125])
    base = fg.closed_form_block(lambda x, y, z: (0 * x + c[0], 0 * x + c[1], 0 * x + c[2]), (16, 16, 16),
                                ghost=1, origin=(0.5, 0.5, 0.5), lo=(0, 0, 0), hi=(16, 16, 16))
    vals = np.concatenate([base.values, 2.0 * base.values, 3.0 * base.values])
    rng = np.random.default_rng(9)
    seeds = (4.0 + rng.integers(0, 6 * 32, size=(200, 3)) / 32.0).astype(np.float32)  # stay inside
    h, steps = 0.5, 8
    tau = (np.arange(steps + 1) * h)[:, None]
    for fmt, layout in ((fg.F32, S.LAYOUT_LINEAR), (fg.F32, S.LAYOUT_CELL), (fg.F16, S.LAYOUT_LINEAR)):
        blk = dataclasses.replace(base, values=vals, n_slices=3, slice_dt=4.0, t0=0.5).quantise(fmt)
        for t_birth, speed in ((10.0, 3.0), (-6.0, 1.0)):
            f = S.Field([blk], fmt, layout=layout)
            f.seed(0, seeds, default_max_steps=steps, t_birth=t_birth)
            st = f.advect(h)
            L = f.lines(0)
            assert st.steps == len(seeds) * steps and (L["codes"] == S.MAX_STEPS).all()
            for i, seg in enumerate(parity.split_lines(L)):
                want = seeds[i].astype(np.float64) + speed * c * tau
                np.testing.assert_allclose(seg, want, rtol=0, atol=1e-5,
                                           err_msg=f"{fg.DTYPE_NAMES[fmt]} layout {layout} birth {t_birth}")
            f.close()

def test_solid_body_rotation_closed_form(S):
    """v = w(-(y-3), x-3, 0) lies in the trilinear span: vertices follow R(hA)^n exactly up
    to FP32 rounding (circles shrinking by the RK4 radius factor)."""
    note("rotation")
    w = 0.7
    blk = fg.closed_form_block(lambda x, y, z: (-w * (y - 3.0), w * (x - 3.0), 0 * z), (7, 7, 4),
                               ghost=1, origin=(0, 0, 0), lo=(-1, -1, -1), hi=(100, 100, 100))
    seeds = np.array([[4.5, 3.0, 1.0], [3.0, 1.2, 2.0], [1.7, 3.9, 0.5]], np.float32)
    h, steps = 0.4, 120
    f, lines, ob, st = run(S, [blk], [seeds], h, steps, fg.F32)
    Z = h * np.array([[0, -w, 0], [w, 0, 0], [0, 0, 0]])
    R = np.eye(3) + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    xc = np.array([3.0, 3.0, 0.0])
    for i, s in enumerate(parity.split_lines(lines[0])):
        assert len(s) == steps + 1
        q = seeds[i].astype(np.float64) - xc
        for n in range(steps + 1):
            assert np.abs(s[n] - xc - q).max() < 2e-5
            q = R @ q


# ---------------------------------------------------------------- ABC (config 1)
def test_abc_periodic_full(S):
    """ABC flow on a 32^3 periodic grid, 1024 seeds, h=0.01, 200 steps: every vertex within
    1e-4 of the 2pi extent of the oracle; per-step check on every vertex; codes exact."""
    note("abc 32^3 full")
    blk = fg.abc_block(32)
    seeds = fg.uniform_seeds(1, 1024, (0, 0, 0), (2 * np.pi,) * 3)
    f, lines, ob, st = run(S, [blk], [seeds], 0.01, 200, fg.F32)
    F = orc_field(blk)
    ref = F.trace(seeds, float(np.float32(0.01)), 200)
    ext = 2 * np.pi
    ratio, npairs = parity.local_check(F, lines[0], 0.01, ext)
    assert npairs == 1024 * 200 and ratio <= 1.0, ratio
    dev, same = parity.global_compare(lines[0], ref, 1024)
    assert same.all() and dev.max() <= 1e-4 * ext, dev.max()
    assert (lines[0]["steps"] == 200).all() and (lines[0]["codes"] == S.MAX_STEPS).all()
    assert st.steps == 1024 * 200 and len(ob) == 0


# ---------------------------------------------------------------- turbulence blocks
@pytest.mark.parametrize("dtype,layout", [(fg.F32, 1), (fg.F32, 2), (fg.F32, 3), (fg.BF16, 1), (fg.BF16, 2),
                                          (fg.F16, 1), (fg.F16, 2)])
def test_turbulence_block_parity(S, dtype, layout):
    """A 40^3 turbulence block (+ghost), 3000 seeds (ragged vs 256-lane workgroups), h=0.5,
    up to 400 steps: local check on every vertex, discrete results exact away from the
    boundary, outbox records equal to the oracle's (sorted by id)."""
    note("turbulence 40^3", fg.DTYPE_NAMES[dtype], "layout", layout)
    blk = fg.turbulence_block(2, edge=40, fmt=dtype, rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    seeds = fg.uniform_seeds(2, 3000, (0, 0, 0), (40, 40, 40), sub=7)
    f, lines, ob, st = run(S, [blk], [seeds], 0.5, 400, dtype, layout=layout)
    F = orc_field(blk)
    ratio, npairs = parity.local_check(F, lines[0], 0.5, 40.0)
    assert ratio <= 1.0, ratio
    ref = F.trace(seeds, 0.5, 400)
    dev, same = parity.global_compare(lines[0], ref, len(seeds))
    sens = parity.boundary_sensitive(ref, lines[0], dev, blk.lo, blk.hi, field=F)
    ok = ~sens
    assert ok.mean() > 0.9
    np.testing.assert_array_equal(lines[0]["codes"][ok], ref["code"][ok])
    np.testing.assert_array_equal(lines[0]["steps"][ok], ref["steps"][ok])
    # ids are 0..n-1 in seed order; the outbox holds exactly the EXIT particles
    srt = np.sort(ob, order="id")
    exits = np.nonzero(lines[0]["codes"] == S.EXIT)[0]
    np.testing.assert_array_equal(srt["id"], exits)
    inb = ok[exits]
    np.testing.assert_array_equal(srt["dest"][inb], ref["out_dest"][exits][inb])
    assert np.abs(srt["pos"][inb] - ref["out_pos"][exits][inb]).max(initial=0) <= 1e-4 * 40 + dev[exits][inb].max(initial=0)
    assert st.steps == int(lines[0]["steps"].sum())


def test_bit_identical_variants(S):
    """Cell cache on/off (in registers or in LDS), node rows / 4^3 and 8^3 bricks / cell records,
    the interior test on/off, hipGraph replay and chunked resume all give bit-identical lines,
    steps, codes and outbox contents; for 16-bit nodes, rows and both brick sizes agree too."""
    note("variants")
    blk = fg.turbulence_block(2, edge=32, rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    seeds = fg.uniform_seeds(2, 2500, (0, 0, 0), (32, 32, 32), sub=9)
    base = run(S, [blk], [seeds], 0.5, 300, fg.F32)
    variants = [dict(no_cell_cache=1), dict(layout=1), dict(layout=2), dict(layout=5), dict(layout=5, no_cell_cache=1),
                dict(layout=3),
                dict(layout=3, no_cell_cache=1), dict(checked_samples=1), dict(layout=1, checked_samples=1),
                dict(use_graph=1), dict(chunk=37),
                dict(waves_per_cu=8, refill_threshold=1), dict(work_order=1), dict(lds_cell_cache=1),
                dict(layout=3, lds_cell_cache=1, checked_samples=1)]
    for v in variants:
        note("variant", v)
        layout = v.pop("layout", 0)
        got = run(S, [blk], [seeds], 0.5, 300, fg.F32, layout=layout, **v)
        for k in ("offsets", "xyz", "steps", "codes", "ids"):
            np.testing.assert_array_equal(got[1][0][k], base[1][0][k])
        np.testing.assert_array_equal(np.sort(got[2], order="id"), np.sort(base[2], order="id"))
    b16 = fg.turbulence_block(2, edge=30, fmt=fg.F16, rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    s16 = fg.uniform_seeds(2, 1500, (0, 0, 0), (30, 30, 30), sub=10)
    base = run(S, [b16], [s16], 0.5, 300, fg.F16, layout=1)
    for layout in (2, 5):
        note("variant 16-bit layout", layout)
        got = run(S, [b16], [s16], 0.5, 300, fg.F16, layout=layout)
        for k in ("offsets", "xyz", "steps", "codes", "ids"):
            np.testing.assert_array_equal(got[1][0][k], base[1][0][k])


@pytest.mark.parametrize("dtype", [fg.BF16, fg.F16])
@pytest.mark.parametrize("kind", ["steady", "unsteady", "batched"])
def test_packed_16bit_cache_bit_identical(S, dtype, kind):
    """16-bit nodes keep their cached corners packed (two per register) and widen them at
    each sample; the results equal those of re-gathering every sample, and those of 8^3-node
    bricks, bit for bit, for one block, for time-blended slices and for several blocks in one
    launch."""
    note("packed 16-bit cache", fg.DTYPE_NAMES[dtype], kind)
    if kind == "batched":
        blocks = [fg.turbulence_block(4, dims=d, fmt=dtype, sub=b, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0),
                                      n_slices=3, slice_dt=50.0)
                  for b, d in enumerate([(20, 28, 16), (32, 12, 24), (16, 16, 30)])]
    else:
        ns = 4 if kind == "unsteady" else 1
        blocks = [fg.turbulence_block(2, edge=28, fmt=dtype, rank_grid=(3, 3, 3), rank_coord=(1, 1, 1),
                                      n_slices=ns, slice_dt=40.0)]
    seeds = [fg.uniform_seeds(2, 1300 + 100 * b, (0, 0, 0), blk.dims, sub=20 + b) for b, blk in enumerate(blocks)]
    base = run(S, blocks, seeds, 0.5, 300, dtype)
    for extra in (dict(no_cell_cache=1), dict(layout=S.LAYOUT_BRICK8)):
        got = run(S, blocks, seeds, 0.5, 300, dtype, **extra)
        assert got[3].steps == base[3].steps > 0
        for b in range(len(blocks)):
            for k in ("offsets", "xyz", "steps", "codes", "ids"):
                np.testing.assert_array_equal(got[1][b][k], base[1][b][k])
        np.testing.assert_array_equal(np.sort(got[2], order=["block", "id"]),
                                      np.sort(base[2], order=["block", "id"]))


def test_graph_replays(S):
    """A captured launch replayed on a fresh particle set each time matches eager runs."""
    note("graph replays")
    blk = fg.turbulence_block(2, edge=24, rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    seeds = fg.uniform_seeds(2, 1000, (0, 0, 0), (24, 24, 24), sub=3)
    eager = run(S, [blk], [seeds], 0.5, 200, fg.F32)[1][0]
    f = S.Field([blk], fg.F32)
    f.seed(0, seeds, default_max_steps=200)
    for rep in range(3):
        st = f.advect(0.5, step_budget=50, use_graph=1)
        import torch
        torch.cuda.synchronize()
    st = f.advect(0.5, step_budget=0, use_graph=1)
    got = f.lines(0)
    for k in ("offsets", "xyz", "steps", "codes"):
        np.testing.assert_array_equal(got[k], eager[k])


# ---------------------------------------------------------------- edge cases
# Every exit, limit and error rule holds for each stored layout and format (the
# values involved are exact in all three formats).
EDGE_FORMS = [(fg.F32, 0), (fg.F32, 1), (fg.F32, 2), (fg.F32, 3), (fg.BF16, 1), (fg.F16, 2)]


@pytest.mark.parametrize("dtype,layout", EDGE_FORMS)
def test_edge_cases(S, dtype, layout):
    note("edge cases", fg.DTYPE_NAMES[dtype], "layout", layout)
    c = (0.25, 0.0, 0.0)
    blk = fg.closed_form_block(lambda x, y, z: (0 * x + c[0], 0 * x, 0 * x), (4, 4, 4), ghost=1,
                               origin=(0.5, 0.5, 0.5), lo=(0, 0, 0), hi=(4, 4, 4),
                               rank_grid=(3, 3, 3), rank_coord=(1, 1, 1), fmt=dtype)
    f = S.Field([blk], dtype, layout=layout)
    seeds = np.array([[4.0, 1, 1], [-1e-3, 1, 1], [1, 1, 1], [1, 2, 3], [2.5, 0.5, 3.9]], np.float32)
    ms = np.array([10, 10, 0, 3, 100], np.int32)
    f.seed(0, seeds, max_steps=ms, record_stride=2)
    st = f.advect(0.5)
    L = f.lines(0)
    assert list(L["codes"]) == [S.EXIT, S.EXIT, S.MAX_STEPS, S.MAX_STEPS, S.EXIT]
    # the last seed moves 0.125 per step from x=2.5 and reaches x=4.0 (outside) at step 12
    assert list(L["steps"]) == [0, 0, 0, 3, 12]
    # stride 2 keeps vertices 0, 2, ... and the last one
    assert list(np.diff(L["offsets"])) == [1, 1, 1, 3, 7]
    ob = np.sort(f.outbox(cap=2), order="id")  # forces the capacity path
    assert list(ob["id"]) == [0, 1, 4] and list(ob["steps"]) == [0, 0, 12]
    assert list(ob["dest"]) == [14, 12, 14]
    # capacity two-call pattern
    rc, need = S.streami_fetch_lines(f.h, 0, 0, 5, np.zeros(6, np.int64), np.zeros((2, 3), np.float32), 2)
    assert rc == S.E_CAPACITY and need == 13
    # advect again: nothing active, nothing changes
    st2 = f.advect(0.5)
    assert st2.steps == 0 and st2.active == 0


@pytest.mark.parametrize("dtype,layout", EDGE_FORMS)
def test_stagnation_nonfinite_halo(S, dtype, layout):
    note("stagnation / nonfinite / halo miss", fg.DTYPE_NAMES[dtype], "layout", layout)
    # stagnant field (1e-7 stores as about 1e-7 in every format, below eps = 1e-6)
    blk = fg.closed_form_block(lambda x, y, z: (0 * x + 1e-7, 0 * x, 0 * x), (4, 4, 4),
                               lo=(-10, -10, -10), hi=(10, 10, 10), fmt=dtype)
    f = S.Field([blk], dtype, layout=layout)
    f.seed(0, np.array([[1, 1, 1]], np.float32), default_max_steps=5)
    f.advect(0.5)
    assert f.lines(0)["codes"][0] == S.STAGNANT
    # NaN node
    b2 = fg.closed_form_block(lambda x, y, z: (0 * x + 1, 0 * x, 0 * x), (4, 4, 4),
                              lo=(-10, -10, -10), hi=(10, 10, 10))
    b2.values[0, 2, 2, 3, 1] = np.nan
    b2 = b2.quantise(dtype)
    f = S.Field([b2], dtype, layout=layout)
    f.seed(0, np.array([[0.25, 1.5, 1.5]], np.float32), default_max_steps=10)
    f.advect(0.5)
    L = f.lines(0)
    assert L["codes"][0] == S.NONFINITE and L["steps"][0] == 1
    np.testing.assert_array_equal(L["xyz"][-1], [0.75, 1.5, 1.5])
    # halo miss
    b3 = fg.closed_form_block(lambda x, y, z: (0 * x + 2.0, 0 * x, 0 * x), (4, 4, 4), ghost=1,
                              origin=(0.5, 0.5, 0.5), lo=(0, 0, 0), hi=(4, 4, 4),
                              rank_grid=(3, 3, 3), rank_coord=(1, 1, 1), fmt=dtype)
    f = S.Field([b3], dtype, layout=layout)
    f.seed(0, np.array([[2.0, 2.0, 2.0]], np.float32), default_max_steps=100)
    f.advect(0.75)
    L = f.lines(0)
    assert L["codes"][0] == S.HALO_MISS and L["steps"][0] == 1
    ob = f.outbox()
    assert len(ob) == 1 and ob["code"][0] == S.HALO_MISS and ob["dest"][0] == 14
    np.testing.assert_array_equal(ob["pos"][0], [3.5, 2.0, 2.0])


# ---------------------------------------------------------------- batched + unsteady
def test_batched_blocks_parity(S):
    """Eight blocks of uneven size and seed counts in one launch (FP16 nodes), per-seed
    limits: each block's lines match the oracle run on that block alone."""
    note("batched blocks")
    rng = np.random.default_rng(5)
    blocks, seeds, ms = [], [], []
    for b in range(8):
        dims = tuple(int(v) for v in rng.integers(12, 33, size=3))
        blk = fg.turbulence_block(4, dims=dims, fmt=fg.F16, sub=b, rank_grid=(1, 1, 1),
                                  rank_coord=(0, 0, 0))
        blocks.append(blk)
        n = int(rng.integers(50, 700))
        seeds.append(fg.uniform_seeds(4, n, (0, 0, 0), dims, sub=100 + b))
        ms.append(rng.integers(10, 300, size=n).astype(np.int32))
    f, lines, ob, st = run(S, blocks, seeds, 0.5, ms, fg.F16)
    for b in range(8):
        F = orc_field(blocks[b])
        ratio, _ = parity.local_check(F, lines[b], 0.5, blocks[b].extent)
        assert ratio <= 1.0, (b, ratio)
        ref = F.trace(seeds[b], 0.5, ms[b])
        dev, same = parity.global_compare(lines[b], ref, len(seeds[b]))
        sens = parity.boundary_sensitive(ref, lines[b], dev, blocks[b].lo, blocks[b].hi, field=F)
        np.testing.assert_array_equal(lines[b]["codes"][~sens], ref["code"][~sens])
        np.testing.assert_array_equal(lines[b]["steps"][~sens], ref["steps"][~sens])
    assert set(np.unique(ob["block"])) <= set(range(8))


def test_unsteady_parity(S):
    """Four time slices blended linearly in time (FP16 nodes): local check with each
    vertex's own time, discrete results exact away from the boundary."""
    note("unsteady")
    blk = fg.turbulence_block(6, edge=24, fmt=fg.F16, n_slices=4, slice_dt=40.0,
                              rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
    seeds = fg.uniform_seeds(6, 1500, (0, 0, 0), (24, 24, 24))
    f, lines, ob, st = run(S, [blk], [seeds], 0.5, 300, fg.F16)
    F = orc_field(blk)
    ratio, _ = parity.local_check(F, lines[0], 0.5, 24.0, t_birth=0.0)
    assert ratio <= 1.0, ratio
    ref = F.trace(seeds, 0.5, 300)
    dev, same = parity.global_compare(lines[0], ref, len(seeds))
    sens = parity.boundary_sensitive(ref, lines[0], dev, blk.lo, blk.hi, field=F)
    np.testing.assert_array_equal(lines[0]["codes"][~sens], ref["code"][~sens])


def test_seed_batches_equal_consecutive_seeds(S):
    """streami_seed_batches gives the same particles, ids, lines and outbox as one
    streami_seed call per batch (device and host inputs, per-batch birth times, auto ids)."""
    import torch
    note("seed batches")
    rng = np.random.default_rng(17)
    blocks, seeds, ms, tbs = [], [], [], []
    for b in range(6):
        dims = tuple(int(v) for v in rng.integers(10, 24, size=3))
        blocks.append(fg.turbulence_block(4, dims=dims, fmt=fg.F16, sub=30 + b, rank_grid=(1, 1, 1),
                                          rank_coord=(0, 0, 0), n_slices=2, slice_dt=60.0))
        n = int(rng.integers(1, 500))
        seeds.append(fg.uniform_seeds(4, n, (-1, -1, -1), tuple(d + 1 for d in dims), sub=300 + b))
        ms.append(rng.integers(0, 200, size=n).astype(np.int32))
        tbs.append((rng.integers(0, 8, size=n) * 0.5).astype(np.float32))
    order = [3, 0, 5, 1, 4, 2, 0]  # uneven order, a block seeded twice
    for dev in (True, False):
        conv = (lambda a: torch.from_numpy(a).cuda()) if dev else (lambda a: a)
        a = S.Field(blocks, fg.F16)
        for b in order:
            a.seed(b, conv(seeds[b]), max_steps=conv(ms[b]), t_births=conv(tbs[b]), record_stride=3)
        a.advect(0.5)
        c = S.Field(blocks, fg.F16)
        c.seed_batches([dict(block=b, xyz=conv(seeds[b]), max_steps=conv(ms[b]), t_births=conv(tbs[b]))
                        for b in order], record_stride=3)
        c.advect(0.5)
        for b in range(len(blocks)):
            la, lc = a.lines(b), c.lines(b)
            for k in ("offsets", "xyz", "steps", "codes", "ids"):
                np.testing.assert_array_equal(la[k], lc[k])
        np.testing.assert_array_equal(np.sort(a.outbox(), order="id"), np.sort(c.outbox(), order="id"))
        a.close()
        c.close()


def test_cell_records_periodic_batched_unsteady(S):
    """Cell records (FP32 interpolant coefficients per cell) on the other paths: the
    periodic ABC block (records wrap across the domain) and several blocks in one launch
    give lines bit-identical to node rows; time-blended slices match the oracle."""
    note("cell records: periodic")
    blk = fg.abc_block(32)
    seeds = fg.uniform_seeds(1, 700, (0, 0, 0), (2 * np.pi,) * 3, sub=3)
    a = run(S, [blk], [seeds], 0.01, 150, fg.F32, layout=S.LAYOUT_LINEAR)
    b = run(S, [blk], [seeds], 0.01, 150, fg.F32, layout=S.LAYOUT_CELL)
    for k in ("offsets", "xyz", "steps", "codes", "ids"):
        np.testing.assert_array_equal(a[1][0][k], b[1][0][k])
    note("cell records: batched")
    rng = np.random.default_rng(11)
    blocks, seeds, ms = [], [], []
    for i in range(5):
        dims = tuple(int(v) for v in rng.integers(10, 30, size=3))
        blocks.append(fg.turbulence_block(4, dims=dims, sub=i, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0)))
        n = int(rng.integers(40, 600))
        seeds.append(fg.uniform_seeds(4, n, (0, 0, 0), dims, sub=200 + i))
        ms.append(rng.integers(10, 250, size=n).astype(np.int32))
    a = run(S, blocks, seeds, 0.5, ms, fg.F32, layout=S.LAYOUT_LINEAR)
    b = run(S, blocks, seeds, 0.5, ms, fg.F32, layout=S.LAYOUT_CELL)
    for i in range(5):
        for k in ("offsets", "xyz", "steps", "codes", "ids"):
            np.testing.assert_array_equal(a[1][i][k], b[1][i][k])
    np.testing.assert_array_equal(np.sort(a[2], order="id"), np.sort(b[2], order="id"))
    note("cell records: unsteady")
    blk = fg.turbulence_block(6, edge=24, n_slices=4, slice_dt=40.0, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
    seeds = fg.uniform_seeds(6, 1500, (0, 0, 0), (24, 24, 24))
    f, lines, ob, st = run(S, [blk], [seeds], 0.5, 300, fg.F32, layout=S.LAYOUT_CELL)
    F = orc_field(blk)
    ratio, _ = parity.local_check(F, lines[0], 0.5, 24.0, t_birth=0.0)
    assert ratio <= 1.0, ratio
    ref = F.trace(seeds, 0.5, 300)
    dev, same = parity.global_compare(lines[0], ref, len(seeds))
    sens = parity.boundary_sensitive(ref, lines[0], dev, blk.lo, blk.hi, field=F)
    np.testing.assert_array_equal(lines[0]["codes"][~sens], ref["code"][~sens])
    np.testing.assert_array_equal(lines[0]["steps"][~sens], ref["steps"][~sens])


def test_automatic_layout_choice(S):
    """AUTO stores a steady FP32 block as cell records (96 B per cell), and 16-bit or
    time-sliced fields as node rows (12 B per FP32 node, 8 B per padded 16-bit node)."""
    note("automatic layout")
    blk = fg.turbulence_block(2, dims=(10, 12, 14))
    f = S.Field([blk], fg.F32)
    assert S.streami_field_info(f.h) == (S.LAYOUT_CELL, 11 * 13 * 15 * 96)
    f.close()
    blk16 = fg.turbulence_block(2, dims=(10, 12, 14), fmt=fg.F16)
    f = S.Field([blk16], fg.F16)
    assert S.streami_field_info(f.h) == (S.LAYOUT_LINEAR, 12 * 14 * 16 * 8)
    f.close()
    blkt = fg.turbulence_block(2, dims=(10, 12, 14), n_slices=3, slice_dt=5.0)
    f = S.Field([blkt], fg.F32)
    assert S.streami_field_info(f.h) == (S.LAYOUT_LINEAR, 3 * 12 * 14 * 16 * 12)
    f.close()


def test_device_inputs_match_host_inputs(S):
    """Seeds, ids, step limits and birth times given as device tensors (step limits reduced
    on the device to size the log) give the same lines and outbox as host arrays, over
    several seed calls into several blocks; a negative device step limit is rejected."""
    import torch
    note("device seed inputs")
    blocks = [fg.turbulence_block(4, dims=d, fmt=fg.F16, sub=b, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
              for b, d in enumerate([(20, 24, 16), (16, 28, 20)])]
    rng = np.random.default_rng(41)
    calls = []
    for c in range(5):
        b = c % 2
        n = int(rng.integers(1, 900))
        calls.append((b, fg.uniform_seeds(4, n, (0, 0, 0), blocks[b].dims, sub=50 + c),
                      rng.integers(0, 300, size=n).astype(np.int32), 3 if c == 3 else 1))
    outs = []
    for on_dev in (False, True):
        f = S.Field(blocks, fg.F16)
        for b, sd, ms, stride in calls:
            if on_dev:
                f.seed(b, torch.from_numpy(sd).cuda(), max_steps=torch.from_numpy(ms).cuda(), record_stride=stride)
            else:
                f.seed(b, sd, max_steps=ms, record_stride=stride)
        f.advect(0.5)
        outs.append(([f.lines(b) for b in range(2)], np.sort(f.outbox(), order=["block", "id"])))
        if on_dev:
            bad = torch.tensor([5, -1, 7], dtype=torch.int32, device="cuda")
            with pytest.raises(S.StreamiError, match="negative"):
                f.seed(0, torch.zeros(3, 3, device="cuda"), max_steps=bad)
        f.close()
    for b in range(2):
        for k in ("offsets", "xyz", "steps", "codes", "ids"):
            np.testing.assert_array_equal(outs[1][0][b][k], outs[0][0][b][k])
    np.testing.assert_array_equal(outs[1][1], outs[0][1])


def _streak_inputs():
    blk = fg.turbulence_block(6, edge=24, fmt=fg.F16, n_slices=4, slice_dt=40.0,
                              rank_grid=(1, 1, 1), rank_coord=(0, 0, 0), sub=1)
    emitters = fg.uniform_seeds(6, 60, (0, 0, 0), (24, 24, 24), sub=31)
    limits = np.random.default_rng(31).integers(40, 240, size=60)
    pos, tb, lim, _ = fg.streakline_particles(emitters, limits, 10, 0.5)
    return blk, pos, tb, lim


def test_streaklines_parity(S):
    """Streakline particles (60 emitters, one particle every 10 steps, each with its own
    birth time) in a 4-slice FP16 block: local check at each vertex's own time against the
    oracle, discrete results exact away from the boundary."""
    note("streaklines")
    blk, pos, tb, lim = _streak_inputs()
    f = S.Field([blk], fg.F16)
    f.seed(0, pos, max_steps=lim, t_births=tb)
    f.advect(0.5)
    L = f.lines(0)
    f.close()
    F = orc_field(blk)
    ratio, npairs = parity.local_check(F, L, 0.5, 24.0, t_birth=tb)
    assert ratio <= 1.0 and npairs > 0.5 * lim.sum(), (ratio, npairs)
    ref = F.trace(pos, 0.5, lim, t_birth=tb)
    dev, same = parity.global_compare(L, ref, len(pos))
    sens = parity.boundary_sensitive(ref, L, dev, blk.lo, blk.hi, field=F)
    assert (~sens).mean() > 0.8
    np.testing.assert_array_equal(L["codes"][~sens], ref["code"][~sens])
    np.testing.assert_array_equal(L["steps"][~sens], ref["steps"][~sens])


@pytest.mark.parametrize("work_order", [0, 1])
def test_time_windows_bit_identical(S, work_order):
    """Advancing the streakline particles in time windows (t_end = 18.5, 37, ...) gives the
    lines, steps, codes and outbox of one unbounded call, bit for bit; after the first
    window every particle still ACTIVE stands at its first step time >= t_end."""
    note("time windows, work order", work_order)
    blk, pos, tb, lim = _streak_inputs()
    h = 0.5
    base = run(S, [blk], [pos], h, [lim], fg.F16, t_births=tb, work_order=work_order)
    f = S.Field([blk], fg.F16)
    f.seed(0, pos, max_steps=lim, t_births=tb)
    W = 37 * h
    t_end = W
    st = f.advect(h, t_end=t_end, work_order=work_order)
    L1 = f.lines(0)
    act = L1["codes"] == S.ACTIVE
    assert act.any() and (~act).any()
    n = L1["steps"][act].astype(np.float64)
    t_next = tb[act].astype(np.float64) + n * h  # exact: multiples of 0.5
    assert (t_next >= t_end).all()
    assert ((n == 0) | (t_next - h < t_end)).all()
    for _ in range(100):
        if st.active == 0:
            break
        t_end += W
        st = f.advect(h, t_end=t_end, work_order=work_order)
    assert st.active == 0
    got = f.lines(0)
    ob = f.outbox()
    f.close()
    for k in ("offsets", "xyz", "steps", "codes", "ids"):
        np.testing.assert_array_equal(got[k], base[1][0][k])
    np.testing.assert_array_equal(np.sort(ob, order="id"), np.sort(base[2], order="id"))


# ---------------------------------------------------------------- full size (config 2)
def test_turbulence_256_full_size_sampled(S):
    """The benchmark's workload and launch: 256^3 FP32 block + ghost, 1M uniform seeds,
    h=0.5, up to 2000 steps, rank grid 4^3.  Sampled outputs (a contiguous 4096-particle
    range of the iid seed set) against the oracle; counts and invariants on all."""
    note("turbulence 256^3 x 1M full size")
    blk = fg.turbulence_block(2, edge=256)
    seeds = fg.uniform_seeds(2, 1 << 20, (0, 0, 0), (256, 256, 256))
    f = S.Field([blk], fg.F32)
    f.seed(0, seeds, default_max_steps=2000)
    st = f.advect(0.5)
    first, count = 123456, 4096
    L = f.lines(0, first, count)
    F = orc_field(blk)
    ratio, _ = parity.local_check(F, L, 0.5, 256.0)
    assert ratio <= 1.0, ratio
    ref = F.trace(seeds[first:first + count], 0.5, 2000)
    dev, same = parity.global_compare(L, ref, count)
    sens = parity.boundary_sensitive(ref, L, dev, blk.lo, blk.hi, field=F)
    np.testing.assert_array_equal(L["codes"][~sens], ref["code"][~sens])
    np.testing.assert_array_equal(L["steps"][~sens], ref["steps"][~sens])
    within = (dev <= 1e-4 * 256).mean()
    frac, bad = parity.restart_check(F, L, 0.5, blk.lo, blk.hi, 2000)
    note(f"full-size: {within:.3f} of sampled lines within 1e-4 extent; whole-line comparison covers "
         f"{(~sens).mean():.3f}, late restart {frac:.4f}; median dev {np.median(dev):.2e} max {dev.max():.2e}")
    # the whole-trajectory comparison must cover a real share of the sample, and the late
    # restart (the oracle resumed from the GPU's vertex 16 steps before the end) nearly all of it
    assert (~sens).mean() >= 0.5, (~sens).mean()
    assert frac >= 0.97 and len(bad) == 0, (frac, bad[:10])
    # invariants over the whole set: every particle terminated, ids conserved
    assert st.active == 0 and sum(st.terminated) == 1 << 20
    ob = f.outbox(cap=1 << 21)
    assert len(ob) == st.terminated[S.EXIT] + st.terminated[S.HALO_MISS]
    assert len(np.unique(ob["id"])) == len(ob)
    assert st.terminated[S.HALO_MISS] == 0  # max |v| = 1 cell, h = 0.5: stages never leave the halo
    # outbox positions lie within h*vmax of the owned bounds, destinations are neighbours
    out = np.maximum(np.maximum(-ob["pos"], ob["pos"] - 256), 0).max(axis=1)
    assert out.max() <= 0.5 + 1e-4
    assert (ob["dest"] >= 0).all() and (ob["dest"] != 1 + 4 * (1 + 4 * 1)).all()


@pytest.mark.parametrize("dtype", [fg.BF16, fg.F16])
def test_turbulence_512_16bit_full_size_sampled(S, dtype):
    """The 16-bit workload and launch as benchmarked: 512^3 block + ghost stored in BF16/FP16,
    4M seeds in 64 Gaussian blobs, h=0.5, up to 4000 steps, every 8th vertex kept.  Sampled
    outputs (4 x 512 particles from 4 blobs) against the oracle on the same stored nodes; the
    per-step rule on 512 blob seeds recorded at stride 1; counts and invariants on all."""
    note("turbulence 512^3 x 4M full size", fg.DTYPE_NAMES[dtype])
    blk = fg.turbulence_block(3, edge=512, fmt=dtype)
    seeds = fg.blob_seeds(3, 64, 65536, 512.0, 24.0, 8.0)
    f = S.Field([blk], dtype)
    f.seed(0, seeds, default_max_steps=4000, record_stride=8)
    st = f.advect(0.5)
    F = orc_field(blk)
    for b in (0, 21, 42, 63):
        first, count = b * 65536 + 1000, 512
        L = f.lines(0, first, count)
        ref = F.trace(seeds[first:first + count], 0.5, 4000, stride=8)
        dev, same = parity.global_compare(L, ref, count)
        sens = parity.boundary_sensitive(ref, L, dev, blk.lo, blk.hi, field=F)
        # chaotic 4000-step lines: FP32 vs FP64 deviation grows, and with it the margin of
        # boundary sensitivity; the whole-line comparison must still cover 40% of the sample
        # (0.51-0.69 measured), the late restart below nearly all of it
        assert (~sens).mean() >= 0.4, (~sens).mean()
        np.testing.assert_array_equal(L["codes"][~sens], ref["code"][~sens])
        np.testing.assert_array_equal(L["steps"][~sens], ref["steps"][~sens])
        frac, bad = parity.restart_check(F, L, 0.5, blk.lo, blk.hi, 4000, stride=8)
        note(f"blob {b}: {(dev <= 2e-3 * 512).mean():.3f} within 2e-3 extent, whole-line comparison covers "
             f"{(~sens).mean():.3f}, late restart {frac:.4f}")
        assert frac >= 0.97 and len(bad) == 0, (b, frac, bad[:10])
    assert st.active == 0 and sum(st.terminated) == len(seeds)
    ob = f.outbox(cap=len(seeds))
    assert len(ob) == st.terminated[S.EXIT] + st.terminated[S.HALO_MISS] and st.terminated[S.HALO_MISS] == 0
    assert len(np.unique(ob["id"])) == len(ob)
    f.close()
    # the per-step rule needs consecutive vertices: a stride-1 run of 512 blob seeds
    g = S.Field([blk], dtype)
    sub = seeds[7 * 65536:7 * 65536 + 512]
    g.seed(0, sub, default_max_steps=4000)
    g.advect(0.5)
    ratio, npairs = parity.local_check(F, g.lines(0), 0.5, 512.0)
    assert ratio <= 1.0 and npairs > 512 * 100, (ratio, npairs)
    g.close()


def test_batched96_full_size_sampled(S):
    """The batched workload and launch as benchmarked: 96 FP16 blocks of uneven shape, 1.33M
    seeds with per-seed limits, one graph-captured persistent launch.  Sampled outputs (256
    particles of each of 6 blocks) against the oracle run on that block alone; counts and
    invariants on all."""
    import torch
    note("batched 96 blocks full size")
    blocks, seeds, limits = fg.batched_blocks(n_blocks=96, fmt=fg.F16)
    f = S.Field(blocks, fg.F16)
    for b in range(96):
        f.seed(b, torch.from_numpy(seeds[b]).cuda(), max_steps=torch.from_numpy(limits[b]).cuda())
    st = f.advect(0.5, use_graph=1)
    n = sum(len(s) for s in seeds)
    assert st.active == 0 and sum(st.terminated) == n
    for b in (0, 17, 35, 52, 70, 95):
        k = min(256, len(seeds[b]))
        L = f.lines(b, 0, k)
        F = orc_field(blocks[b])
        ratio, _ = parity.local_check(F, L, 0.5, blocks[b].extent)
        assert ratio <= 1.0, (b, ratio)
        ref = F.trace(seeds[b][:k], 0.5, limits[b][:k])
        dev, same = parity.global_compare(L, ref, k)
        sens = parity.boundary_sensitive(ref, L, dev, blocks[b].lo, blocks[b].hi, field=F)
        np.testing.assert_array_equal(L["codes"][~sens], ref["code"][~sens])
        np.testing.assert_array_equal(L["steps"][~sens], ref["steps"][~sens])
        frac, bad = parity.restart_check(F, L, 0.5, blocks[b].lo, blocks[b].hi, limits[b][:k])
        note(f"block {b}: whole-line comparison covers {(~sens).mean():.3f}, late restart {frac:.4f}")
        assert (~sens).mean() >= 0.5, (b, (~sens).mean())
        assert frac >= 0.97 and len(bad) == 0, (b, frac, bad[:10])
    ob = f.outbox(cap=n)
    assert len(ob) == st.terminated[S.EXIT] + st.terminated[S.HALO_MISS]
    assert set(np.unique(ob["block"])) <= set(range(96))
    assert len(np.unique(ob["id"])) == len(ob)
    f.close()


def test_streaklines96_full_size_sampled(S):
    """The unsteady batched workload and launch as benchmarked: 96 FP16 blocks x 16 time slices
    of the 512-mode generator (phases drifting linearly), every seed a streakline emitter that
    releases a particle every 10 steps until its step limit (about 3.4e8 particles, each with
    its birth time and remaining limit), one graph-captured persistent launch, seed and last
    vertex kept.  From 6 blocks, 64 particles each are seeded in a batch of their own with
    every vertex kept: their vertices pass the per-step rule at their own times, and their
    codes and step counts equal the oracle's (whole trajectory away from the bounds, and from a
    late restart).  Counts and invariants over all particles."""
    import dataclasses
    import torch
    from fieldgen import device as fgd
    note("streaklines 96 blocks x 16 slices full size: generating")
    blocks, nodes, emitters, elim = fgd.batched_blocks(n_blocks=96, fmt=fg.F16, n_slices=16, n_modes=512)
    parts = [fgd.streakline_particles(torch.from_numpy(e).cuda(), torch.from_numpy(m).cuda(), 10, 0.5)
             for e, m in zip(emitters, elim)]
    n_all = sum(int(p[0].shape[0]) for p in parts)
    sample_blocks = (3, 20, 38, 55, 71, 90)
    bulk, samp = [], {}
    for b, (pos, tb, lim, _) in enumerate(parts):
        if b in sample_blocks:
            n = pos.shape[0]
            idx = torch.unique(torch.linspace(0, n - 1, 64, device="cuda").round().long())
            keep = torch.ones(n, dtype=torch.bool, device="cuda")
            keep[idx] = False
            bulk.append(dict(block=b, xyz=pos[keep].contiguous(), max_steps=lim[keep].contiguous(),
                             t_births=tb[keep].contiguous()))
            samp[b] = dict(block=b, xyz=pos[idx].contiguous(), max_steps=lim[idx].contiguous(),
                           t_births=tb[idx].contiguous(), n_bulk=int(keep.sum()))
        else:
            bulk.append(dict(block=b, xyz=pos, max_steps=lim, t_births=tb))
    note(f"streaklines: {n_all} particles; advecting")
    f = S.Field(blocks, fg.F16, nodes=nodes)
    f.seed_batches(bulk, record_stride=1 << 20)
    f.seed_batches([{k: v for k, v in d.items() if k != "n_bulk"} for d in samp.values()], record_stride=1)
    st = f.advect(0.5, use_graph=1)
    assert st.active == 0 and sum(st.terminated) == n_all
    assert st.terminated[S.HALO_MISS] == 0
    for b in sample_blocks:
        d = samp[b]
        k = int(d["xyz"].shape[0])
        L = f.lines(b, d["n_bulk"], k)
        blk = dataclasses.replace(blocks[b])
        blk.stored = nodes[b].cpu().numpy().view(np.uint16)
        F = orc_field(blk)
        xyz, lim, tb = (d[key].cpu().numpy() for key in ("xyz", "max_steps", "t_births"))
        np.testing.assert_array_equal(L["xyz"][L["offsets"][:-1]], xyz)  # the sampled particles, in order
        ratio, npairs = parity.local_check(F, L, 0.5, blk.extent, t_birth=tb)
        assert ratio <= 1.0 and npairs >= k, (b, ratio, npairs)
        ref = F.trace(xyz, 0.5, lim, t_birth=tb)
        dev, same = parity.global_compare(L, ref, k)
        sens = parity.boundary_sensitive(ref, L, dev, blk.lo, blk.hi, field=F)
        np.testing.assert_array_equal(L["codes"][~sens], ref["code"][~sens])
        np.testing.assert_array_equal(L["steps"][~sens], ref["steps"][~sens])
        frac, bad = parity.restart_check(F, L, 0.5, blk.lo, blk.hi, lim, t_birth=tb)
        note(f"block {b}: {k} particles, {npairs} steps checked; whole-line comparison covers "
             f"{(~sens).mean():.3f}, late restart {frac:.4f}")
        assert (~sens).mean() >= 0.5 and frac >= 0.95 and len(bad) == 0, (b, (~sens).mean(), frac, bad[:10])
    # the outbox (one 32-byte record per exit) fetched into device memory: ids unique
    buf = torch.empty((n_all, 4), dtype=torch.int64, device="cuda")
    rc, n_out = S.streami_fetch_outbox(f.h, buf, n_all)
    assert rc == S.OK and n_out == st.terminated[S.EXIT]
    assert torch.unique(buf[:n_out, 0]).numel() == n_out
    f.close()


def test_argument_errors_on_a_live_handle(S):
    """Errors are reported as codes with a message and leave the handle usable: advect before
    seeding, a NaN window end, an out-of-range launch shape, a window in surrogate mode,
    negative step limits; an empty seed batch is a no-op."""
    note("argument errors")
    blk = fg.turbulence_block(2, edge=16, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
    f = S.Field([blk], fg.F32)
    with pytest.raises(S.StreamiError) as e:
        f.advect(0.5)
    assert e.value.code == S.E_STATE
    f.seed(0, np.zeros((0, 3), np.float32), default_max_steps=10)
    with pytest.raises(S.StreamiError) as e:
        f.seed(0, np.ones((2, 3), np.float32), max_steps=np.array([3, -1], np.int32))
    assert e.value.code == S.E_ARG and "max_steps" in str(e.value)
    seeds = fg.uniform_seeds(2, 300, (0, 0, 0), (16, 16, 16))
    f.seed(0, seeds, default_max_steps=50)
    for kw, code in ((dict(t_end=float("nan")), S.E_ARG), (dict(waves_per_cu=65), S.E_ARG),
                     (dict(refill_threshold=-1), S.E_ARG), (dict(work_order=2), S.E_ARG),
                     (dict(mode=S.MODE_SURROGATE, t_end=1.0), S.E_UNSUPPORTED)):
        with pytest.raises(S.StreamiError) as e:
            f.advect(0.5, **kw)
        assert e.value.code == code, (kw, e.value)
    with pytest.raises(S.StreamiError) as e:
        f.advect(float("inf"))
    assert e.value.code == S.E_ARG
    st = f.advect(0.5)  # still usable after every refusal
    assert st.active == 0 and st.steps == int(f.lines(0)["steps"].sum()) > 0
    f.close()
