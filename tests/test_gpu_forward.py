"""Loopback forwarding (the exchange of outgoing particles between macrocells, Sec. 3.1.2 and
the step() listing of Sec. 3.2) on one GPU: one turbulence field split into a 2 x 2 x 2 rank
grid of blocks in one handle, every exit routed on the device into the block that owns the new
position, repeated until no particle is active.

The stitched lines (each id's segments in step order, joined at their shared exit vertex) are
checked against the FP64 oracle tracing the whole, unsplit field: every vertex passes the local
one-step rule, and step counts and termination codes are exact for particles whose end is not
boundary-sensitive.  The exchange granularity (one step per round, k steps, or run-to-exit) does
not change any line, bit for bit.
"""
import sys

import numpy as np
import pytest

import fieldgen as fg
import oracle
from tests.parity import boundary_sensitive, global_compare, local_check, restart_check

pytestmark = pytest.mark.gpu

H = 0.5
EDGE = 64
M = 600


def note(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    import paper_2606_02627_amd as S
    S._load()
    return S


@pytest.fixture(scope="module")
def field():
    whole = fg.turbulence_block(2, edge=EDGE, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
    parts = fg.partition(whole, (2, 2, 2))
    seeds = fg.uniform_seeds(2, 3000, (0, 0, 0), (EDGE,) * 3, sub=40)
    owner = (np.floor(seeds / (EDGE // 2)).astype(int) * np.array([1, 2, 4])).sum(axis=1)
    return whole, parts, seeds, owner


def _stitch(S, f, n_blocks):
    """Segments of every id, stitched in step order: {id: (vertices, steps, code, segments)}."""
    segs = {}
    for b in range(n_blocks):
        L = f.lines(b)
        off = L["offsets"]
        for i, pid in enumerate(L["ids"]):
            v = L["xyz"][off[i]:off[i + 1]]
            first = int(L["steps"][i]) - (len(v) - 1)
            segs.setdefault(int(pid), []).append((first, v, int(L["steps"][i]), int(L["codes"][i]), b))
    out = {}
    for pid, ss in segs.items():
        ss.sort(key=lambda s: s[0])
        assert ss[0][0] == 0, (pid, [s[0] for s in ss])
        verts = [ss[0][1]]
        for a, c in zip(ss[:-1], ss[1:]):
            assert a[3] == S.EXIT, (pid, a[3])             # only an exit hands a particle on
            assert c[0] == a[2], (pid, a[2], c[0])          # the next segment continues its step count
            np.testing.assert_array_equal(c[1][0], a[1][-1])  # ... from the shared joint vertex
            assert c[4] != a[4]
            verts.append(c[1][1:])
        out[pid] = (np.concatenate(verts), ss[-1][2], ss[-1][3], len(ss))
    return out


def _run(S, parts, seeds, owner, layout=0, fmt=None, **kw):
    fmt = S.F32 if fmt is None else fmt
    f = S.Field(parts if fmt == S.F32 else [p.quantise(fmt) for p in parts], fmt, layout=layout)
    f.seed_batches([dict(block=b, xyz=np.ascontiguousarray(seeds[owner == b]),
                         ids=np.nonzero(owner == b)[0].astype(np.uint64)) for b in range(8)],
                   default_max_steps=M)
    rounds, st = f.trace(H, **kw)
    lines = _stitch(S, f, 8)
    ob = f.outbox(cap=len(seeds))
    f.close()
    return rounds, st, lines, ob


def test_forwarded_lines_match_whole_field_oracle(S, field):
    whole, parts, seeds, owner = field
    note("forwarding: 2x2x2 blocks of a 64^3 field, 3000 seeds")
    rounds, st, lines, ob = _run(S, parts, seeds, owner)
    n = len(seeds)
    assert st.active == 0 and sorted(lines) == list(range(n))
    multi = np.array([lines[i][3] for i in range(n)])
    note(f"{rounds} rounds, {st.steps} steps, segments per line: max {multi.max()}, "
         f"{(multi > 1).mean():.2f} of the lines cross a block face")
    assert (multi > 1).mean() > 0.3
    # every record left in the outbox leaves the whole field (no block owns its macrocell)
    assert (ob["dest"] == -1).all() and (ob["code"] == S.EXIT).all()
    ended_exit = np.array([lines[i][2] == S.EXIT for i in range(n)])
    assert sorted(ob["id"].tolist()) == np.nonzero(ended_exit)[0].tolist()
    # the oracle on the unsplit field
    W = oracle.Field.from_block(whole)
    ref = W.trace(seeds, float(np.float32(H)), M)
    xyz = [lines[i][0] for i in range(n)]
    L = dict(offsets=np.concatenate([[0], np.cumsum([len(v) for v in xyz])]), xyz=np.concatenate(xyz))
    worst, cnt = local_check(W, L, H, EDGE)
    note(f"local rule: worst ratio {worst:.3f} over {cnt} steps")
    assert worst <= 1.0 and cnt > 0.9 * st.steps
    steps = np.array([lines[i][1] for i in range(n)])
    codes = np.array([lines[i][2] for i in range(n)])
    dev, _ = global_compare(L, ref, n)
    sens = boundary_sensitive(ref, L, dev, whole.lo, whole.hi, field=W)
    note(f"non-sensitive {(~sens).mean():.3f}")
    assert (~sens).mean() > 0.5
    np.testing.assert_array_equal(steps[~sens], ref["steps"][~sens])
    np.testing.assert_array_equal(codes[~sens], ref["code"][~sens])


@pytest.mark.parametrize("budget", [1, 7])
def test_exchange_granularity_is_bit_identical(S, field, budget):
    """One exchange per step (the paper's step()) or per k steps gives the same lines as
    running the local particles to their exit before each exchange."""
    whole, parts, seeds, owner = field
    seeds, owner = seeds[:400], owner[:400]
    note(f"forwarding: exchange every {budget} steps")
    r0, st0, l0, _ = _run(S, parts, seeds, owner)
    rk, stk, lk, _ = _run(S, parts, seeds, owner, step_budget=budget)
    assert rk > r0 and stk.steps == st0.steps
    for i in range(len(seeds)):
        np.testing.assert_array_equal(lk[i][0], l0[i][0])
        assert lk[i][1:] == l0[i][1:]


def test_forwarding_on_node_rows_and_16bit(S, field):
    """The same exchange on node rows (FP32) and FP16 nodes: ids conserved, joints shared,
    codes and steps of the FP32 rows equal the cell records' (bit-identical layouts)."""
    whole, parts, seeds, owner = field
    seeds, owner = seeds[:600], owner[:600]
    note("forwarding: layouts and formats")
    _, st_c, lc, _ = _run(S, parts, seeds, owner, layout=S.LAYOUT_CELL)
    _, st_r, lr, _ = _run(S, parts, seeds, owner, layout=S.LAYOUT_LINEAR)
    for i in range(len(seeds)):
        np.testing.assert_array_equal(lr[i][0], lc[i][0])
    _, st_h, lh, ob = _run(S, parts, seeds, owner, fmt=S.F16)
    assert st_h.active == 0 and sorted(lh) == list(range(len(seeds)))


def test_forward_without_a_common_rank_grid_is_refused(S):
    blocks, _, _ = fg.batched_blocks(n_blocks=2, fmt=fg.F16, edge_lo=8, edge_hi=8)
    f = S.Field(blocks, S.F16)  # both blocks claim macrocell (0,0,0) of a 1x1x1 grid
    with pytest.raises(S.StreamiError) as e:
        f.forward()
    assert e.value.code == S.E_UNSUPPORTED
    f.close()


def test_forward256_full_size_sampled(S):
    """The forwarding workload as benchmarked: the 256^3 field split into 2 x 2 x 2 blocks of 128^3
    in one handle, 1M seeds each in the block that owns it, limits of 2000 steps, traced with
    run-to-exit rounds.  4096 sample seeds record every vertex (the rest their seed and last
    vertex of each segment, which forwarding preserves per particle); their stitched lines pass
    the per-step rule against the oracle of the whole, unsplit field, and their codes and step
    counts equal its late restarts.  Every id ends exactly once, in one block, after at most one
    segment per block visited."""
    import torch
    note("forwarding at full size: 2x2x2 blocks of 128^3, 1M seeds")
    edge, m = 256, 2000
    whole = fg.turbulence_block(2, edge=edge, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
    parts = fg.partition(whole, (2, 2, 2))
    seeds = fg.uniform_seeds(2, 1 << 20, (0, 0, 0), (edge,) * 3)
    owner = (np.floor(seeds / (edge // 2)).astype(int) * np.array([1, 2, 4])).sum(axis=1)
    sample = np.zeros(len(seeds), bool)
    sample[123456:123456 + 4096] = True
    f = S.Field(parts, S.F32)
    for stride, sel in ((1 << 20, ~sample), (1, sample)):
        f.seed_batches([dict(block=b, xyz=torch.from_numpy(np.ascontiguousarray(seeds[(owner == b) & sel])).cuda(),
                             ids=torch.from_numpy(np.nonzero((owner == b) & sel)[0].astype(np.uint64)).cuda())
                        for b in range(8)], default_max_steps=m, record_stride=stride)
    rounds, st = f.trace(H)
    assert st.active == 0
    # segments of every id, ordered by their step counts (any record stride): a segment that
    # hands the particle on ends with EXIT at the vertex the next one, in another block, starts
    segs = {}
    for b in range(8):
        Lb = f.lines(b)
        off = Lb["offsets"]
        for i, pid in enumerate(Lb["ids"].tolist()):
            segs.setdefault(pid, []).append((int(Lb["steps"][i]), Lb["xyz"][off[i]:off[i + 1]], int(Lb["codes"][i]), b))
    assert sorted(segs) == list(range(len(seeds)))
    lines = {}
    for pid, ss in segs.items():
        # chained by their joints: a particle that leaves exactly at its step limit is handed on
        # and ends at once in the next block, so step counts alone can tie
        ss.sort(key=lambda q: q[0])
        chain = [next((q for q in ss if np.array_equal(q[1][0], seeds[pid])), ss[0])]
        rest = [q for q in ss if q is not chain[0]]
        while rest:
            nxt = [q for q in rest if np.array_equal(q[1][0], chain[-1][1][-1]) and q[0] >= chain[-1][0]]
            if not nxt:
                break
            chain.append(nxt[0])
            rest = [q for q in rest if q is not nxt[0]]
        ok = not rest and np.array_equal(chain[0][1][0], seeds[pid])
        ss = chain
        for a, c in zip(ss[:-1], ss[1:]):
            ok = ok and a[2] in (S.EXIT, S.HALO_MISS) and c[3] != a[3] and np.array_equal(c[1][0], a[1][-1])
        if not ok:
            note(f"id {pid} seed {seeds[pid].tolist()} owner {owner[pid]}: segments (steps, code, block, first, last): "
                 + "; ".join(f"({q[0]}, {q[2]}, {q[3]}, {q[1][0].tolist()}, {q[1][-1].tolist()})" for q in ss))
            raise AssertionError(f"segments of id {pid} do not chain")
        if sample[pid]:
            lines[pid] = (np.concatenate([ss[0][1]] + [q[1][1:] for q in ss[1:]]), ss[-1][0], ss[-1][2], len(ss))
    ids = np.nonzero(sample)[0]
    note(f"{rounds} rounds, {st.steps} steps; checking {len(ids)} stitched lines")
    xyz = [lines[i][0] for i in ids]
    assert all(len(v) == lines[i][1] + 1 for v, i in zip(xyz, ids))  # stride 1: one vertex per step
    L = dict(offsets=np.concatenate([[0], np.cumsum([len(v) for v in xyz])]), xyz=np.concatenate(xyz),
             steps=np.array([lines[i][1] for i in ids], np.int32), codes=np.array([lines[i][2] for i in ids], np.int32))
    W = oracle.Field.from_block(whole)
    worst, cnt = local_check(W, L, H, edge)
    frac, bad = restart_check(W, L, H, whole.lo, whole.hi, m)
    segs = np.array([lines[i][3] for i in ids])
    note(f"local rule: worst ratio {worst:.3f} over {cnt} steps; late restart compares {frac:.4f}; "
         f"{(segs > 1).mean():.2f} of the sampled lines cross a block face (max {segs.max()} segments)")
    assert worst <= 1.0 and cnt > 4096 * 100
    assert frac >= 0.97 and len(bad) == 0, (frac, bad[:10])
    assert (segs > 1).mean() > 0.3
    ob = f.outbox(cap=len(seeds))
    assert (ob["dest"] == -1).all() and len(np.unique(ob["id"])) == len(ob)
    f.close()
