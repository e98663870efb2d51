"""GPU tests of the unstructured field: streami_field_create_hex.

Voxel hexahedra (every cell of a structured grid) sample what the structured grid samples
(pinned on the CPU for the two oracles), so their lines are checked against the structured
FP64 oracle, which runs fast; general (jittered) hexahedra, and tetrahedra, wedges and
pyramids (jittered cubes split into conforming cells), against the unstructured oracle.
Per-step rule at every vertex; step counts and codes from a late restart; exits, halo misses
and destinations from the outbox."""
import sys

import numpy as np
import pytest

import fieldgen as fg
import oracle
from oracle import hex as ohex
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


def hex_oracle(mesh):
    return ohex.HexField(mesh["vertices"], mesh["values"], mesh["cells"], mesh["lo"], mesh["hi"],
                         mesh["rank_grid"], mesh["rank_coord"], cell_types=mesh.get("cell_types"))


def test_voxel_hexahedra_follow_the_structured_field(S):
    note("hex: voxel hexahedra of a 24^3 block")
    blk = fg.turbulence_block(15, edge=24, rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    mesh = fg.hex_mesh_from_block(blk)
    F = oracle.Field.from_block(blk)
    seeds = fg.uniform_seeds(15, 3000, (0, 0, 0), (24, 24, 24))
    f = S.Field.hex(mesh)
    assert S.streami_field_info(f.h)[0] == S.LAYOUT_HEX
    f.seed(0, seeds, default_max_steps=300)
    st = f.advect(0.5)
    L = f.lines(0)
    ratio, npairs = parity.local_check(F, L, 0.5, 24.0)
    assert ratio <= 1.0 and npairs > 3000 * 20, (ratio, npairs)
    frac, bad = parity.restart_check(F, L, 0.5, blk.lo, blk.hi, 300)
    ref = F.trace(seeds, 0.5, 300)
    dev, _ = parity.global_compare(L, ref, len(seeds))
    sens = parity.boundary_sensitive(ref, L, dev, blk.lo, blk.hi, field=F)
    note(f"hex voxels: {npairs} steps, local ratio {ratio:.3f}, restart compares {frac:.4f}, whole lines "
         f"{(~sens).mean():.3f}, {st.gathers / max(1, st.steps):.3f} BVH walks per step")
    assert frac >= 0.97 and len(bad) == 0, (frac, bad[:10])
    np.testing.assert_array_equal(L["codes"][~sens], ref["code"][~sens])
    # exits go to the outbox with the structured field's destinations
    ob = f.outbox(cap=len(seeds))
    assert len(ob) == st.terminated[S.EXIT] + st.terminated[S.HALO_MISS] and st.terminated[S.HALO_MISS] == 0
    np.testing.assert_array_equal(ob["dest"], F.dest(ob["pos"].astype(np.float64)))
    f.close()


def test_general_hexahedra_against_the_hex_oracle(S):
    """Jittered (non-affine) cells; owned bounds one cell inside the mesh, so particles exit
    through the owned faces and halo misses happen where a step reaches the mesh's edge."""
    note("hex: jittered mesh")
    mesh = fg.distorted_hex_mesh(16, (14, 12, 10), jitter=0.25)
    mesh.update(lo=(1.0, 1.0, 1.0), hi=(13.0, 11.0, 9.0), rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    H = hex_oracle(mesh)
    seeds = fg.uniform_seeds(16, 400, (1, 1, 1), (13, 11, 9), sub=2)
    f = S.Field.hex(mesh)
    f.seed(0, seeds, default_max_steps=300)
    st = f.advect(0.25)
    L = f.lines(0)
    ratio, npairs = parity.local_check(H, L, 0.25, 14.0)
    assert ratio <= 1.0 and npairs > 400 * 20, (ratio, npairs)
    frac, bad = parity.restart_check(H, L, 0.25, mesh["lo"], mesh["hi"], 300)
    note(f"hex jittered: {npairs} steps, local ratio {ratio:.3f}, restart compares {frac:.4f}; codes "
         f"{np.bincount(L['codes'], minlength=6).tolist()}")
    assert frac >= 0.95 and len(bad) == 0, (frac, bad[:10])
    assert st.terminated[S.EXIT] > 20
    ob = f.outbox(cap=len(seeds))
    assert len(ob) == st.terminated[S.EXIT] + st.terminated[S.HALO_MISS]
    ex = ob["code"] == S.EXIT
    np.testing.assert_array_equal(ob["dest"][ex], H.dest(ob["pos"][ex].astype(np.float64)))
    f.close()
    # a mesh without halo: steps that reach its edge miss, at the old position (outbox, steps unchanged)
    m2 = dict(mesh, lo=(0.0, 0.0, 0.0), hi=(14.0, 12.0, 10.0))
    H2 = hex_oracle(m2)
    s2 = fg.uniform_seeds(16, 300, (0, 0, 0), (14, 12, 10), sub=3)
    g = S.Field.hex(m2)
    g.seed(0, s2, default_max_steps=120)
    st2 = g.advect(0.6)
    L2 = g.lines(0)
    frac, bad = parity.restart_check(H2, L2, 0.6, m2["lo"], m2["hi"], 120)
    assert st2.terminated[S.HALO_MISS] > 10 and frac >= 0.9 and len(bad) == 0, (st2.terminated, frac, bad)
    g.close()


@pytest.mark.parametrize("kind", ["tetra", "wedge", "pyramid", "hex+pyramid"])
def test_split_cells_against_the_unstructured_oracle(S, kind):
    """Tetrahedra, wedges, pyramids and a hexahedron/pyramid checkerboard (6 x 6 x 5 jittered
    cubes split into conforming cells, owned bounds one cube inside): per-step rule at every
    vertex, late-restart codes and steps, exits with their destinations; neighbour hops and the
    BVH walk both run (a walk per step is far rarer than a cell change).  A fifth of the seeds
    start within 0.06 of a lattice vertex, where Newton from a warped cell's centre can end at
    the map's second root: no stage point inside the mesh goes unfound (no halo miss)."""
    note("unstructured:", kind)
    mesh = fg.split_hex_mesh(fg.distorted_hex_mesh(21, (6, 6, 5), jitter=0.2, sub=len(kind)), kind)
    mesh.update(lo=(1.0, 1.0, 1.0), hi=(5.0, 5.0, 4.0), rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    H = hex_oracle(mesh)
    k, j, i = np.meshgrid(np.arange(2, 4), np.arange(2, 5), np.arange(2, 5), indexing="ij")
    near = np.repeat(mesh["vertices"][(i + 7 * (j + 7 * k)).ravel()], 3, 0).astype(np.float64)
    near += np.random.default_rng(len(kind)).uniform(-0.06, 0.06, near.shape)
    seeds = np.concatenate([fg.uniform_seeds(21, 196, (1, 1, 1), (5, 5, 4), sub=len(kind)),
                            near.astype(np.float32)])
    assert len(seeds) == 250
    f = S.Field.hex(mesh)
    f.seed(0, seeds, default_max_steps=200)
    st = f.advect(0.08)
    L = f.lines(0)
    ratio, npairs = parity.local_check(H, L, 0.08, 6.0)
    frac, bad = parity.restart_check(H, L, 0.08, mesh["lo"], mesh["hi"], 200)
    note(f"{kind}: {len(mesh['cells'])} cells, {npairs} steps, local ratio {ratio:.3f}, restart compares "
         f"{frac:.4f}, {st.gathers / max(1, st.steps):.4f} BVH walks per step; codes "
         f"{np.bincount(L['codes'], minlength=6).tolist()}")
    assert ratio <= 1.0 and npairs > 250 * 15, (ratio, npairs)
    assert frac >= 0.95 and len(bad) == 0, (frac, bad[:10])
    assert st.active == 0 and st.terminated[S.EXIT] > 20 and st.terminated[S.HALO_MISS] == 0
    assert 0 < st.gathers < 0.1 * st.steps
    ob = f.outbox(cap=len(seeds))
    assert len(ob) == st.terminated[S.EXIT] + st.terminated[S.HALO_MISS]
    ex = ob["code"] == S.EXIT
    np.testing.assert_array_equal(ob["dest"][ex], H.dest(ob["pos"][ex].astype(np.float64)))
    f.close()


def test_hex_refusals(S):
    note("hex: refusals")
    mesh = fg.distorted_hex_mesh(17, (3, 3, 3), jitter=0.1)
    f = S.Field.hex(mesh)
    f.seed(0, fg.uniform_seeds(17, 10, (0, 0, 0), (3, 3, 3)), default_max_steps=5)
    with pytest.raises(S.StreamiError) as e:
        f.advect(0.01, mode=S.MODE_SURROGATE, residual_tol_cells=1.0)
    assert e.value.code in (S.E_UNSUPPORTED, S.E_STATE)
    st = f.advect(0.3)
    assert st.active == 0
    f.close()
    # an unknown cell type (VTK_QUAD) is refused, naming the cell
    types = np.full(len(mesh["cells"]), 12, np.uint8)
    types[5] = 9
    with pytest.raises(S.StreamiError) as e:
        S.Field.hex(dict(mesh, cell_types=types))
    assert e.value.code == S.E_ARG and "cell 5" in str(e.value)


def test_hex256_full_size_sampled(S):
    """The hexahedral workload as benchmarked: the 256^3 block's 16,974,593 cells, the 1M seeds
    and 2000-step limits of the structured workload.  A contiguous 4096-particle sample against
    the structured FP64 oracle (equal to the hexahedral oracle on voxel cells): per-step rule at
    every vertex and late-restart codes and steps; invariants over all particles."""
    note("hex 256^3 full size: building")
    blk = fg.turbulence_block(2, edge=256)
    seeds = fg.uniform_seeds(2, 1 << 20, (0, 0, 0), (256, 256, 256))
    f = S.Field.hex(fg.hex_mesh_from_block(blk))
    f.seed(0, seeds, default_max_steps=2000)
    note("hex 256^3 full size: advecting")
    st = f.advect(0.5)
    first, count = 123456, 4096
    L = f.lines(0, first, count)
    F = oracle.Field.from_block(blk)
    ratio, npairs = parity.local_check(F, L, 0.5, 256.0)
    frac, bad = parity.restart_check(F, L, 0.5, blk.lo, blk.hi, 2000)
    note(f"hex 256^3: {st.steps} steps, {st.gathers / st.steps:.4f} BVH walks per step; sample: {npairs} steps, "
         f"local ratio {ratio:.3f}, restart compares {frac:.4f}")
    assert ratio <= 1.0 and npairs > count * 100, (ratio, npairs)
    assert frac >= 0.97 and len(bad) == 0, (frac, bad[:10])
    assert st.active == 0 and sum(st.terminated) == 1 << 20 and st.terminated[S.HALO_MISS] == 0
    ob = f.outbox(cap=1 << 21)
    assert len(ob) == st.terminated[S.EXIT] and len(np.unique(ob["id"])) == len(ob)
    f.close()
