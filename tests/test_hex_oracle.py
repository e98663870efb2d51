"""Pins of the hexahedral-field oracle (oracle/hex.py), on the CPU.

  * voxel hexahedra: a mesh made of every cell of a structured block's grid samples exactly
    what the (separately pinned) structured oracle samples there, defined and undefined
    alike, and its RK4 trajectories (exits, step limits, halo misses, destinations) equal the
    structured oracle's;
  * affine cells (a sheared lattice) reproduce an affine field exactly, as trilinear
    interpolation must;
  * general cells (a jittered lattice): a point built from a cell's own parametric
    coordinates is located in that cell at those coordinates, and vertex values are
    reproduced at the vertices;
  * a plausible slip (a wrong VTK vertex order) is caught by these pins.
"""
import numpy as np
import pytest

import fieldgen as fg
import oracle
from oracle import hex as ohex


def hexfield(mesh):
    return ohex.HexField(mesh["vertices"], mesh["values"], mesh["cells"], mesh["lo"], mesh["hi"],
                         mesh["rank_grid"], mesh["rank_coord"])


@pytest.fixture(scope="module")
def voxels():
    blk = fg.turbulence_block(12, dims=(10, 9, 8), rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    return blk, oracle.Field.from_block(blk), hexfield(fg.hex_mesh_from_block(blk))


def test_voxel_hexahedra_sample_as_the_structured_grid(voxels):
    blk, F, H = voxels
    rng = np.random.default_rng(1)
    x = rng.uniform(-1.0, 10.5, size=(3000, 3))  # sample domain [-0.5, n + 0.5] and beyond
    x[:20] = np.round(x[:20])  # node positions +-0.5: on faces and corners of cells
    x[:20] += 0.5
    v1, ok1 = F.sample(x)
    v2, ok2 = H.sample(x)
    np.testing.assert_array_equal(ok1, ok2)
    assert ok1.mean() > 0.5 and (~ok1).sum() > 100
    np.testing.assert_allclose(v2[ok2], v1[ok1], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(H.dest(x), F.dest(x))


def test_voxel_hexahedra_trace_as_the_structured_grid(voxels):
    blk, F, H = voxels
    seeds = fg.uniform_seeds(12, 150, (-0.2, -0.2, -0.2), (10.2, 9.2, 8.2), sub=3)
    a = F.trace(seeds, 0.5, 40)
    b = H.trace(seeds, 0.5, 40)
    for k in ("steps", "code", "n_verts", "in_outbox", "out_dest"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_allclose(b["final_pos"], a["final_pos"], rtol=0, atol=1e-9)
    assert {oracle.EXIT, oracle.MAX_STEPS} <= set(a["code"].tolist())
    # a halo miss: a seed inside the owned bounds whose stage points leave the sample domain
    # (the field scaled up so a step spans more than the half-cell halo)
    big = fg.turbulence_block(12, dims=(10, 9, 8), rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    big.stored = big.stored * np.float32(8.0)
    Fb, Hb = oracle.Field.from_block(big), hexfield(fg.hex_mesh_from_block(big))
    a = Fb.trace(seeds, 0.5, 40)
    b = Hb.trace(seeds, 0.5, 40)
    assert (a["code"] == oracle.HALO_MISS).sum() > 5
    for k in ("steps", "code", "in_outbox", "out_dest"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_allclose(b["out_pos"][a["in_outbox"] == 1], a["out_pos"][a["in_outbox"] == 1], atol=1e-9)


def _sheared_mesh():
    A = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])
    lat = fg.distorted_hex_mesh(13, (5, 4, 6), jitter=0.0)
    verts = (lat["vertices"].astype(np.float64) @ A.T + np.array([2.0, -1.0, 0.5])).astype(np.float32)
    M = np.array([[0.2, -0.5, 0.1], [0.4, 0.05, -0.3], [-0.1, 0.3, 0.2]])
    c = np.array([0.3, -0.2, 0.1])
    vals = (verts.astype(np.float64) @ M.T + c).astype(np.float32)
    return dict(lat, vertices=verts, values=vals), A, M, c


def test_affine_cells_reproduce_an_affine_field():
    mesh, A, M, c = _sheared_mesh()
    H = hexfield(mesh)
    rng = np.random.default_rng(2)
    r = rng.uniform(0.01, 0.99, size=(2000, 3)) * np.array([5, 4, 6])
    x = r @ A.T + np.array([2.0, -1.0, 0.5])
    v, ok = H.sample(x)
    assert ok.all()
    # the stored values are FP32-rounded: compare with the affine field of the rounded vertices
    want = x @ M.T + c
    assert np.abs(v - want).max() < 1e-6 * np.abs(want).max()
    # exactly the affine interpolant of the stored vertex values: refit M, c from the stored data
    V = mesh["vertices"].astype(np.float64)
    coef, *_ = np.linalg.lstsq(np.c_[V, np.ones(len(V))], mesh["values"].astype(np.float64), rcond=None)
    resid = np.abs(np.c_[V, np.ones(len(V))] @ coef - mesh["values"]).max()
    assert np.abs(v - np.c_[x, np.ones(len(x))] @ coef).max() <= 4 * resid + 1e-12


def test_general_cells_invert_their_own_map():
    mesh = fg.distorted_hex_mesh(14, (6, 5, 4), jitter=0.22, sub=1)
    H = hexfield(mesh)
    rng = np.random.default_rng(3)
    nc = len(mesh["cells"])
    cell = rng.integers(0, nc, size=1500)
    rsu = rng.uniform(0.02, 0.98, size=(1500, 3))
    x = np.einsum("nk,nkc->nc", ohex.weights(rsu), H.X[cell])
    got_cell, got_rsu = H.locate(x)
    np.testing.assert_array_equal(got_cell, cell)
    np.testing.assert_allclose(got_rsu, rsu, rtol=0, atol=1e-10)
    # vertex values at the vertices
    V = mesh["vertices"].astype(np.float64)
    v, ok = H.sample(V)
    assert ok.all()
    np.testing.assert_allclose(v, mesh["values"], rtol=0, atol=1e-12)
    # points beyond the mesh are undefined
    _, ok = H.sample(np.array([[-0.5, 1, 1], [3, 3, 4.5], [np.nan, 1, 1]]))
    assert not ok.any()


def test_pins_catch_a_wrong_vertex_order(monkeypatch, voxels):
    blk = voxels[0]
    mesh = fg.hex_mesh_from_block(blk)
    monkeypatch.setattr(ohex, "VTK_OF_CORNER", np.array([0, 1, 2, 3, 4, 5, 6, 7]))  # VTK read as bit order
    bad = hexfield(mesh)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, 8.0, size=(300, 3))
    v1, ok1 = voxels[1].sample(x)
    v2, ok2 = bad.sample(x)
    assert not (np.array_equal(ok1, ok2) and np.allclose(v1[ok1], v2[ok2], atol=1e-9))
    mesh_s, A, M, c = _sheared_mesh()
    bad = hexfield(mesh_s)
    xs = (rng.uniform(0.1, 0.9, size=(300, 3)) * np.array([5, 4, 6])) @ A.T + np.array([2.0, -1.0, 0.5])
    v, ok = bad.sample(xs)
    assert not (ok.all() and np.abs(v - (xs @ M.T + c)).max() < 1e-5)
