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
  * a plausible slip (a wrong VTK vertex order) is caught by these pins;
  * tetrahedra, wedges and pyramids (cubes of a jittered lattice split into conforming cells):
    every point of the box lies in exactly one cell (a folded map leaves gaps and overlaps, and
    a wrongly ordered pyramid base or wedge triangle is caught), a tetrahedron's coordinates
    are its volume ratios, and a pyramid base or wedge side face interpolates as the
    hexahedron's face does, with vertex values reproduced (a pyramid's apex: near it).
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


# ---------------------------------------------------------------- tetrahedra, wedges, pyramids
def mixedfield(mesh):
    return ohex.HexField(mesh["vertices"], mesh["values"], mesh["cells"], mesh["lo"], mesh["hi"],
                         mesh["rank_grid"], mesh["rank_coord"], cell_types=mesh.get("cell_types"))


def containing_cells(H, x, tol=1e-9):
    """How many cells hold each point (every cell tested, no box culling)."""
    count = np.zeros(len(x), np.int64)
    for kind in np.unique(H.types).tolist():
        cells = np.nonzero(H.types == kind)[0]
        for c in cells:
            ci = np.full(len(x), c)
            r = H.invert(ci, x) if kind == ohex.VTK_HEXAHEDRON else H.invert_kind(kind, ci, x)
            with np.errstate(invalid="ignore"):
                count += ohex.in_domain(kind, r, tol)
    return count


@pytest.mark.parametrize("kind", ["tetra", "wedge", "pyramid", "hex+pyramid"])
def test_split_cubes_hold_each_point_once(kind):
    """Cubes of a jittered lattice split into tetrahedra, wedges or pyramids: every point of the
    box lies in exactly one cell and a point outside in none.  A folded map (a vertex order the
    shape functions do not expect) leaves gaps and overlaps, so this pins each kind's shape
    functions, parametric domain and inversion."""
    mesh = fg.split_hex_mesh(fg.distorted_hex_mesh(18, (2, 2, 2), jitter=0.2), kind)
    H = mixedfield(mesh)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.02, 1.98, size=(400, 3))
    np.testing.assert_array_equal(containing_cells(H, x), 1)
    out = np.array([[-0.1, 1, 1], [1, 2.1, 1], [1, 1, -0.05]])
    np.testing.assert_array_equal(containing_cells(H, out), 0)
    cell, _ = H.locate(x)
    assert (cell >= 0).all()


@pytest.mark.parametrize("kind", ["wedge", "pyramid", "hex+pyramid"])
def test_points_near_warped_cell_vertices_are_found(kind):
    """Near a vertex of a warped (jittered) cell, Newton from the domain's centre can end at a
    second root of the map outside the domain; the nearest-vertex restart still finds the cell.
    Points within 0.06 of every interior lattice vertex of 6 x 6 x 5 jittered cubes."""
    mesh = fg.split_hex_mesh(fg.distorted_hex_mesh(21, (6, 6, 5), jitter=0.2, sub=len(kind)), kind)
    H = mixedfield(mesh)
    k, j, i = np.meshgrid(np.arange(1, 5), np.arange(1, 6), np.arange(1, 6), indexing="ij")
    lattice = (i + 7 * (j + 7 * k)).ravel()  # interior vertices of the 7 x 7 x 6 vertex lattice
    rng = np.random.default_rng(9)
    x = np.repeat(mesh["vertices"][lattice].astype(np.float64), 8, 0) + rng.uniform(-0.06, 0.06, (8 * len(lattice), 3))
    cell, _ = H.locate(x)
    assert (cell >= 0).all(), np.nonzero(cell < 0)[0][:10]


def test_tetra_coordinates_are_volume_ratios():
    """A tetrahedron's parametric coordinates are its barycentric coordinates: the volume of
    the tetrahedron with the point in place of a vertex over the whole volume."""
    mesh = fg.split_hex_mesh(fg.distorted_hex_mesh(19, (2, 1, 1), jitter=0.25), "tetra")
    H = mixedfield(mesh)
    rng = np.random.default_rng(6)
    x = rng.uniform(0.05, 0.95, size=(300, 3)) * np.array([2, 1, 1])
    cell, rst = H.locate(x)
    assert (cell >= 0).all()
    P = H.P[H.cells[cell, :4]]

    def vol(a, b, c, d):
        return np.linalg.det(np.stack([b - a, c - a, d - a], 1))

    whole = vol(P[:, 0], P[:, 1], P[:, 2], P[:, 3])
    lam = np.stack([vol(P[:, 0], x, P[:, 2], P[:, 3]), vol(P[:, 0], P[:, 1], x, P[:, 3]),
                    vol(P[:, 0], P[:, 1], P[:, 2], x)], 1) / whole[:, None]
    np.testing.assert_allclose(rst, lam, rtol=0, atol=1e-12)


def test_split_cells_interpolate_like_the_hexahedron_on_quad_faces():
    """A pyramid's base and a wedge's side faces are whole faces of the cube: there each
    interpolates its four vertices bilinearly, as the hexahedron does, so on those faces the
    split cube samples what the whole cube samples; at the pyramids' apex it samples the centre
    vertex's value, and every kind reproduces its vertex values at its vertices."""
    mesh = fg.distorted_hex_mesh(20, (1, 1, 1), jitter=0.0)
    rng = np.random.default_rng(7)
    mesh["values"] = rng.normal(size=mesh["values"].shape).astype(np.float32)
    Hh = mixedfield(mesh)
    u = rng.uniform(0.05, 0.95, size=(200, 2))
    # points on the faces x = 0, x = 1, y = 0, y = 1 (wedges and pyramids) and z = 0, z = 1 (pyramids)
    faces = {}
    for a in range(3):
        for side in (0.0, 1.0):
            p = np.insert(u, a, side, axis=1)
            p[:, a] = np.clip(p[:, a], 1e-9, 1 - 1e-9)  # just inside the cube
            faces[(a, side)] = p
    want = {k: Hh.sample(p)[0] for k, p in faces.items()}
    Hp = mixedfield(fg.split_hex_mesh(mesh, "pyramid"))
    Hw = mixedfield(fg.split_hex_mesh(mesh, "wedge"))
    for k, p in faces.items():
        np.testing.assert_allclose(Hp.sample(p)[0], want[k], rtol=0, atol=1e-7)
        if k[0] < 2:
            np.testing.assert_allclose(Hw.sample(p)[0], want[k], rtol=0, atol=1e-7)
    pm = fg.split_hex_mesh(mesh, "pyramid")
    apex = pm["vertices"][-1].astype(np.float64)
    near = apex + np.array([[1e-9, 2e-9, -1e-9], [1e-7, 0, 0], [0, 0, 1e-6]])
    v, ok = Hp.sample(near)
    assert ok.all()
    np.testing.assert_allclose(v, np.repeat(pm["values"][-1:], 3, 0), rtol=0, atol=1e-5)
    for kind in ("tetra", "wedge", "pyramid"):
        m = fg.split_hex_mesh(mesh, kind)
        H = mixedfield(m)
        corners = len(mesh["vertices"])  # a pyramid's map is singular at its apex: tested near it above
        vv, ok = H.sample(np.clip(m["vertices"][:corners].astype(np.float64), 1e-12, 1 - 1e-12))
        assert ok.all()
        np.testing.assert_allclose(vv, m["values"][:corners], rtol=0, atol=1e-9)


def test_pins_catch_a_folded_pyramid_or_wedge(monkeypatch):
    """The cover pin fails when the pyramid base or a wedge triangle is read in the wrong order."""
    mesh = fg.distorted_hex_mesh(18, (2, 2, 2), jitter=0.2)
    x = np.random.default_rng(5).uniform(0.02, 1.98, size=(200, 3))
    for kind, swap in (("pyramid", [0, 1, 3, 2, 4]), ("wedge", [0, 1, 2, 3, 5, 4])):
        m = fg.split_hex_mesh(mesh, kind)
        cells = m["cells"].copy()
        k = len(swap)
        cells[:, :k] = cells[:, swap]
        H = mixedfield(dict(m, cells=cells))
        assert not (containing_cells(H, x) == 1).all(), kind
