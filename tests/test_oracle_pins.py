"""Pins for the FP64 oracle, independent of the oracle's own formulas.

Each test checks the oracle against something the mathematics fixes: closed
forms of the discrete method, exact-rational brute force, a library
interpolator, invariants and convergence order.  A plausible slip in the
oracle (a dropped RK4 term, a wrong stage weight, a transposed axis, an
off-by-one cell index, a wrong termination order) fails at least one of them.
"""
from decimal import Decimal as Dc, localcontext
import math

import numpy as np
import pytest

import fieldgen as fg
import oracle
from oracle import ACTIVE, EXIT, HALO_MISS, MAX_STEPS, NONFINITE, STAGNANT

RNG = np.random.default_rng(12345)


def grid_field(fn, dims=(5, 6, 7), ghost=1, origin=(0.25, -1.0, 2.0), spacing=(0.5, 0.75, 1.25),
               periodic=False, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0), lo=None, hi=None):
    b = fg.closed_form_block(fn, dims, ghost=ghost, origin=origin, spacing=spacing, lo=lo, hi=hi,
                             boundary=int(periodic), rank_grid=rank_grid, rank_coord=rank_coord)
    f = oracle.Field(b.dims, b.ghost, b.origin, b.spacing, b.lo, b.hi, periodic=periodic,
                     rank_grid=b.rank_grid, rank_coord=b.rank_coord, nodes=b.values,
                     fmt=oracle.FMT_F64)
    return f, b


def domain_points(b, n):
    lo = np.array(b.origin) - np.array(b.spacing) * b.ghost
    hi = np.array(b.origin) + (np.array(b.dims) - 1 + b.ghost) * np.array(b.spacing)
    return lo + RNG.random((n, 3)) * (hi - lo), lo, hi


# ---------------------------------------------------------------- sampling
def test_trilinear_exact_on_its_span():
    """The trilinear interpolant reproduces span{1,x,y,z,xy,xz,yz,xyz} exactly."""
    c = RNG.normal(size=(3, 8))

    def fn(x, y, z):
        basis = [np.ones_like(x), x, y, z, x * y, x * z, y * z, x * y * z]
        return tuple(sum(c[k, j] * basis[j] for j in range(8)) for k in range(3))

    f, b = grid_field(fn)
    x, _, _ = domain_points(b, 2000)
    v, d = f.sample(x)
    assert d.all()
    ex = np.stack(fn(x[:, 0], x[:, 1], x[:, 2]), axis=1)
    np.testing.assert_allclose(v, ex, rtol=0, atol=1e-11 * np.abs(ex).max())


def test_trilinear_matches_scipy_regular_grid():
    """Same interpolant as scipy's RegularGridInterpolator(method='linear')."""
    from scipy.interpolate import RegularGridInterpolator
    dims, ghost = (6, 5, 4), 1
    vals = RNG.normal(size=(dims[2] + 2, dims[1] + 2, dims[0] + 2, 3))
    origin, spacing = (1.0, 2.0, -3.0), (0.5, 0.25, 2.0)
    f = oracle.Field(dims, ghost, origin, spacing, (0, 0, 0), (1, 1, 1), nodes=vals[None],
                     fmt=oracle.FMT_F64)
    axes = [origin[a] + (np.arange(dims[a] + 2) - 1) * spacing[a] for a in range(3)]
    x = np.stack([axes[a][0] + RNG.random(3000) * (axes[a][-1] - axes[a][0]) for a in range(3)], 1)
    interp = RegularGridInterpolator((axes[2], axes[1], axes[0]), vals, method="linear")
    ref = interp(x[:, ::-1])
    v, d = f.sample(x)
    assert d.all()
    np.testing.assert_allclose(v, ref, rtol=0, atol=1e-12)


def test_sample_reproduces_nodes_and_domain_is_closed():
    dims, ghost = (4, 3, 5), 1
    vals = RNG.normal(size=(1, dims[2] + 2, dims[1] + 2, dims[0] + 2, 3))
    f = oracle.Field(dims, ghost, (0, 0, 0), (1, 1, 1), (0, 0, 0), (3, 2, 4), nodes=vals,
                     fmt=oracle.FMT_F64)
    # every stored node, incl. the far ghost corner (f = 1 on the last cell)
    idx = np.stack(np.meshgrid(np.arange(6), np.arange(5), np.arange(7), indexing="ij"), -1).reshape(-1, 3)
    x = idx.astype(float) - 1.0
    v, d = f.sample(x)
    assert d.all()
    np.testing.assert_array_equal(v, vals[0][idx[:, 2], idx[:, 1], idx[:, 0]])
    # just outside the stored nodes on each face: undefined
    eps = 1e-9
    out = np.array([[-1 - eps, 0, 0], [4 + eps, 0, 0], [0, -1 - eps, 0], [0, 3 + eps, 0],
                    [0, 0, -1 - eps], [0, 0, 5 + eps], [np.nan, 0, 0]])
    _, d = f.sample(out)
    assert not d.any()


def test_periodic_wrap_equals_extended_grid():
    """Periodic sampling = non-periodic sampling of the grid extended by one wrapped layer."""
    n = 6
    vals = RNG.normal(size=(n, n, n, 3))
    sp = 2 * np.pi / n
    fp = oracle.Field((n, n, n), 0, (0, 0, 0), (sp,) * 3, (0, 0, 0), (2 * np.pi,) * 3,
                      periodic=True, nodes=vals[None], fmt=oracle.FMT_F64)
    ext = np.concatenate([vals, vals[:1]], axis=0)
    ext = np.concatenate([ext, ext[:, :1]], axis=1)
    ext = np.concatenate([ext, ext[:, :, :1]], axis=2)
    fe = oracle.Field((n + 1,) * 3, 0, (0, 0, 0), (sp,) * 3, (0, 0, 0), (1, 1, 1),
                      nodes=ext[None], fmt=oracle.FMT_F64)
    x = RNG.random((500, 3)) * 2 * np.pi
    shift = RNG.integers(-3, 4, size=(500, 3)) * 2 * np.pi
    v1, _ = fp.sample(x + shift)
    v2, d2 = fe.sample(x)
    assert d2.all()
    np.testing.assert_allclose(v1, v2, atol=1e-12)


def test_stored_formats_decode_exactly():
    vals = RNG.normal(size=(1, 3, 3, 3, 3))
    for fmt in (fg.F32, fg.F16, fg.BF16):
        st = fg.quantize(vals, fmt)
        f = oracle.Field((1, 1, 1), 1, (0, 0, 0), (1, 1, 1), (0, 0, 0), (1, 1, 1), nodes=st,
                         fmt=fmt)
        x = np.array([[-1.0, 0.0, 1.0], [0.0, -1.0, 0.0], [1.0, 1.0, 1.0]])
        v, _ = f.sample(x)
        exact = fg.stored_as_f64(st, fmt)[0]
        ref = np.array([exact[2, 1, 0], exact[1, 0, 1], exact[2, 2, 2]])
        np.testing.assert_array_equal(v, ref)


# ---------------------------------------------------------------- RK4 closed forms
def test_uniform_flow_straight_lines_and_exit_step():
    """v = c (dyadic): P_n = P0 + n h c exactly; exit at the first n outside [lo,hi)."""
    c = np.array([0.375, -0.25, 0.125])
    f, b = grid_field(lambda x, y, z: (0 * x + c[0], 0 * x + c[1], 0 * x + c[2]),
                      dims=(9, 9, 9), origin=(0.5, 0.5, 0.5), spacing=(1, 1, 1),
                      lo=(0, 0, 0), hi=(9, 9, 9), rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    seeds = np.array([[4.0, 4.0, 4.0], [1.0, 7.5, 0.25], [8.5, 0.5, 8.75]])
    h = 0.5
    r = f.trace(seeds, h, 1000)
    for i, p0 in enumerate(seeds):
        n = r["steps"][i]
        path = p0 + np.arange(n + 1)[:, None] * h * c
        np.testing.assert_array_equal(r["verts"][i, :n + 1], path)
        # first step index at which the position leaves [0, 9)
        k = np.arange(1, 1000)
        pos = p0 + k[:, None] * h * c
        first = k[np.any((pos < 0) | (pos >= 9), axis=1)][0]
        assert n == first and r["code"][i] == EXIT
        exp_r = 1 + np.floor(pos[first - 1] / 9).astype(int)
        assert r["out_dest"][i] == exp_r[0] + 3 * (exp_r[1] + 3 * exp_r[2])
        np.testing.assert_array_equal(r["out_pos"][i], path[-1])


def rk4_matrix(Z):
    I = np.eye(3)
    return I + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24


def test_linear_field_closed_form_rotation():
    """v = A (x - xc): RK4 gives P_n - xc = R(hA)^n (P0 - xc), R the 4th-order Taylor polynomial.
    For solid-body rotation the radius scales by sqrt(1 - t^6/72 + t^8/576) per step."""
    w, xc = 0.7, np.array([3.0, 3.0, 0.0])
    A = np.array([[0, -w, 0], [w, 0, 0], [0, 0, 0]])
    f, b = grid_field(lambda x, y, z: (-w * (y - 3.0), w * (x - 3.0), 0 * z),
                      dims=(7, 7, 4), origin=(0, 0, 0), spacing=(1, 1, 1), lo=(-1, -1, -1),
                      hi=(100, 100, 100))
    h, steps = 0.4, 120
    seeds = np.array([[4.5, 3.0, 1.0], [3.0, 1.2, 2.0], [1.7, 3.9, 0.5]])
    r = f.trace(seeds, h, steps)
    R = rk4_matrix(h * A)
    theta = w * h
    gain = math.sqrt(1 - theta ** 6 / 72 + theta ** 8 / 576)
    for i, p0 in enumerate(seeds):
        assert r["code"][i] == MAX_STEPS and r["steps"][i] == steps
        q = p0 - xc
        for n in range(steps + 1):
            np.testing.assert_allclose(r["verts"][i, n] - xc, q, atol=1e-11)
            q = R @ q
        rad = np.hypot(*(r["verts"][i, :steps + 1, :2] - xc[:2]).T)
        np.testing.assert_allclose(rad[1:] / rad[:-1], gain, rtol=1e-13)
        assert abs(rad[-1] / rad[0] - gain ** steps) < 1e-12 and gain ** steps < 1 - 2e-4


def test_unsteady_time_blend_closed_form():
    """Slices V0 = c, V1 = 2c over [t0, t0+dt]: x' = c (1 + (t-t0)/dt) and RK4 is exact on
    polynomials in t of degree <= 4: P_n = P0 + c (tau + tau^2/(2 dt)), tau = n h."""
    c = np.array([0.25, 0.5, -0.125])
    dims = (6, 6, 6)
    one = fg.closed_form_block(lambda x, y, z: (0 * x + c[0], 0 * x + c[1], 0 * x + c[2]), dims,
                               ghost=1, lo=(-100, -100, -100), hi=(100, 100, 100))
    vals = np.concatenate([one.values, 2 * one.values], axis=0)
    t0, dt, h = 0.5, 4.0, 0.25
    f = oracle.Field(dims, 1, (0, 0, 0), (1, 1, 1), (-100,) * 3, (100,) * 3, n_slices=2, t0=t0,
                     slice_dt=dt, nodes=vals, fmt=oracle.FMT_F64)
    p0 = np.array([[2.0, 2.0, 2.5]])
    r = f.trace(p0, h, 16, t_birth=t0)
    tau = np.arange(17) * h
    ref = p0 + (tau + tau ** 2 / (2 * dt))[:, None] * c
    np.testing.assert_allclose(r["verts"][0, :17], ref, atol=1e-13)
    # a time-constant slice stack gives exactly the steady result
    g = RNG.normal(size=(1,) + one.values.shape[1:]) * 0.1
    fs = oracle.Field(dims, 1, (0, 0, 0), (1, 1, 1), (-100,) * 3, (100,) * 3, nodes=g,
                      fmt=oracle.FMT_F64)
    fu = oracle.Field(dims, 1, (0, 0, 0), (1, 1, 1), (-100,) * 3, (100,) * 3, n_slices=3,
                      t0=0.0, slice_dt=1.0, nodes=np.concatenate([g, g, g]), fmt=oracle.FMT_F64)
    s = np.array([[2.2, 2.3, 2.4], [1.1, 3.3, 0.7]])
    np.testing.assert_array_equal(fs.trace(s, 0.3, 12)["verts"], fu.trace(s, 0.3, 12)["verts"])



def test_unsteady_time_clamped_at_both_ends():
    """Outside the slices' time span the field is the end slice (linear blend clamped): with
    slices c, 2c, 3c at t0 = 0.5, dt = 4, a particle born at t = 10 (past the last slice, 8.5)
    moves on a straight line at 3c and one that lives in t < t0 at c. One that crosses t0 leaves
    the straight line, so the clamp is not a constant offset."""
    c = np.array([0.25, 0.5, -0.125])
    dims = (6, 6, 6)
    one = fg.closed_form_block(lambda x, y, z: (0 * x + c[0], 0 * x + c[1], 0 * x + c[2]), dims,
                               ghost=1, lo=(-100, -100, -100), hi=(100, 100, 100))
    vals = np.concatenate([one.values, 2 * one.values, 3 * one.values], axis=0)
    f = oracle.Field(dims, 1, (0, 0, 0), (1, 1, 1), (-100,) * 3, (100,) * 3, n_slices=3, t0=0.5,
                     slice_dt=4.0, nodes=vals, fmt=oracle.FMT_F64)
    p0 = np.array([[2.0, 2.0, 2.5]])
    h, n = 0.25, 8  # the particles stay inside the stored nodes
    tau = (np.arange(n + 1) * h)[:, None]
    late = f.trace(p0, h, n, t_birth=10.0)["verts"][0, :n + 1]
    np.testing.assert_allclose(late, p0 + 3 * c * tau, rtol=0, atol=1e-13)
    early = f.trace(p0, h, n, t_birth=-6.0)["verts"][0, :n + 1]  # t stays below -4
    np.testing.assert_allclose(early, p0 + c * tau, rtol=0, atol=1e-13)
    across = f.trace(p0, h, n, t_birth=-1.0)["verts"][0, :n + 1]  # t runs from -1 to 1
    assert np.abs(across[-1] - (p0[0] + c * n * h)).max() > 1e-3

def _rk4_error(field, p0, T, h, ref):
    n = int(round(T / h))
    r = field.trace(p0, h, n, eps=0.0, keep_verts=False)
    return np.abs(r["final_pos"] - ref).max()


def test_rk4_order_four_on_analytic_abc():
    fa = oracle.Field.abc_analytic()
    p0 = np.array([[1.0, 2.0, 3.0], [4.0, 0.5, 5.5]])
    T = 2.0
    ref = fa.trace(p0, T / 8192, 8192, eps=0.0, keep_verts=False)["final_pos"]
    errs = [_rk4_error(fa, p0, T, h, ref) for h in (0.2, 0.1, 0.05, 0.025)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for q in ratios:
        assert 14.0 < q < 18.5, ratios


def test_rk4_order_four_on_grid_trilinear_span_field():
    """v = (yz, xz, xy) is divergence-free and inside the trilinear span: the grid field equals
    the analytic one, so the grid trajectories converge at order 4 too."""
    f, b = grid_field(lambda x, y, z: (y * z, x * z, x * y), dims=(5, 5, 5), ghost=1,
                      origin=(-1, -1, -1), spacing=(0.5, 0.5, 0.5), lo=(-5, -5, -5), hi=(5, 5, 5))
    p0 = np.array([[0.3, -0.2, 0.1], [-0.4, 0.25, 0.35]])
    T = 1.0
    ref = f.trace(p0, T / 4096, 4096, eps=0.0, keep_verts=False)["final_pos"]
    errs = [_rk4_error(f, p0, T, h, ref) for h in (0.25, 0.125, 0.0625)]
    for i in range(2):
        assert 14.0 < errs[i] / errs[i + 1] < 18.5, errs


# ---------------------------------------------------------------- termination rules
def test_stagnation_max_steps_and_nonfinite():
    eps = 1e-6
    for mag, code in ((0.9e-6, STAGNANT), (1.1e-6, MAX_STEPS)):
        f, _ = grid_field(lambda x, y, z: (0 * x + mag, 0 * x, 0 * x), dims=(4, 4, 4),
                          lo=(-10, -10, -10), hi=(10, 10, 10))
        r = f.trace(np.array([[1.0, 0.0, 3.0]]), 0.5, 7, eps=eps)
        assert r["code"][0] == code
        assert r["steps"][0] == (0 if code == STAGNANT else 7)
        assert r["n_verts"][0] == r["steps"][0] + 1
    # a NaN node poisons the cell it touches
    b = fg.closed_form_block(lambda x, y, z: (0 * x + 1, 0 * x, 0 * x), (4, 4, 4), ghost=1,
                             lo=(-10, -10, -10), hi=(10, 10, 10))
    v = b.values.copy()
    v[0, 2, 2, 3, 1] = np.nan  # node (x=2, y=1, z=1)
    f = oracle.Field(b.dims, 1, b.origin, b.spacing, b.lo, b.hi, nodes=v, fmt=oracle.FMT_F64)
    r = f.trace(np.array([[0.25, 1.5, 1.5]]), 0.5, 10)
    assert r["code"][0] == NONFINITE
    # steps taken before the NaN cell is reached: stages at x+0.5h*1, x+h... reach x>=1 first
    # at the step starting from x=0.75 (k4 at x=1.25 lies in the cell [1,2])
    assert r["steps"][0] == 1
    np.testing.assert_array_equal(r["final_pos"][0], [0.75, 1.5, 1.5])


def test_halo_miss_goes_to_outbox_at_old_position():
    """A stage point outside the stored nodes makes sample() undefined: the particle is
    handed to the outbox at P0 with its step count unchanged, dest of the failing point."""
    c = (2.0, 0.0, 0.0)
    f, b = grid_field(lambda x, y, z: (0 * x + c[0], 0 * x, 0 * x), dims=(4, 4, 4), ghost=1,
                      origin=(0.5, 0.5, 0.5), spacing=(1, 1, 1), lo=(0, 0, 0), hi=(4, 4, 4),
                      rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    # stored nodes reach x = 4.5; from x=2.0 with h=0.75: k2 stage at 2.75, k4 stage at 3.5 ok,
    # P1 = 3.5; next step: k2 stage at 4.25 ok, k4 stage at 5.0 > 4.5 -> undefined
    r = f.trace(np.array([[2.0, 2.0, 2.0]]), 0.75, 100)
    assert r["code"][0] == HALO_MISS and r["steps"][0] == 1 and r["in_outbox"][0] == 1
    np.testing.assert_array_equal(r["out_pos"][0], [3.5, 2.0, 2.0])
    assert r["out_dest"][0] == 2 + 3 * (1 + 3 * 1)  # x = 5.0 lies in rank column 2


def test_seed_outside_bounds_exits_immediately():
    f, b = grid_field(lambda x, y, z: (0 * x + 0.25, 0 * x, 0 * x), dims=(4, 4, 4), ghost=1,
                      origin=(0.5, 0.5, 0.5), spacing=(1, 1, 1), lo=(0, 0, 0), hi=(4, 4, 4),
                      rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    r = f.trace(np.array([[4.0, 1.0, 1.0], [-0.0, 1.0, 1.0]]), 0.5, 10)
    assert list(r["code"]) == [EXIT, MAX_STEPS]
    assert r["steps"][0] == 0 and r["in_outbox"][0] == 1 and r["out_dest"][0] == 2 + 3 * 4


def test_destination_id_rank_grid():
    f, _ = grid_field(lambda x, y, z: (0 * x, 0 * x, 0 * x), dims=(4, 4, 4), ghost=1,
                      origin=(0.5, 0.5, 0.5), spacing=(1, 1, 1), lo=(0, 0, 0), hi=(4, 4, 4),
                      rank_grid=(4, 3, 2), rank_coord=(1, 1, 0))
    pts, exp = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                p = np.array([2.0 + 4 * dx + 0.3, 2.0 + 4 * dy - 0.7, 2.0 + 4 * dz + 0.1])
                r = np.array([1 + dx, 1 + dy, 0 + dz])
                ok = np.all(r >= 0) and np.all(r < [4, 3, 2])
                pts.append(p)
                exp.append(int(r[0] + 4 * (r[1] + 3 * r[2])) if ok else -1)
    # the half-open bounds put a point on hi into the next rank
    pts.append(np.array([4.0, 0.0, 0.0]))
    exp.append(2 + 4 * (1 + 3 * 0))
    np.testing.assert_array_equal(f.dest(np.array(pts)), exp)


def test_record_stride_rule():
    """Vertex j is kept when j % stride == 0, and the final vertex always."""
    c = (0.25, 0.0, 0.0)
    f, _ = grid_field(lambda x, y, z: (0 * x + c[0], 0 * x, 0 * x), dims=(10, 4, 4), ghost=1,
                      origin=(0.5, 0.5, 0.5), spacing=(1, 1, 1), lo=(0, 0, 0), hi=(10, 4, 4))
    seeds = np.array([[0.5, 1.0, 1.0], [1.0, 1.0, 1.0]])
    full = f.trace(seeds, 1.0, 37, stride=1)
    sub = f.trace(seeds, 1.0, 37, stride=5)
    for i in range(2):
        n = full["steps"][i]
        keep = [j for j in range(n + 1) if j % 5 == 0 or j == n]
        assert sub["n_verts"][i] == len(keep)
        np.testing.assert_array_equal(sub["verts"][i, :len(keep)], full["verts"][i, keep])


# ---------------------------------------------------------------- high-precision brute force
def _hp_sample(V, dims, ghost, origin, spacing, x):
    idx, fr = [], []
    for a in range(3):
        ns = dims[a] + 2 * ghost
        s = (x[a] - origin[a]) / spacing[a] + ghost
        if s < 0 or s > ns - 1:
            return None
        i = min(int(s.to_integral_value(rounding="ROUND_FLOOR")), ns - 2)
        idx.append(i)
        fr.append(s - i)
    out = [Dc(0)] * 3
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((fr[0] if dx else 1 - fr[0]) * (fr[1] if dy else 1 - fr[1]) *
                     (fr[2] if dz else 1 - fr[2]))
                node = V[idx[2] + dz][idx[1] + dy][idx[0] + dx]
                out = [out[c] + w * node[c] for c in range(3)]
    return out


def _hp_trace(V, dims, ghost, origin, spacing, lo, hi, p0, h, m, eps2):
    """Independent 60-digit evaluation of the update loop (no oracle code)."""
    P = list(p0)
    verts = [tuple(P)]
    inside = lambda q: all(lo[a] <= q[a] < hi[a] for a in range(3))
    if not inside(P):
        return verts, 0, EXIT
    n = 0
    while True:
        if n >= m:
            return verts, n, MAX_STEPS
        k1 = _hp_sample(V, dims, ghost, origin, spacing, P)
        if k1 is None:
            return verts, n, HALO_MISS
        if sum(c * c for c in k1) < eps2:
            return verts, n, STAGNANT
        q = [P[a] + h / 2 * k1[a] for a in range(3)]
        k2 = _hp_sample(V, dims, ghost, origin, spacing, q)
        if k2 is None:
            return verts, n, HALO_MISS
        q = [P[a] + h / 2 * k2[a] for a in range(3)]
        k3 = _hp_sample(V, dims, ghost, origin, spacing, q)
        if k3 is None:
            return verts, n, HALO_MISS
        q = [P[a] + h * k3[a] for a in range(3)]
        k4 = _hp_sample(V, dims, ghost, origin, spacing, q)
        if k4 is None:
            return verts, n, HALO_MISS
        P = [P[a] + h / 6 * (k1[a] + 2 * k2[a] + 2 * k3[a] + k4[a]) for a in range(3)]
        n += 1
        verts.append(tuple(P))
        if not inside(P):
            return verts, n, EXIT


@pytest.mark.parametrize("case", range(6))
def test_brute_force_high_precision(case):
    """Tiny grids (2^3 and 3x4x2 interior nodes), 8 seeds, <= 10 steps, dyadic data, evaluated
    with 60 significant digits: the FP64 oracle must agree to rounding, and exactly in codes."""
    rng = np.random.default_rng(100 + case)
    dims = (2, 2, 2) if case < 3 else (3, 4, 2)
    ghost = 1
    lo, hi = (0, 0, 0), tuple(dims)
    shape = (dims[2] + 2, dims[1] + 2, dims[0] + 2)
    ints = rng.integers(-12, 13, size=shape + (3,))
    if case == 2:
        ints[..., :] = 0  # stagnant everywhere
    hq = 0.25 if case % 2 == 0 else 0.375
    m = 10
    eps = 1e-6
    seeds = rng.integers(0, 64 * np.array(dims), size=(8, 3)) / 64.0
    f = oracle.Field(dims, ghost, (0.5, 0.5, 0.5), (1, 1, 1), lo, hi,
                     nodes=(ints / 16.0)[None], fmt=oracle.FMT_F64)
    r = f.trace(seeds, hq, m, eps=eps)
    with localcontext() as ctx:
        ctx.prec = 60
        V = [[[[Dc(int(ints[z, y, x, c])) / 16 for c in range(3)] for x in range(shape[2])]
              for y in range(shape[1])] for z in range(shape[0])]
        for i, s in enumerate(seeds):
            verts, n, code = _hp_trace(V, dims, ghost, (Dc("0.5"),) * 3, (Dc(1),) * 3, lo, hi,
                                       [Dc(float(c)) for c in s], Dc(hq), m, Dc(eps) ** 2)
            ref = np.array([[float(c) for c in v] for v in verts])
            got = r["verts"][i, :len(verts)]
            near = np.min(np.abs(np.concatenate([ref - np.array(lo), ref - np.array(hi)], 1))) < 1e-9
            if not near:
                assert r["steps"][i] == n and r["code"][i] == code, (i, n, code)
            np.testing.assert_allclose(got, ref, atol=1e-12)
