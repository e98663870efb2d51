"""Seeded synthetic inputs for the field-line workloads.

This module makes inputs only (vector-field node values, seed sets, block
descriptions) and quantises FP64 node values to the storage formats with
round-to-nearest-even.  It holds none of the advection method's arithmetic;
both the FP64 oracle and the GPU library consume the bytes it produces.

Workload recipes (all synthetic; the paper's own data sets are not used):

* ``abc_block``: steady Arnold-Beltrami-Childress flow, A=sqrt(3), B=sqrt(2),
  C=1, sampled at nodes i*2pi/N of a periodic N^3 grid.
* ``turbulence_block``: a rank's block of divergence-free random-Fourier-mode
  turbulence (k^-5/3 energy spectrum over |k| in [1,32]), voxel-centred nodes
  with one ghost layer, normalised to max node |v| = 1 cell per unit time.
* closed-form fields (uniform, linear, (yz,xz,xy)) for the exactness pins.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfieldgen.so")
_lib = None

F32, F16, BF16 = 0, 1, 2
DTYPE_NAMES = {F32: "f32", F16: "f16", BF16: "bf16"}
DTYPE_BYTES = {F32: 4, F16: 2, BF16: 2}

# stream purposes
P_MODES, P_SEEDS, P_BLOB, P_MAXSTEPS, P_BLOCKSHAPE, P_NSEEDS, P_MLP, P_TRAIN, P_HEXJIT = range(1, 10)


def build(verbose: bool = False) -> str:
    """Compile libfieldgen.so with gcc (portable flags so values match across hosts)."""
    src = os.path.join(_HERE, "gen.c")
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-pthread", src, "-o", _LIB_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u64, i64, dbl, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.fg_stream.restype = u64
    lib.fg_stream.argtypes = [u64, u64, u64]
    lib.fg_u64.restype = u64
    lib.fg_u64.argtypes = [u64, u64]
    for name in ("fg_unif_fill", "fg_unif24_fill", "fg_normal_fill"):
        getattr(lib, name).argtypes = [u64, u64, i64, vp]
        getattr(lib, name).restype = None
    lib.fg_quantize.argtypes = [vp, i64, ctypes.c_int, vp]
    lib.fg_quantize.restype = None
    lib.fg_turb_modes.argtypes = [u64, ctypes.c_int, dbl, dbl, dbl] + [vp] * 6
    lib.fg_turb_modes.restype = None
    lib.fg_turb_eval.argtypes = [ctypes.c_int] + [vp] * 5 + [ctypes.c_int] * 3 + [dbl] * 4 + [vp, ctypes.c_int]
    lib.fg_turb_eval.restype = dbl
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def stream(config: int, purpose: int, sub: int = 0) -> int:
    return int(_load().fg_stream(config, purpose, sub))


def uniform(strm: int, n: int, first: int = 0) -> np.ndarray:
    out = np.empty(n, np.float64)
    _load().fg_unif_fill(strm, first, n, _ptr(out))
    return out


def uniform24(strm: int, n: int, first: int = 0) -> np.ndarray:
    """Uniform values k*2^-24 in [0,1): exactly representable in FP32."""
    out = np.empty(n, np.float64)
    _load().fg_unif24_fill(strm, first, n, _ptr(out))
    return out


def normal(strm: int, n: int, first: int = 0) -> np.ndarray:
    out = np.empty(n, np.float64)
    _load().fg_normal_fill(strm, first, n, _ptr(out))
    return out


def u64(strm: int, i: int) -> int:
    return int(_load().fg_u64(strm, i))


def quantize(values: np.ndarray, fmt: int) -> np.ndarray:
    """RNE-quantise FP64 values directly to FP32 (float32 array) or FP16/BF16 (uint16 bits)."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = np.empty(v.shape, np.float32 if fmt == F32 else np.uint16)
    _load().fg_quantize(_ptr(v), v.size, fmt, _ptr(out))
    return out


def stored_as_f64(stored: np.ndarray, fmt: int) -> np.ndarray:
    """Exact FP64 value of stored FP32/FP16/BF16 node data."""
    if fmt == F32:
        return stored.astype(np.float64)
    if fmt == F16:
        return stored.view(np.float16).astype(np.float64)
    return (stored.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Block description shared by the workloads
# ---------------------------------------------------------------------------
BOUNDARY_BLOCK, BOUNDARY_PERIODIC = 0, 1


@dataclasses.dataclass
class Block:
    """One rank-local block: interior nodes, ghost layers, world mapping, owned bounds.

    ``values`` holds FP64 node values [S][nz+2g][ny+2g][nx+2g][3], x fastest;
    ``stored`` the same values quantised to ``fmt``.
    """
    dims: tuple            # interior nodes (nx, ny, nz)
    ghost: int
    origin: tuple          # world position of interior node 0
    spacing: tuple
    lo: tuple              # owned bounds, half-open
    hi: tuple
    boundary: int = BOUNDARY_BLOCK
    rank_grid: tuple = (1, 1, 1)
    rank_coord: tuple = (0, 0, 0)
    n_slices: int = 1
    t0: float = 0.0
    slice_dt: float = 1.0
    values: Optional[np.ndarray] = None
    fmt: int = F32
    stored: Optional[np.ndarray] = None

    def quantise(self, fmt: int) -> "Block":
        b = dataclasses.replace(self, fmt=fmt)
        b.stored = quantize(self.values, fmt)
        return b

    @property
    def store_shape(self):
        nx, ny, nz = self.dims
        g = self.ghost
        return (self.n_slices, nz + 2 * g, ny + 2 * g, nx + 2 * g, 3)

    @property
    def extent(self) -> float:
        return float(max(h - l for l, h in zip(self.lo, self.hi)))


def _node_coords(n: int, origin: float, spacing: float, ghost: int) -> np.ndarray:
    return origin + (np.arange(n + 2 * ghost) - ghost) * spacing


def sample_closed_form(fn, dims, ghost, origin, spacing) -> np.ndarray:
    """Evaluate fn(x, y, z) -> (vx, vy, vz) at the stored nodes, FP64, [1][z][y][x][3]."""
    xs = _node_coords(dims[0], origin[0], spacing[0], ghost)
    ys = _node_coords(dims[1], origin[1], spacing[1], ghost)
    zs = _node_coords(dims[2], origin[2], spacing[2], ghost)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    vx, vy, vz = fn(X, Y, Z)
    out = np.empty(X.shape + (3,), np.float64)
    out[..., 0] = vx
    out[..., 1] = vy
    out[..., 2] = vz
    return out[None]


ABC = (np.sqrt(3.0), np.sqrt(2.0), 1.0)


def abc_velocity(x, y, z, A=ABC[0], B=ABC[1], C=ABC[2]):
    """Arnold-Beltrami-Childress flow (standard form)."""
    return (A * np.sin(z) + C * np.cos(y), B * np.sin(x) + A * np.cos(z), C * np.sin(y) + B * np.cos(x))


def abc_block(n: int = 32, fmt: int = F32) -> Block:
    """Periodic N^3 grid over [0, 2pi)^3, nodes at i*2pi/N, no ghost layer."""
    d = 2.0 * np.pi / n
    b = Block(dims=(n, n, n), ghost=0, origin=(0.0, 0.0, 0.0), spacing=(d, d, d),
              lo=(0.0, 0.0, 0.0), hi=(2 * np.pi,) * 3, boundary=BOUNDARY_PERIODIC)
    b.values = sample_closed_form(abc_velocity, b.dims, 0, b.origin, b.spacing)
    return b.quantise(fmt)


def closed_form_block(fn, dims, ghost=1, origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0),
                      lo=None, hi=None, fmt=F32, boundary=BOUNDARY_BLOCK,
                      rank_grid=(1, 1, 1), rank_coord=(0, 0, 0)) -> Block:
    if lo is None:
        lo = tuple(o for o in origin)
        hi = tuple(o + (n - 1) * s for o, n, s in zip(origin, dims, spacing))
    b = Block(dims=tuple(dims), ghost=ghost, origin=tuple(origin), spacing=tuple(spacing),
              lo=tuple(lo), hi=tuple(hi), boundary=boundary, rank_grid=tuple(rank_grid),
              rank_coord=tuple(rank_coord))
    b.values = sample_closed_form(fn, b.dims, ghost, b.origin, b.spacing)
    return b.quantise(fmt)


def _cache_dir() -> str:
    d = os.environ.get("STREAMI_CACHE", "/tmp/streami_cache")
    os.makedirs(d, exist_ok=True)
    return d


def turbulence_values(config: int, dims, sub: int = 0, n_modes: int = 512, kmin: float = 1.0,
                      kmax: float = 32.0, n_slices: int = 1, threads: int = 0) -> np.ndarray:
    """Voxel-centred turbulence, one ghost layer, FP64 [S][nz+2][ny+2][nx+2][3].

    Interior node i sits at i+0.5 (cell units).  Normalised so that the largest
    stored |v| over every slice is exactly 1.  With n_slices > 1 the mode phases
    drift linearly: phi_m(s) = phi_m + 2pi r_m s/(S-1).
    """
    nx, ny, nz = dims
    key = f"turb-{config}-{sub}-{nx}x{ny}x{nz}-{n_modes}-{kmin}-{kmax}-{n_slices}-v1"
    path = os.path.join(_cache_dir(), hashlib.sha1(key.encode()).hexdigest()[:16] + ".npy")
    if os.path.exists(path):
        try:
            return np.load(path, mmap_mode=None, allow_pickle=False)
        except Exception:
            pass
    lib = _load()
    L = float(max(dims))
    M = n_modes
    kappa, amp, phi, drift = (np.empty(M) for _ in range(4))
    u, e = np.empty(3 * M), np.empty(3 * M)
    lib.fg_turb_modes(stream(config, P_MODES, sub), M, kmin, kmax, L, _ptr(kappa), _ptr(u),
                      _ptr(e), _ptr(amp), _ptr(phi), _ptr(drift))
    out = np.empty((n_slices, nz + 2, ny + 2, nx + 2, 3), np.float64)
    threads = threads or min(16, os.cpu_count() or 1)
    vmax = 0.0
    for s in range(n_slices):
        ph = phi + (2 * np.pi * drift * s / (n_slices - 1) if n_slices > 1 else 0.0)
        ph = np.ascontiguousarray(ph)
        m = lib.fg_turb_eval(M, _ptr(kappa), _ptr(u), _ptr(e), _ptr(amp), _ptr(ph), nx + 2, ny + 2,
                             nz + 2, -0.5, -0.5, -0.5, 1.0, _ptr(out[s]), threads)
        vmax = max(vmax, m)
    out /= vmax
    try:
        np.save(path + ".tmp.npy", out)
        os.replace(path + ".tmp.npy", path)
    except OSError:
        pass
    return out


def turbulence_block(config: int, edge=256, fmt: int = F32, sub: int = 0, n_slices: int = 1,
                     slice_dt: float = 1.0, rank_grid=(4, 4, 4), rank_coord=(1, 1, 1),
                     dims=None) -> Block:
    """A rank's block in cell units: owned bounds [0,n), sample domain [-0.5, n+0.5]."""
    dims = tuple(dims) if dims is not None else (edge, edge, edge)
    b = Block(dims=dims, ghost=1, origin=(0.5, 0.5, 0.5), spacing=(1.0, 1.0, 1.0),
              lo=(0.0, 0.0, 0.0), hi=tuple(float(n) for n in dims), boundary=BOUNDARY_BLOCK,
              rank_grid=tuple(rank_grid), rank_coord=tuple(rank_coord), n_slices=n_slices,
              t0=0.0, slice_dt=slice_dt)
    b.values = turbulence_values(config, dims, sub=sub, n_slices=n_slices)
    return b.quantise(fmt)


def partition(blk: Block, parts) -> list:
    """Split a one-ghost-layer block into a px x py x pz grid of sub-blocks (x fastest), each
    holding its share of the interior nodes plus one ghost layer copied from the neighbouring
    nodes of the whole array, with owned bounds the matching share of the whole block's bounds
    and rank grid `parts`.  Every sub-block samples the whole field's interpolant on its domain.
    Interior node counts must divide evenly."""
    assert blk.ghost == 1 and blk.boundary == BOUNDARY_BLOCK
    parts = tuple(int(p) for p in parts)
    n = [d // p for d, p in zip(blk.dims, parts)]
    assert all(d == k * p for d, k, p in zip(blk.dims, n, parts)), "interior nodes must split evenly"
    out = []
    for k in range(parts[2]):
        for j in range(parts[1]):
            for i in range(parts[0]):
                c = (i, j, k)
                sl = tuple(slice(c[a] * n[a], c[a] * n[a] + n[a] + 2) for a in range(3))
                lo = tuple(blk.lo[a] + c[a] * n[a] * blk.spacing[a] for a in range(3))
                hi = tuple(blk.hi[a] if c[a] == parts[a] - 1 else blk.lo[a] + (c[a] + 1) * n[a] * blk.spacing[a]
                           for a in range(3))
                sub = dataclasses.replace(
                    blk, dims=tuple(n), lo=lo, hi=hi, rank_grid=parts, rank_coord=c,
                    origin=tuple(blk.origin[a] + c[a] * n[a] * blk.spacing[a] for a in range(3)),
                    values=np.ascontiguousarray(blk.values[:, sl[2], sl[1], sl[0]]),
                    stored=np.ascontiguousarray(blk.stored[:, sl[2], sl[1], sl[0]]))
                out.append(sub)
    return out


# ---------------------------------------------------------------------------
# Seeds
# ---------------------------------------------------------------------------
def uniform_seeds(config: int, n: int, lo, hi, sub: int = 0) -> np.ndarray:
    """n FP32 seeds uniform in [lo, hi) (24-bit grid, so exactly representable)."""
    out = np.empty((n, 3), np.float32)
    for a in range(3):
        u = uniform24(stream(config, P_SEEDS, sub * 3 + a), n)
        v = lo[a] + u * (hi[a] - lo[a])
        out[:, a] = v.astype(np.float32)
        # round-to-nearest can land on hi: keep the half-open interval
        bad = out[:, a] >= np.float32(hi[a])
        out[bad, a] = np.nextafter(np.float32(hi[a]), np.float32(lo[a]))
    return out


def blob_seeds(config: int, n_blobs: int, per_blob: int, edge: float, margin: float,
               sigma: float) -> np.ndarray:
    """Gaussian blobs: centres uniform in [margin, edge-margin)^3, points N(c, sigma^2 I),
    points outside [0, edge) redrawn from the next counters."""
    cs = np.stack([margin + uniform(stream(config, P_BLOB, a), n_blobs) * (edge - 2 * margin)
                   for a in range(3)], axis=1)
    out = np.empty((n_blobs * per_blob, 3), np.float32)
    for b in range(n_blobs):
        pts = np.empty((per_blob, 3), np.float64)
        need = np.arange(per_blob)
        draw = 0
        while need.size:
            for a in range(3):
                strm = stream(config, P_BLOB, 1000 + b * 3 + a)
                pts[need, a] = cs[b, a] + sigma * normal(strm, need.size, first=draw)
            draw += per_blob
            f = pts[need].astype(np.float32)
            inside = np.all((f >= 0) & (f < np.float32(edge)), axis=1)
            need = need[~inside]
        out[b * per_blob:(b + 1) * per_blob] = pts.astype(np.float32)
    return out


def int_uniform(config: int, purpose: int, n: int, lo: int, hi: int, sub: int = 0) -> np.ndarray:
    """n integers uniform in {lo..hi} (inclusive)."""
    u = uniform(stream(config, purpose, sub), n)
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64).clip(lo, hi)


# ---------------------------------------------------------------------------
# Learned flow-map surrogate: initial weights and training samples
# ---------------------------------------------------------------------------
MLP_WIDTHS = (3, 256, 256, 256, 256, 3)


def mlp_init(config: int = 5, widths=MLP_WIDTHS, sub: int = 0):
    """Initial parameters, U(-1/sqrt(fan_in), 1/sqrt(fan_in)), FP32: list of (W [out, in], b [out])."""
    params = []
    for l in range(len(widths) - 1):
        fi, fo = widths[l], widths[l + 1]
        r = 1.0 / np.sqrt(fi)
        w = (uniform(stream(config, P_MLP, sub * 64 + 2 * l), fo * fi) * 2 - 1) * r
        b = (uniform(stream(config, P_MLP, sub * 64 + 2 * l + 1), fo) * 2 - 1) * r
        params.append((w.reshape(fo, fi).astype(np.float32), b.astype(np.float32)))
    return params


def training_starts(config: int, n: int, period: float, sub: int = 0) -> np.ndarray:
    """n FP32 start points uniform in [0, period)^3 for flow-map training windows."""
    return uniform_seeds(config, n, (0, 0, 0), (period,) * 3, sub=1000 + sub)


# ---------------------------------------------------------------------------
# Batched uneven blocks
# ---------------------------------------------------------------------------
def batched_blocks(config: int = 4, n_blocks: int = 96, edge_lo: int = 32, edge_hi: int = 192,
                   fmt: int = F16, n_slices: int = 1, n_modes: int = 512, h: float = 0.5,
                   m_lo: int = 100, m_hi: int = 5000, seeds_lo: int = 1024, seeds_hi: int = 65536,
                   seed_scale: float = 1.0):
    """Independent turbulence blocks with uneven shapes and seed sets.

    Each axis edge ~ U{edge_lo..edge_hi}; each block its own generator
    realisation (sub-stream b), normalised per block; seeds per block
    round(exp(U[ln seeds_lo, ln seeds_hi])) * seed_scale, uniform in the block;
    per-seed step limits ~ U{m_lo..m_hi}.  With n_slices > 1 the slices are
    spaced slice_dt = m_hi*h/(n_slices-1) so the longest seeds span them all.
    Returns (blocks, seeds per block, max steps per block).
    """
    edges = int_uniform(config, P_BLOCKSHAPE, n_blocks * 3, edge_lo, edge_hi).reshape(n_blocks, 3)
    counts = np.round(np.exp(np.log(seeds_lo) + uniform(stream(config, P_NSEEDS), n_blocks)
                             * (np.log(seeds_hi) - np.log(seeds_lo))) * seed_scale).astype(np.int64)
    counts = np.maximum(counts, 1)
    slice_dt = m_hi * h / (n_slices - 1) if n_slices > 1 else 1.0
    blocks, seeds, limits = [], [], []
    for b in range(n_blocks):
        dims = tuple(int(v) for v in edges[b])
        blk = Block(dims=dims, ghost=1, origin=(0.5, 0.5, 0.5), spacing=(1.0, 1.0, 1.0), lo=(0.0, 0.0, 0.0),
                    hi=tuple(float(v) for v in dims), boundary=BOUNDARY_BLOCK, rank_grid=(1, 1, 1),
                    rank_coord=(0, 0, 0), n_slices=n_slices, t0=0.0, slice_dt=slice_dt)
        blk.values = turbulence_values(config, dims, sub=b, n_slices=n_slices, n_modes=n_modes)
        blocks.append(blk.quantise(fmt))
        seeds.append(uniform_seeds(config, int(counts[b]), (0, 0, 0), dims, sub=10 + b))
        limits.append(int_uniform(config, P_MAXSTEPS, int(counts[b]), m_lo, m_hi, sub=b).astype(np.int32))
    return blocks, seeds, limits


def streakline_particles(emitters: np.ndarray, limits: np.ndarray, every: int, h: float):
    """Particles released by emitters every `every` steps: emitter e releases at steps
    0, every, 2*every, ... < limits[e]; the particle born at step b runs to step
    limits[e] (limit limits[e] - b) from time b*h.  Returned emitter-major,
    birth-minor: (positions, birth times, step limits, emitter index)."""
    births = [np.arange(0, int(m), every) for m in limits]
    emi = np.concatenate([np.full(len(b), e, np.int64) for e, b in enumerate(births)])
    bsteps = np.concatenate(births)
    pos = np.ascontiguousarray(emitters[emi], np.float32)
    tb = (bsteps * h).astype(np.float32)
    lim = (np.asarray(limits)[emi] - bsteps).astype(np.int32)
    return pos, tb, lim, emi


# ---------------------------------------------------------------------------
# Hexahedral meshes (unstructured field inputs): vertices, per-vertex values and
# cells of 8 vertex indices in VTK hexahedron order
# ---------------------------------------------------------------------------
VTK_HEX_CORNERS = ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1))


def _lattice_cells(nx, ny, nz):
    """Cells of an nx x ny x nz lattice of vertices (x fastest), VTK order, int32 [cells, 8]."""
    k, j, i = np.meshgrid(np.arange(nz - 1), np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    return np.stack([(i + a) + nx * ((j + b) + ny * (k + c)) for a, b, c in VTK_HEX_CORNERS], 1).astype(np.int32)


def hex_mesh_from_block(blk: Block) -> dict:
    """Every cell of a steady FP32 block's stored grid as a hexahedron (the paper's conversion of
    voxel data to an unstructured field): vertices = the stored nodes' world positions, values
    = the stored node values, same owned bounds and rank grid."""
    assert blk.n_slices == 1 and blk.fmt == F32 and blk.boundary == BOUNDARY_BLOCK
    nx, ny, nz = (d + 2 * blk.ghost for d in blk.dims)
    xs, ys, zs = (_node_coords(d, o, s, blk.ghost) for d, o, s in zip(blk.dims, blk.origin, blk.spacing))
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)
    return dict(vertices=verts, values=np.ascontiguousarray(blk.stored[0].reshape(-1, 3), np.float32),
                cells=_lattice_cells(nx, ny, nz), lo=tuple(blk.lo), hi=tuple(blk.hi),
                rank_grid=tuple(blk.rank_grid), rank_coord=tuple(blk.rank_coord))


# VTK cell type codes of the unstructured meshes
VTK_TETRA, VTK_HEXAHEDRON, VTK_WEDGE, VTK_PYRAMID = 10, 12, 13, 14
_VTK_HEX_INDEX = {c: i for i, c in enumerate(VTK_HEX_CORNERS)}  # corner bits (x, y, z) -> VTK vertex
# six tetrahedra around the diagonal (0,0,0)-(1,1,1) of a cube, one per order of the axes
# (the Kuhn / Freudenthal subdivision: neighbouring cubes split shared faces alike)
_KUHN = []
for _ax in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
    _p = [0, 0, 0]
    _path = [tuple(_p)]
    for _a in _ax:
        _p[_a] = 1
        _path.append(tuple(_p))
    _KUHN.append([_VTK_HEX_INDEX[q] for q in _path])
# two wedges: bottom and top quads split along the diagonal (0,0)-(1,1)
_WEDGES = [[0, 1, 2, 4, 5, 6], [0, 2, 3, 4, 6, 7]]
# six faces of a cube (VTK vertex indices, each in cyclic order) as pyramid bases around the centre
_FACES = [[0, 1, 2, 3], [4, 7, 6, 5], [0, 4, 5, 1], [3, 2, 6, 7], [0, 3, 7, 4], [1, 5, 6, 2]]


def split_hex_mesh(mesh: dict, kind: str) -> dict:
    """Every hexahedron of a lattice mesh (hex_mesh_from_block, distorted_hex_mesh) split into
    conforming cells of other kinds: "tetra" (6 per cube, Kuhn subdivision), "wedge" (2 per
    cube), "pyramid" (6 per cube around a new centre vertex: the mean of the cube's corners,
    value the mean of their values, FP32), "hex+pyramid" (a checkerboard of whole cubes and
    cubes of 6 pyramids; a pyramid base is a whole cube face, so neighbours interpolate
    alike on it).  cells: [n, 8] int32, each row the cell's vertices in VTK order and -1 after
    them; cell_types: [n] uint8 VTK codes.  Same bounds and rank grid."""
    cells = np.asarray(mesh["cells"], np.int64)
    V = np.asarray(mesh["vertices"], np.float64)
    W = np.asarray(mesh["values"], np.float64)
    out_cells, out_types = [], []
    verts, vals = [mesh["vertices"]], [mesh["values"]]
    n_v = len(V)
    if kind == "hex+pyramid":
        c0 = V[cells[:, 0]]
        parity = np.floor(c0 + 0.5).astype(np.int64).sum(axis=1) % 2 if len(cells) else np.zeros(0, np.int64)
    for c, row in enumerate(cells):
        if kind == "tetra":
            for t in _KUHN:
                out_cells.append(list(row[t]) + [-1] * 4)
                out_types.append(VTK_TETRA)
        elif kind == "wedge":
            for w in _WEDGES:
                out_cells.append(list(row[w]) + [-1] * 2)
                out_types.append(VTK_WEDGE)
        elif kind == "pyramid" or (kind == "hex+pyramid" and parity[c] == 1):
            centre = n_v + len(verts) - 1
            verts.append(V[row].mean(axis=0, keepdims=True).astype(np.float32))
            vals.append(W[row].mean(axis=0, keepdims=True).astype(np.float32))
            for f in _FACES:
                out_cells.append(list(row[f]) + [centre] + [-1] * 3)
                out_types.append(VTK_PYRAMID)
        elif kind == "hex+pyramid":
            out_cells.append(list(row))
            out_types.append(VTK_HEXAHEDRON)
        else:
            raise ValueError(kind)
    return dict(mesh, vertices=np.ascontiguousarray(np.concatenate(verts), np.float32),
                values=np.ascontiguousarray(np.concatenate(vals), np.float32),
                cells=np.asarray(out_cells, np.int32).reshape(-1, 8),
                cell_types=np.asarray(out_types, np.uint8))


def distorted_hex_mesh(config: int, dims, jitter: float = 0.2, sub: int = 0, field=None) -> dict:
    """A conforming mesh of dims = (cx, cy, cz) hexahedra over [0, cx] x [0, cy] x [0, cz]: a unit
    lattice whose vertices move by up to `jitter` (uniform, per coordinate; vertices on the
    box's faces stay on them), so cells are general (non-affine) hexahedra.  Values: field(x, y,
    z) -> (vx, vy, vz) at the vertices (default a smooth divergence-free rotation-like flow),
    FP32.  Owned bounds: the box."""
    cx, cy, cz = (int(d) for d in dims)
    nx, ny, nz = cx + 1, cy + 1, cz + 1
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(np.float64)
    jit = (uniform(stream(config, P_HEXJIT, sub), base.size).reshape(-1, 3) * 2 - 1) * jitter
    for a, n in enumerate((nx, ny, nz)):  # keep face vertices on their faces
        on = (base[:, a] == 0) | (base[:, a] == n - 1)
        jit[on, a] = 0.0
    verts = (base + jit).astype(np.float32)
    if field is None:
        def field(x, y, z):
            return (np.sin(0.4 * z) + 0.5 * np.cos(0.3 * y), 0.6 * np.sin(0.35 * x) + 0.4 * np.cos(0.25 * z),
                    0.5 * np.sin(0.3 * y) + 0.45 * np.cos(0.4 * x))
    v = np.stack(field(*verts.astype(np.float64).T), 1)
    return dict(vertices=verts, values=v.astype(np.float32), cells=_lattice_cells(nx, ny, nz),
                lo=(0.0, 0.0, 0.0), hi=(float(cx), float(cy), float(cz)), rank_grid=(1, 1, 1), rank_coord=(0, 0, 0))
