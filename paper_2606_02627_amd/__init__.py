"""Python binding of libstreami (MI355X/gfx950 field-line advection).

Argument marshalling only: every function below calls the C-ABI entry point
of the same name in ``libstreami.so`` (declared in ``include/streami.h``).
Arrays may be numpy arrays (host memory) or torch tensors (host or device);
the HIP stream defaults to torch's current stream.  There is no CPU fallback:
importing this package fails if the HIP library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # torch first: its HIP runtime is the one libstreami binds to
    import torch
except ImportError:  # pragma: no cover - torch is part of the supported environment
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstreami.so")

OK, E_ARG, E_NOMEM, E_DEVICE, E_STATE, E_CAPACITY, E_UNSUPPORTED, E_IO = range(8)
SHAPE_LINE, SHAPE_PLANE = 0, 1
F32, F16, BF16 = 0, 1, 2
BOUNDARY_BLOCK, BOUNDARY_PERIODIC = 0, 1
ACTIVE, MAX_STEPS, EXIT, STAGNANT, HALO_MISS, NONFINITE = range(6)
LAYOUT_AUTO, LAYOUT_LINEAR, LAYOUT_BRICK4, LAYOUT_CELL, LAYOUT_HEX, LAYOUT_BRICK8 = 0, 1, 2, 3, 4, 5
MODE_PLAIN, MODE_SURROGATE = 0, 1


class StreamiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"streami error {code}: {msg}")
        self.code = code


class BlockDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("ghost", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3),
                ("bounds_lo", ctypes.c_double * 3), ("bounds_hi", ctypes.c_double * 3),
                ("boundary", ctypes.c_int32), ("rank_grid", ctypes.c_int32 * 3),
                ("rank_coord", ctypes.c_int32 * 3), ("n_slices", ctypes.c_int32),
                ("t0", ctypes.c_double), ("slice_dt", ctypes.c_double),
                ("nodes", ctypes.c_void_p), ("nodes_on_device", ctypes.c_int32)]


class HexDesc(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("vertices", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("n_cells", ctypes.c_int64), ("cells", ctypes.c_void_p), ("bounds_lo", ctypes.c_double * 3),
                ("bounds_hi", ctypes.c_double * 3), ("rank_grid", ctypes.c_int32 * 3),
                ("rank_coord", ctypes.c_int32 * 3), ("inputs_on_device", ctypes.c_int32),
                ("cell_types", ctypes.c_void_p)]


class FieldOpts(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32)]


class SeedOpts(ctypes.Structure):
    _fields_ = [("default_max_steps", ctypes.c_int32), ("record_stride", ctypes.c_int32),
                ("inputs_on_device", ctypes.c_int32), ("t_birth", ctypes.c_float),
                ("t_births", ctypes.c_void_p)]


class SeedBatch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("ids", ctypes.c_void_p),
                ("max_steps", ctypes.c_void_p), ("t_births", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Shape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("origin", ctypes.c_double * 3), ("u", ctypes.c_double * 3),
                ("v", ctypes.c_double * 3), ("nu", ctypes.c_int64), ("nv", ctypes.c_int64)]


class AdvectParams(ctypes.Structure):
    _fields_ = [("h", ctypes.c_float), ("step_budget", ctypes.c_int32),
                ("stagnation_eps", ctypes.c_float), ("mode", ctypes.c_int32),
                ("mlp", ctypes.c_void_p), ("residual_tol_cells", ctypes.c_float),
                ("residual_kind", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("refill_threshold", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("no_cell_cache", ctypes.c_int32), ("work_order", ctypes.c_int32),
                ("use_t_end", ctypes.c_int32), ("t_end", ctypes.c_float),
                ("checked_samples", ctypes.c_int32), ("lds_cell_cache", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("vertices", ctypes.c_int64), ("outbox", ctypes.c_int64),
                ("surrogate_accepted", ctypes.c_int64), ("surrogate_fallback", ctypes.c_int64),
                ("terminated", ctypes.c_int64 * 6), ("device_ms", ctypes.c_double),
                ("gathers", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "terminated"}
        d["terminated"] = list(self.terminated)
        return d


OUTBOX_DTYPE = np.dtype([("id", "<u8"), ("pos", "<f4", (3,)), ("steps", "<i4"), ("dest", "<i4"),
                         ("code", "<i2"), ("block", "<i2")])
assert OUTBOX_DTYPE.itemsize == 32

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "streami_field_create": [vp, i32, i32, vp, vp, vp],
        "streami_field_destroy": [vp],
        "streami_field_create_hex": [vp, vp, vp],
        "streami_seed": [vp, i32, vp, vp, vp, i64, vp],
        "streami_seed_batches": [vp, vp, i32, vp],
        "streami_seed_shape": [vp, i32, vp, vp, vp],
        "streami_write_obj": [ctypes.c_char_p, i64, vp, vp, i32, vp],
        "streami_write_obj_field": [vp, ctypes.c_char_p],
        "streami_advect": [vp, vp, vp],
        "streami_fetch_lines": [vp, i32, i64, i64, vp, vp, i64, vp, vp, vp, vp],
        "streami_fetch_outbox": [vp, vp, i64, vp],
        "streami_block_info": [vp, i32, vp, vp],
        "streami_field_info": [vp, vp, vp],
        "streami_clear": [vp],
        "streami_forward": [vp, vp, vp],
        "streami_trace": [vp, vp, i32, vp, vp],
        "streami_mlp_create": [vp, vp, ctypes.c_float, vp, vp],
        "streami_mlp_destroy": [vp],
        "streami_mlp_set_params": [vp, vp],
        "streami_mlp_get_params": [vp, vp],
        "streami_mlp_forward": [vp, vp, i64, vp],
        "streami_mlp_train_step": [vp, vp, vp, i64, ctypes.c_float, vp, vp],
        "streami_mlp_train_step_noalloc": [vp, vp, vp, i64, ctypes.c_float, vp, vp],
        "streami_probe_gather": [vp, i64, i32, i32, i32, i32, vp, vp, vp],
        "streami_probe_valu": [i32, i32, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.streami_last_error.restype = ctypes.c_char_p
    lib.streami_last_error.argtypes = []
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise StreamiError(rc, _load().streami_last_error().decode(errors="replace"))
    return rc


def _addr(a):
    """(pointer, on_device) of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None, False
    if torch is not None and isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), a.is_cuda
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return ctypes.c_void_p(a.ctypes.data), False
    raise TypeError(f"unsupported array type {type(a)}")


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    if torch is not None and torch.cuda.is_available():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


def make_block_desc(blk, nodes=None):
    """BlockDesc from a duck-typed block (dims, ghost, origin, spacing, lo, hi, boundary,
    rank_grid, rank_coord, n_slices, t0, slice_dt) and its stored nodes."""
    d = BlockDesc()
    d.dims[:] = [int(v) for v in blk.dims]
    d.ghost = int(blk.ghost)
    d.origin[:] = [float(v) for v in blk.origin]
    d.spacing[:] = [float(v) for v in blk.spacing]
    d.bounds_lo[:] = [float(v) for v in blk.lo]
    d.bounds_hi[:] = [float(v) for v in blk.hi]
    d.boundary = int(blk.boundary)
    d.rank_grid[:] = [int(v) for v in blk.rank_grid]
    d.rank_coord[:] = [int(v) for v in blk.rank_coord]
    d.n_slices = int(blk.n_slices)
    d.t0 = float(blk.t0)
    d.slice_dt = float(blk.slice_dt)
    arr = blk.stored if nodes is None else nodes
    ptr, dev = _addr(arr)
    d.nodes = ptr.value if ptr is not None else None
    d.nodes_on_device = int(dev)
    return d


# ---------------------------------------------------------------- C-ABI calls
def streami_field_create(descs, dtype, layout=LAYOUT_AUTO, stream=None):
    arr = (BlockDesc * len(descs))(*descs)
    opts = FieldOpts(layout=layout)
    out = ctypes.c_void_p()
    _check(_load().streami_field_create(arr, len(descs), dtype, ctypes.byref(opts), _stream(stream),
                                        ctypes.byref(out)))
    return out


def streami_field_create_hex(mesh, stream=None):
    """Handle over an unstructured field: mesh = dict(vertices [nv,3] f32, values [nv,3] f32, cells
    [nc,8] int32 (VTK order), optional cell_types [nc] uint8 (VTK codes; absent: hexahedra), lo,
    hi, rank_grid, rank_coord), all host or all device arrays."""
    arrs = [mesh["vertices"], mesh["values"], mesh["cells"]]
    types = mesh.get("cell_types")
    if types is not None:
        arrs.append(types)
    if isinstance(arrs[0], np.ndarray):
        conv = [np.float32, np.float32, np.int32, np.uint8]
        arrs = [np.ascontiguousarray(a, t) for a, t in zip(arrs, conv)]
    ptrs = [_addr(a) for a in arrs]
    if len({d for _, d in ptrs}) != 1:
        raise ValueError("vertices, values, cells and cell_types must all be host or all device arrays")
    d = HexDesc(n_vertices=int(arrs[0].shape[0]), n_cells=int(arrs[2].shape[0]),
                inputs_on_device=int(ptrs[0][1]))
    d.vertices, d.values, d.cells = (p.value for p, _ in ptrs[:3])
    d.cell_types = ptrs[3][0].value if types is not None else None
    d.bounds_lo[:] = [float(v) for v in mesh["lo"]]
    d.bounds_hi[:] = [float(v) for v in mesh["hi"]]
    d.rank_grid[:] = [int(v) for v in mesh.get("rank_grid", (1, 1, 1))]
    d.rank_coord[:] = [int(v) for v in mesh.get("rank_coord", (0, 0, 0))]
    out = ctypes.c_void_p()
    _check(_load().streami_field_create_hex(ctypes.byref(d), _stream(stream), ctypes.byref(out)))
    return out


def streami_field_destroy(f):
    return _check(_load().streami_field_destroy(f))


def streami_seed(f, block, xyz, ids=None, max_steps=None, default_max_steps=0, record_stride=1,
                 t_birth=0.0, t_births=None):
    px, dx = _addr(xyz)
    pi, di = _addr(ids)
    pm, dm = _addr(max_steps)
    pt, dt = _addr(t_births)
    on_dev = dx
    if ((ids is not None and di != on_dev) or (max_steps is not None and dm != on_dev)
            or (t_births is not None and dt != on_dev)):
        raise ValueError("xyz, ids, max_steps and t_births must all be host or all device arrays")
    n = (xyz.numel() if hasattr(xyz, "numel") else xyz.size) // 3
    opts = SeedOpts(default_max_steps=int(default_max_steps), record_stride=int(record_stride),
                    inputs_on_device=int(on_dev), t_birth=float(t_birth),
                    t_births=None if pt is None else pt.value)
    return _check(_load().streami_seed(f, int(block), px, pi, pm, int(n), ctypes.byref(opts)))


def streami_seed_batches(f, batches, default_max_steps=0, record_stride=1, t_birth=0.0):
    """Seed several batches with shared options; each batch is a dict with block, xyz and
    optionally ids, max_steps, t_births (all host or all device arrays, like streami_seed)."""
    arr = (SeedBatch * max(1, len(batches)))()
    on_dev = None
    for k, b in enumerate(batches):
        xyz = b["xyz"]
        px, dx = _addr(xyz)
        parts = [_addr(b.get(key)) for key in ("ids", "max_steps", "t_births")]
        for key, (_, d) in zip(("ids", "max_steps", "t_births"), parts):
            if b.get(key) is not None and d != dx:
                raise ValueError("a batch's arrays must all be host or all device arrays")
        if on_dev is None:
            on_dev = dx
        elif dx != on_dev:
            raise ValueError("all batches must be host or all device arrays")
        n = (xyz.numel() if hasattr(xyz, "numel") else xyz.size) // 3
        arr[k].block = int(b["block"])
        arr[k].xyz = px.value
        arr[k].ids, arr[k].max_steps, arr[k].t_births = (None if p is None else p.value for p, _ in parts)
        arr[k].n = int(n)
    opts = SeedOpts(default_max_steps=int(default_max_steps), record_stride=int(record_stride),
                    inputs_on_device=int(bool(on_dev)), t_birth=float(t_birth), t_births=None)
    return _check(_load().streami_seed_batches(f, arr, len(batches), ctypes.byref(opts)))


def streami_seed_shape(f, block, kind, origin, u, v=(0.0, 0.0, 0.0), nu=1, nv=1, max_steps=None,
                       default_max_steps=0, record_stride=1, t_birth=0.0, t_births=None):
    """Seed an nu x nv midpoint grid on a line (origin, origin + u) or a parallelogram
    (origin, edges u and v), generated on the device."""
    sh = Shape(kind=int(kind), nu=int(nu), nv=int(nv))
    sh.origin[:] = [float(c) for c in origin]
    sh.u[:] = [float(c) for c in u]
    sh.v[:] = [float(c) for c in v]
    pm, dm = _addr(max_steps)
    pt, dt = _addr(t_births)
    if max_steps is not None and t_births is not None and dm != dt:
        raise ValueError("max_steps and t_births must both be host or both device arrays")
    on_dev = dm if max_steps is not None else dt
    opts = SeedOpts(default_max_steps=int(default_max_steps), record_stride=int(record_stride),
                    inputs_on_device=int(bool(on_dev)), t_birth=float(t_birth),
                    t_births=None if pt is None else pt.value)
    return _check(_load().streami_seed_shape(f, int(block), ctypes.byref(sh), pm, ctypes.byref(opts)))


def streami_write_obj(path, offsets, xyz, append=False, vertex_base=0):
    """Write CSR lines (host arrays) as an OBJ file; returns the vertex count after this call."""
    off = np.ascontiguousarray(offsets, np.int64)
    pts = np.ascontiguousarray(xyz, np.float32)
    base = ctypes.c_int64(int(vertex_base))
    _check(_load().streami_write_obj(os.fsencode(path), len(off) - 1, _addr(off)[0], _addr(pts)[0], int(append),
                                     ctypes.byref(base)))
    return base.value


def streami_write_obj_field(f, path):
    return _check(_load().streami_write_obj_field(f, os.fsencode(path)))


def streami_advect(f, params: AdvectParams, want_stats=True):
    st = Stats() if want_stats else None
    _check(_load().streami_advect(f, ctypes.byref(params), ctypes.byref(st) if st else None))
    return st


def streami_fetch_lines(f, block, first, count, offsets, xyz, cap_vertices, steps=None, codes=None,
                        ids=None):
    needed = ctypes.c_int64()
    rc = _load().streami_fetch_lines(f, int(block), int(first), int(count), _addr(offsets)[0],
                                     _addr(xyz)[0], int(cap_vertices), _addr(steps)[0],
                                     _addr(codes)[0], _addr(ids)[0], ctypes.byref(needed))
    if rc == E_CAPACITY:
        return rc, needed.value
    _check(rc)
    return rc, needed.value


def streami_fetch_outbox(f, out, cap):
    n = ctypes.c_int64()
    rc = _load().streami_fetch_outbox(f, _addr(out)[0], int(cap), ctypes.byref(n))
    if rc != E_CAPACITY:
        _check(rc)
    return rc, n.value


def streami_clear(f):
    return _check(_load().streami_clear(f))


def streami_forward(f):
    """Loopback exchange of the outbox between the handle's blocks: (forwarded, active)."""
    fw, act = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().streami_forward(f, ctypes.byref(fw), ctypes.byref(act)))
    return fw.value, act.value


def streami_trace(f, params: AdvectParams, max_rounds=1 << 20, want_stats=True):
    """Advect and forward until no particle is active: (rounds, stats or None)."""
    st = Stats() if want_stats else None
    r = ctypes.c_int32()
    _check(_load().streami_trace(f, ctypes.byref(params), int(max_rounds), ctypes.byref(r),
                                 ctypes.byref(st) if st else None))
    return r.value, st


def streami_probe_gather(buf, record_bytes, loads_per_lane, in_flight=4, waves_per_cu=16, stream=None):
    """Random record gathers over a device tensor: (ms of the timed launch, records read)."""
    ptr, dev = _addr(buf)
    if not dev:
        raise ValueError("the probe reads device memory")
    ms, n = ctypes.c_float(), ctypes.c_int64()
    _check(_load().streami_probe_gather(ptr, buf.numel() * buf.element_size(), int(record_bytes),
                                        int(loads_per_lane), int(in_flight), int(waves_per_cu), _stream(stream),
                                        ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def streami_probe_valu(kind, waves_per_cu=32, stream=None):
    """VALU issue-rate probe (kind 0 v_fma_f32, 1 v_add_u32, 2 v_exp_f32, 3 v_rcp_f32): (ms, wave-level
    instructions)."""
    ms, n = ctypes.c_float(), ctypes.c_int64()
    _check(_load().streami_probe_valu(int(kind), int(waves_per_cu), _stream(stream), ctypes.byref(ms),
                                      ctypes.byref(n)))
    return ms.value, n.value


def streami_field_info(f):
    """(layout in use, device bytes of the stored field)."""
    lay, nb = ctypes.c_int32(), ctypes.c_int64()
    _check(_load().streami_field_info(f, ctypes.byref(lay), ctypes.byref(nb)))
    return lay.value, nb.value


def streami_block_info(f, block):
    n, v = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().streami_block_info(f, int(block), ctypes.byref(n), ctypes.byref(v)))
    return n.value, v.value


def advect_params(h, step_budget=0, eps=1e-6, **kw):
    p = AdvectParams()
    p.h = float(h)
    p.step_budget = int(step_budget)
    p.stagnation_eps = float(eps)
    p.mode = kw.pop("mode", MODE_PLAIN)
    net = kw.pop("mlp", None)
    p.mlp = net.value if isinstance(net, ctypes.c_void_p) else net
    t_end = kw.pop("t_end", None)
    if t_end is not None:
        p.use_t_end, p.t_end = 1, float(t_end)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------- convenience
class Field:
    """Owning wrapper around a field handle (marshalling only)."""

    def __init__(self, blocks, dtype, layout=LAYOUT_AUTO, stream=None, nodes=None):
        blocks = list(blocks)
        nodes = nodes if nodes is not None else [None] * len(blocks)
        self._descs = [make_block_desc(b, n) for b, n in zip(blocks, nodes)]
        self.h = streami_field_create(self._descs, dtype, layout, stream)
        self.n_blocks = len(blocks)

    @classmethod
    def hex(cls, mesh, stream=None):
        """A handle over a hexahedral field (streami_field_create_hex)."""
        f = cls.__new__(cls)
        f._descs = []
        f.h = streami_field_create_hex(mesh, stream)
        f.n_blocks = 1
        return f

    def close(self):
        if self.h is not None and self.h.value:
            streami_field_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self):
        return streami_clear(self.h)

    def seed(self, block, xyz, **kw):
        return streami_seed(self.h, block, xyz, **kw)

    def seed_batches(self, batches, **kw):
        return streami_seed_batches(self.h, batches, **kw)

    def seed_shape(self, block, kind, origin, u, v=(0.0, 0.0, 0.0), nu=1, nv=1, **kw):
        return streami_seed_shape(self.h, block, kind, origin, u, v, nu, nv, **kw)

    def write_obj(self, path):
        return streami_write_obj_field(self.h, path)

    def advect(self, h, **kw):
        return streami_advect(self.h, advect_params(h, **kw))

    def forward(self):
        return streami_forward(self.h)

    def trace(self, h, max_rounds=1 << 20, **kw):
        return streami_trace(self.h, advect_params(h, **kw), max_rounds)

    def lines(self, block=0, first=0, count=None):
        """Lines of a block in seed order (host numpy CSR)."""
        n, _ = streami_block_info(self.h, block)
        count = n - first if count is None else count
        rc, need = streami_fetch_lines(self.h, block, first, count, None, None, -1)
        off = np.zeros(count + 1, np.int64)
        xyz = np.zeros((max(need, 1), 3), np.float32)
        steps = np.zeros(count, np.int32)
        codes = np.zeros(count, np.int32)
        ids = np.zeros(count, np.uint64)
        streami_fetch_lines(self.h, block, first, count, off, xyz, need, steps, codes, ids)
        return dict(offsets=off, xyz=xyz[:need], steps=steps, codes=codes, ids=ids)

    def outbox(self, cap=None):
        if cap is None:
            cap = 1 << 16
        recs = []
        while True:
            buf = np.zeros(cap, OUTBOX_DTYPE)
            rc, n = streami_fetch_outbox(self.h, buf, cap)
            recs.append(buf[:n])
            if rc != E_CAPACITY:
                break
        return np.concatenate(recs)


# ---------------------------------------------------------------- surrogate network
MLP_WIDTHS = (3, 256, 256, 256, 256, 3)
MLP_N_PARAMS = sum(MLP_WIDTHS[i] * MLP_WIDTHS[i + 1] + MLP_WIDTHS[i + 1] for i in range(5))


def flatten_params(params):
    """[(W, b), ...] -> flat FP32 array in the library's parameter order."""
    return np.ascontiguousarray(np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(),
                                                                np.asarray(b, np.float32).ravel()])
                                                for W, b in params]), np.float32)


def unflatten_params(flat):
    out, off = [], 0
    for i in range(5):
        fi, fo = MLP_WIDTHS[i], MLP_WIDTHS[i + 1]
        W = flat[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = flat[off:off + fo]
        off += fo
        out.append((W, b))
    return out


def streami_mlp_create(params, sigma, period, stream=None):
    flat = flatten_params(params) if isinstance(params, (list, tuple)) else np.ascontiguousarray(params, np.float32)
    assert flat.size == MLP_N_PARAMS
    sig = np.ascontiguousarray(sigma, np.float32)
    out = ctypes.c_void_p()
    _check(_load().streami_mlp_create(_addr(flat)[0], _addr(sig)[0], float(period), _stream(stream),
                                      ctypes.byref(out)))
    return out


def streami_mlp_destroy(m):
    return _check(_load().streami_mlp_destroy(m))


def streami_mlp_get_params(m):
    flat = np.zeros(MLP_N_PARAMS, np.float32)
    _check(_load().streami_mlp_get_params(m, _addr(flat)[0]))
    return flat


def streami_mlp_set_params(m, params):
    flat = flatten_params(params) if isinstance(params, (list, tuple)) else np.ascontiguousarray(params, np.float32)
    return _check(_load().streami_mlp_set_params(m, _addr(flat)[0]))


def streami_mlp_forward(m, xyz, out):
    n = xyz.numel() // 3
    return _check(_load().streami_mlp_forward(m, _addr(xyz)[0], int(n), _addr(out)[0]))


def streami_mlp_train_step(m, xyz, target, lr, want_loss=True, want_grads=False):
    n = xyz.numel() // 3
    loss = ctypes.c_float()
    grads = np.zeros(MLP_N_PARAMS, np.float32) if want_grads else None
    _check(_load().streami_mlp_train_step(m, _addr(xyz)[0], _addr(target)[0], int(n), float(lr),
                                          ctypes.byref(loss) if want_loss else None,
                                          _addr(grads)[0] if want_grads else None))
    return (loss.value if want_loss else None), grads


MLP_NOALLOC_MAX_BATCH = 8192  # STREAMI_MLP_NOALLOC_MAX_BATCH


def streami_mlp_train_step_noalloc(m, xyz, target, lr, want_loss=True, want_grads=False):
    """streami_mlp_train_step on the library's static per-device workspace (no allocation in
    the call; at most MLP_NOALLOC_MAX_BATCH rows)."""
    n = xyz.numel() // 3
    loss = ctypes.c_float()
    grads = np.zeros(MLP_N_PARAMS, np.float32) if want_grads else None
    _check(_load().streami_mlp_train_step_noalloc(m, _addr(xyz)[0], _addr(target)[0], int(n), float(lr),
                                                  ctypes.byref(loss) if want_loss else None,
                                                  _addr(grads)[0] if want_grads else None))
    return (loss.value if want_loss else None), grads
