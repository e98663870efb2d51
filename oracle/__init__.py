"""FP64 CPU oracle for rank-local RK4 field-line advection -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.

``oracle.c`` holds the advection oracle (sample(), destinationID(), the RK4
update with its termination rules, whole trajectories); ``mlp.py`` holds the
FP64 network oracle of the learned flow-map form.  Both are plain definitions,
written from the paper (Sec. 3.1.1 sampling/forwarding, Sec. 3.1.2 update
kernel, Sec. 3.2 streamlines/streaklines and one field per time step, Sec. 3.3
structured fields).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
# a test may point this at a deliberately mutated build to check that the pins catch it
_LIB_PATH = os.environ.get("STREAMI_ORACLE_LIB", _DEFAULT_LIB)
_lib = None

ACTIVE, MAX_STEPS, EXIT, STAGNANT, HALO_MISS, NONFINITE = range(6)
FMT_F32, FMT_F16, FMT_BF16, FMT_F64 = 0, 1, 2, 3
FIELD_GRID, FIELD_ABC = 0, 1


def build(verbose: bool = False, src: str = None, out: str = None) -> str:
    """Compile liboracle.so: plain C, -O2, no fast-math, no contraction."""
    src = src or os.path.join(_HERE, "oracle.c")
    out = out or _DEFAULT_LIB
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-pthread", src, "-o", out, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return out


class _Block(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("ghost", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("periodic", ctypes.c_int32), ("rank_grid", ctypes.c_int32 * 3),
                ("rank_coord", ctypes.c_int32 * 3), ("n_slices", ctypes.c_int32),
                ("t0", ctypes.c_double), ("slice_dt", ctypes.c_double),
                ("nodes", ctypes.c_void_p), ("fmt", ctypes.c_int32),
                ("field_kind", ctypes.c_int32), ("abc", ctypes.c_double * 3)]


class _TraceIO(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("seeds", "max_steps", "t_birth", "steps", "code", "final_pos", "n_verts",
                 "verts", "in_outbox", "out_pos", "out_dest")]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    lib.orc_sizeof_block.restype = ctypes.c_int32
    lib.orc_sizeof_io.restype = ctypes.c_int32
    assert lib.orc_sizeof_block() == ctypes.sizeof(_Block), "oracle block struct mismatch"
    assert lib.orc_sizeof_io() == ctypes.sizeof(_TraceIO), "oracle io struct mismatch"
    lib.orc_sample_batch.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.orc_sample_batch.restype = None
    lib.orc_dest_batch.argtypes = [vp, i64, vp, vp]
    lib.orc_dest_batch.restype = None
    lib.orc_step_batch.argtypes = [vp, i64, vp, vp, dbl, dbl, vp, vp]
    lib.orc_step_batch.restype = None
    lib.orc_trace.argtypes = [vp, i64, vp, dbl, dbl, i64, i64, ctypes.c_int]
    lib.orc_trace.restype = None
    _lib = lib
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class Field:
    """Oracle view of one block.

    ``nodes`` is the stored node array [S][nz+2g][ny+2g][nx+2g][3] (float32,
    uint16 FP16/BF16 bits, or float64) and ``fmt`` names its format.
    """

    def __init__(self, dims, ghost, origin, spacing, lo, hi, periodic=False, rank_grid=(1, 1, 1),
                 rank_coord=(0, 0, 0), n_slices=1, t0=0.0, slice_dt=1.0, nodes=None, fmt=FMT_F64,
                 analytic_abc=None):
        self._nodes = None if nodes is None else np.ascontiguousarray(nodes)
        b = _Block()
        b.dims[:] = [int(v) for v in dims]
        b.ghost = int(ghost)
        b.origin[:] = [float(v) for v in origin]
        b.spacing[:] = [float(v) for v in spacing]
        b.lo[:] = [float(v) for v in lo]
        b.hi[:] = [float(v) for v in hi]
        b.periodic = int(bool(periodic))
        b.rank_grid[:] = [int(v) for v in rank_grid]
        b.rank_coord[:] = [int(v) for v in rank_coord]
        b.n_slices = int(n_slices)
        b.t0 = float(t0)
        b.slice_dt = float(slice_dt)
        b.nodes = None if self._nodes is None else self._nodes.ctypes.data
        b.fmt = int(fmt)
        b.field_kind = FIELD_GRID if analytic_abc is None else FIELD_ABC
        if analytic_abc is not None:
            b.abc[:] = [float(v) for v in analytic_abc]
        self.b = b
        self.periodic = bool(periodic)
        _load()

    @classmethod
    def from_block(cls, blk, use_values: bool = False):
        """Build from a duck-typed block (dims, ghost, origin, spacing, lo, hi, boundary,
        rank_grid, rank_coord, n_slices, t0, slice_dt, stored/fmt, values)."""
        nodes, fmt = (blk.values, FMT_F64) if use_values else (blk.stored, int(blk.fmt))
        return cls(blk.dims, blk.ghost, blk.origin, blk.spacing, blk.lo, blk.hi,
                   periodic=(blk.boundary == 1), rank_grid=blk.rank_grid,
                   rank_coord=blk.rank_coord, n_slices=blk.n_slices, t0=blk.t0,
                   slice_dt=blk.slice_dt, nodes=nodes, fmt=fmt)

    @classmethod
    def abc_analytic(cls, A=np.sqrt(3.0), B=np.sqrt(2.0), C=1.0):
        tp = 2 * np.pi
        return cls((1, 1, 1), 0, (0, 0, 0), (1, 1, 1), (0, 0, 0), (tp, tp, tp), periodic=True,
                   analytic_abc=(A, B, C))

    def _bp(self):
        return ctypes.byref(self.b)

    def sample(self, x, t=None):
        x = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1, 3))
        n = x.shape[0]
        tt = None if t is None else np.ascontiguousarray(np.broadcast_to(np.asarray(t, np.float64), (n,)))
        v = np.zeros((n, 3), np.float64)
        d = np.zeros(n, np.int32)
        _lib.orc_sample_batch(self._bp(), n, _p(x), _p(tt), _p(v), _p(d))
        return v, d.astype(bool)

    def dest(self, x):
        x = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1, 3))
        d = np.zeros(x.shape[0], np.int32)
        _lib.orc_dest_batch(self._bp(), x.shape[0], _p(x), _p(d))
        return d

    def step(self, p0, h, eps=0.0, t=None):
        """One RK4 update per row of p0; returns (p1, status) with status ACTIVE when taken."""
        p0 = np.ascontiguousarray(np.asarray(p0, np.float64).reshape(-1, 3))
        n = p0.shape[0]
        tt = None if t is None else np.ascontiguousarray(np.broadcast_to(np.asarray(t, np.float64), (n,)))
        p1 = np.full((n, 3), np.nan)
        st = np.zeros(n, np.int32)
        _lib.orc_step_batch(self._bp(), n, _p(p0), _p(tt), float(h), float(eps), _p(p1), _p(st))
        return p1, st

    def trace(self, seeds, h, max_steps, eps=1e-6, t_birth=None, cap=None, stride=1,
              threads=None, keep_verts=True):
        """Trace to termination.  Returns a dict of numpy arrays:
        steps, code, final_pos, n_verts, verts [n][cap][3] (if kept), in_outbox,
        out_pos, out_dest."""
        seeds = np.ascontiguousarray(np.asarray(seeds, np.float64).reshape(-1, 3))
        n = seeds.shape[0]
        ms = np.ascontiguousarray(np.broadcast_to(np.asarray(max_steps, np.int32), (n,)))
        tb = None if t_birth is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(t_birth, np.float64), (n,)))
        if cap is None:
            cap = int(ms.max(initial=0)) // max(1, stride) + 2
        r = dict(steps=np.zeros(n, np.int32), code=np.zeros(n, np.int32),
                 final_pos=np.zeros((n, 3)), n_verts=np.zeros(n, np.int64),
                 verts=np.full((n, cap, 3), np.nan) if keep_verts else None,
                 in_outbox=np.zeros(n, np.int8), out_pos=np.full((n, 3), np.nan),
                 out_dest=np.zeros(n, np.int32))
        io = _TraceIO()
        io.seeds, io.max_steps, io.t_birth = seeds.ctypes.data, ms.ctypes.data, (
            None if tb is None else tb.ctypes.data)
        for k in ("steps", "code", "final_pos", "n_verts", "verts", "in_outbox", "out_pos",
                  "out_dest"):
            setattr(io, k, None if r[k] is None else r[k].ctypes.data)
        threads = threads or min(16, os.cpu_count() or 1)
        _lib.orc_trace(self._bp(), n, ctypes.byref(io), float(h), float(eps), int(cap),
                       int(stride), int(threads))
        return r
