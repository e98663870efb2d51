"""FP64 oracle of an unstructured field -- TEST INFRASTRUCTURE.

Only tests/ may import it.  It shares no code with the GPU library.

The paper's second field type (Sec. 3.3) is an unstructured grid of tetrahedra, pyramids,
wedges (prisms) and hexahedra located by point containment; its benchmark converts every
voxel of a structured data set to a hexahedron (Sec. 5).  Definitions, written out plainly
(no acceleration structure: every cell whose vertex box holds the point is tested):

  * each cell lists its vertices in VTK order (VTK_TETRA 4, VTK_PYRAMID 5, VTK_WEDGE 6,
    VTK_HEXAHEDRON 8 vertices) and maps parametric coordinates (r, s, t) to space with the
    VTK linear shape functions N_i:
      hexahedron  the trilinear weights w(r) w(s) w(t), w(0) = 1 - r, w(1) = r, of the corner
                  with parametric coordinates in {0,1}^3; the corner r + 2s + 4t is vertex
                  VTK_OF_CORNER[r + 2s + 4t]; domain [0,1]^3;
      tetra       1 - r - s - t, r, s, t;  domain r, s, t >= 0, r + s + t <= 1;
      wedge       (1-r-s)(1-t), r(1-t), s(1-t), (1-r-s)t, r t, s t;
                  domain r, s >= 0, r + s <= 1, 0 <= t <= 1;
      pyramid     (1-r)(1-s)(1-t), r(1-s)(1-t), r s (1-t), (1-r) s (1-t), t;  domain [0,1]^3
                  (the base quad in order, the apex last);
  * x lies in a cell iff X(r,s,t) = sum N_i X_i = x has a solution in the cell's domain (found
    by Newton's method to FP64 convergence; a tetrahedron's map is affine).  A non-affine map
    can have a second root outside the domain, which Newton from the domain's centre may
    reach when x lies near a vertex of a warped cell: a start that does not end inside the
    domain is retried once from the parametric point of the cell vertex nearest to x, moved a
    fifth of the way to the centre;
  * sample(x) = sum N_i V_i at that solution in the first such cell in cell order (on a mesh
    whose neighbouring cells interpolate alike on shared faces every containing cell gives
    the same value); undefined (False) when no cell contains x (Sec. 3.1.1: sample() fails);
  * destinationID, the owned bounds and the RK4 update with its termination rules are those
    of the structured oracle (Sec. 3.1.1, Sec. 3.1.2).
"""
from __future__ import annotations

import numpy as np

from . import ACTIVE, EXIT, HALO_MISS, MAX_STEPS, NONFINITE, STAGNANT

# VTK_HEXAHEDRON vertex order: 0 (0,0,0), 1 (1,0,0), 2 (1,1,0), 3 (0,1,0), 4 (0,0,1), 5 (1,0,1),
# 6 (1,1,1), 7 (0,1,1); corner index r + 2s + 4u -> VTK vertex
VTK_OF_CORNER = np.array([0, 1, 3, 2, 4, 5, 7, 6])
CORNER_BITS = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], np.float64)
INSIDE_TOL = 1e-12  # parametric slack for points on a cell face

# VTK cell type codes and vertex counts
VTK_TETRA, VTK_HEXAHEDRON, VTK_WEDGE, VTK_PYRAMID = 10, 12, 13, 14
N_VERTS = {VTK_TETRA: 4, VTK_HEXAHEDRON: 8, VTK_WEDGE: 6, VTK_PYRAMID: 5}
START = {VTK_TETRA: (0.25, 0.25, 0.25), VTK_WEDGE: (1 / 3, 1 / 3, 0.5), VTK_PYRAMID: (0.5, 0.5, 0.5),
         VTK_HEXAHEDRON: (0.5, 0.5, 0.5)}
# parametric points of each kind's vertices (VTK order; a pyramid's apex at r = s = 1/2)
VERTEX_PARAM = {VTK_TETRA: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)],
                VTK_WEDGE: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1)],
                VTK_PYRAMID: [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0.5, 0.5, 1)],
                VTK_HEXAHEDRON: [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1),
                                 (0, 1, 1)]}


def shape(kind, rst):
    """VTK shape functions of a tetra, wedge or pyramid at parametric points rst [n, 3]:
    (N [n, k], dN/d(r,s,t) [n, k, 3])."""
    rst = np.asarray(rst, np.float64)
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    o, z = np.ones_like(r), np.zeros_like(r)
    if kind == VTK_TETRA:
        N = [1 - r - s - t, r, s, t]
        dN = [(-o, -o, -o), (o, z, z), (z, o, z), (z, z, o)]
    elif kind == VTK_WEDGE:
        a = 1 - r - s
        N = [a * (1 - t), r * (1 - t), s * (1 - t), a * t, r * t, s * t]
        dN = [(-(1 - t), -(1 - t), -a), (1 - t, z, -r), (z, 1 - t, -s), (-t, -t, a), (t, z, r), (z, t, s)]
    elif kind == VTK_PYRAMID:
        N = [(1 - r) * (1 - s) * (1 - t), r * (1 - s) * (1 - t), r * s * (1 - t), (1 - r) * s * (1 - t), t]
        dN = [(-(1 - s) * (1 - t), -(1 - r) * (1 - t), -(1 - r) * (1 - s)),
              ((1 - s) * (1 - t), -r * (1 - t), -r * (1 - s)),
              (s * (1 - t), r * (1 - t), -r * s),
              (-s * (1 - t), (1 - r) * (1 - t), -(1 - r) * s),
              (z, z, o)]
    else:
        raise ValueError(kind)
    return np.stack(N, 1), np.stack([np.stack(d, 1) for d in dN], 1)


def in_domain(kind, rst, tol):
    """Parametric points [n, 3] inside a cell kind's domain, with slack tol."""
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    if kind == VTK_TETRA:
        return (r >= -tol) & (s >= -tol) & (t >= -tol) & (r + s + t <= 1 + tol)
    if kind == VTK_WEDGE:
        return (r >= -tol) & (s >= -tol) & (r + s <= 1 + tol) & (t >= -tol) & (t <= 1 + tol)
    return np.all((rst >= -tol) & (rst <= 1 + tol), axis=1)


def weights(rsu):
    """Trilinear weights [n, 8] of the corners at parametric points rsu [n, 3]."""
    rsu = np.asarray(rsu, np.float64)
    w = np.ones((len(rsu), 8))
    for a in range(3):
        t = rsu[:, a:a + 1]
        w *= np.where(CORNER_BITS[None, :, a] == 1, t, 1.0 - t)
    return w


def weight_derivs(rsu):
    """d weights / d(r, s, u): [n, 8, 3]."""
    rsu = np.asarray(rsu, np.float64)
    d = np.ones((len(rsu), 8, 3))
    for a in range(3):  # derivative with respect to coordinate a
        for b in range(3):
            t = rsu[:, b:b + 1]
            if a == b:
                f = np.where(CORNER_BITS[None, :, b] == 1, 1.0, -1.0) * np.ones_like(t)
            else:
                f = np.where(CORNER_BITS[None, :, b] == 1, t, 1.0 - t)
            d[:, :, a] *= f
    return d


class HexField:
    """A steady unstructured field: vertices [nv, 3], values [nv, 3], cells [nc, 8] (each row
    the cell's vertices in VTK order, unused trailing entries ignored), cell_types [nc] (VTK
    codes; None: all hexahedra), owned bounds [lo, hi) and a rank grid for destinationID."""

    def __init__(self, vertices, values, cells, lo, hi, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0),
                 cell_types=None):
        vertices = np.asarray(vertices, np.float64)
        values = np.asarray(values, np.float64)
        cells = np.asarray(cells, np.int64)
        nc = len(cells)
        self.types = (np.full(nc, VTK_HEXAHEDRON, np.int64) if cell_types is None
                      else np.asarray(cell_types, np.int64).reshape(nc))
        assert set(np.unique(self.types).tolist()) <= set(N_VERTS), "unknown cell type"
        self.cells = cells
        self.P = vertices
        self.Vv = values
        hexes = self.types == VTK_HEXAHEDRON
        safe = np.where(hexes[:, None], cells, 0)
        self.X = vertices[safe[:, VTK_OF_CORNER]]  # [nc, 8, 3] hexahedron corners by parametric index
        self.V = values[safe[:, VTK_OF_CORNER]]
        self.box_lo = np.empty((nc, 3))
        self.box_hi = np.empty((nc, 3))
        for kind, k in N_VERTS.items():
            sel = self.types == kind
            if sel.any():
                pts = vertices[cells[sel, :k]]
                self.box_lo[sel] = pts.min(axis=1)
                self.box_hi[sel] = pts.max(axis=1)
        self.lo = np.asarray(lo, np.float64)
        self.hi = np.asarray(hi, np.float64)
        self.rank_grid = np.asarray(rank_grid, np.int64)
        self.rank_coord = np.asarray(rank_coord, np.int64)
        self.periodic = False

    # ------------------------------------------------------------ location
    def retry_start(self, kind, cell, x):
        """The second Newton start: the parametric point of the cell vertex nearest to x, a fifth
        of the way towards the domain's centre."""
        P = self.P[self.cells[cell, :N_VERTS[kind]]]
        near = np.argmin(((P - x[:, None, :]) ** 2).sum(axis=2), axis=1)
        return 0.8 * np.asarray(VERTEX_PARAM[kind], np.float64)[near] + 0.2 * np.asarray(START[kind])

    def invert(self, cell, x, iters=60, start=None):
        """Parametric coordinates of x in each given hexahedron (Newton from the centre or from
        `start`); NaN rows where the iteration does not converge."""
        X = self.X[cell]
        rsu = np.full((len(cell), 3), 0.5) if start is None else np.array(start, np.float64)
        done = np.zeros(len(cell), bool)
        for _ in range(iters):
            F = np.einsum("nk,nkc->nc", weights(rsu), X) - x
            J = np.einsum("nka,nkc->nca", weight_derivs(rsu), X)  # J[n, c, a] = dX_c / d rsu_a
            # a degenerate cell (singular map) contains no point: its rows become NaN
            with np.errstate(all="ignore"):
                det = np.linalg.det(J)
                sing = ~(np.abs(det) > 1e-300) | ~np.isfinite(det)
                J[sing] = np.eye(3)
                delta = np.linalg.solve(J, F[:, :, None])[:, :, 0]
            delta[sing] = np.nan
            delta[done] = 0.0
            rsu = rsu - delta
            done |= np.abs(delta).max(axis=1) <= 1e-12  # the next step would be at rounding level
            if done.all():
                break
        rsu[~done | ~np.isfinite(rsu).all(axis=1)] = np.nan
        return rsu

    def invert_kind(self, kind, cell, x, iters=60, start=None):
        """Parametric coordinates of x in tetra, wedge or pyramid cells of one kind (Newton from
        the domain's centre or from `start`; one step for a tetrahedron); NaN rows where it does
        not converge."""
        P = self.P[self.cells[cell, :N_VERTS[kind]]]  # [m, k, 3]
        rst = np.tile(np.array(START[kind]), (len(cell), 1)) if start is None else np.array(start, np.float64)
        done = np.zeros(len(cell), bool)
        for _ in range(iters):
            N, dN = shape(kind, rst)
            F = np.einsum("nk,nkc->nc", N, P) - x
            J = np.einsum("nka,nkc->nca", dN, P)
            with np.errstate(all="ignore"):
                det = np.linalg.det(J)
                sing = ~(np.abs(det) > 1e-300) | ~np.isfinite(det)
                J[sing] = np.eye(3)
                delta = np.linalg.solve(J, F[:, :, None])[:, :, 0]
            delta[sing] = np.nan
            delta[done] = 0.0
            rst = rst - delta
            step = np.abs(delta)
            if kind == VTK_PYRAMID:  # r and s move a point by (1 - t) times their step
                step[:, :2] *= np.abs(1.0 - rst[:, 2:3])
            done |= step.max(axis=1) <= 1e-12
            if done.all():
                break
        rst[~done | ~np.isfinite(rst).all(axis=1)] = np.nan
        return rst

    def locate(self, x):
        """(cell, rsu) of the first cell (in cell order) containing each point; cell -1 if none."""
        x = np.asarray(x, np.float64).reshape(-1, 3)
        n = len(x)
        cell = np.full(n, -1, np.int64)
        rsu = np.full((n, 3), np.nan)
        fin = np.isfinite(x).all(axis=1)
        cand = fin[:, None] & np.all((x[:, None, :] >= self.box_lo[None] - 1e-12)
                                     & (x[:, None, :] <= self.box_hi[None] + 1e-12), axis=2)
        pi, ci = np.nonzero(cand)  # candidate pairs, cells in increasing order per point
        if len(pi):
            r = np.full((len(pi), 3), np.nan)
            kinds = self.types[ci]
            for kind in np.unique(kinds).tolist():
                sel = kinds == kind
                r[sel] = (self.invert(ci[sel], x[pi[sel]]) if kind == VTK_HEXAHEDRON
                          else self.invert_kind(kind, ci[sel], x[pi[sel]]))
            ok = np.zeros(len(pi), bool)
            for kind in np.unique(kinds).tolist():
                sel = kinds == kind
                with np.errstate(invalid="ignore"):
                    ok[sel] = in_domain(kind, r[sel], INSIDE_TOL)
                if kind == VTK_TETRA:
                    continue
                again = np.nonzero(sel & ~ok)[0]  # the second start
                if len(again):
                    st = self.retry_start(kind, ci[again], x[pi[again]])
                    r2 = (self.invert(ci[again], x[pi[again]], start=st) if kind == VTK_HEXAHEDRON
                          else self.invert_kind(kind, ci[again], x[pi[again]], start=st))
                    with np.errstate(invalid="ignore"):
                        ok2 = in_domain(kind, r2, INSIDE_TOL)
                    r[again[ok2]] = r2[ok2]
                    ok[again[ok2]] = True
            pi, ci, r = pi[ok], ci[ok], r[ok]
            first = np.unique(pi, return_index=True)[1]  # first containing cell per point
            cell[pi[first]] = ci[first]
            hexa = self.types[ci[first]] == VTK_HEXAHEDRON
            rsu[pi[first]] = np.where(hexa[:, None], np.clip(r[first], 0.0, 1.0), r[first])
        return cell, rsu

    def sample(self, x, t=None):
        """(values [n, 3], defined [n]) at points x."""
        cell, rsu = self.locate(x)
        ok = cell >= 0
        v = np.zeros((len(cell), 3))
        kinds = np.where(ok, self.types[np.maximum(cell, 0)], -1)
        for kind in np.unique(kinds[ok]).tolist():
            sel = kinds == kind
            if kind == VTK_HEXAHEDRON:
                v[sel] = np.einsum("nk,nkc->nc", weights(rsu[sel]), self.V[cell[sel]])
            else:
                N, _ = shape(kind, rsu[sel])
                v[sel] = np.einsum("nk,nkc->nc", N, self.Vv[self.cells[cell[sel], :N_VERTS[kind]]])
        return v, ok

    def dest(self, x):
        """destinationID: flat rank of the macrocell holding x, -1 outside the rank grid."""
        x = np.asarray(x, np.float64).reshape(-1, 3)
        r = self.rank_coord[None, :] + np.floor((x - self.lo) / (self.hi - self.lo)).astype(np.int64)
        ok = np.all((r >= 0) & (r < self.rank_grid[None, :]), axis=1)
        d = r[:, 0] + self.rank_grid[0] * (r[:, 1] + self.rank_grid[1] * r[:, 2])
        return np.where(ok, d, -1)

    # ------------------------------------------------------------ RK4
    def step(self, p0, h, eps=0.0, t=None):
        """One classical RK4 update per row (the structured oracle's rules): (p1, status)."""
        p0 = np.asarray(p0, np.float64).reshape(-1, 3)
        n = len(p0)
        st = np.full(n, ACTIVE, np.int32)
        p1 = np.full((n, 3), np.nan)
        fail = np.full((n, 3), np.nan)
        live = np.ones(n, bool)
        k1, ok = self.sample(p0)
        st[~ok] = HALO_MISS
        fail[~ok] = p0[~ok]
        live &= ok
        bad = live & ~np.isfinite(k1).all(axis=1)
        st[bad] = NONFINITE
        live &= ~bad
        stag = live & (np.sqrt((k1 * k1).sum(axis=1)) < eps)
        st[stag] = STAGNANT
        live &= ~stag
        ks = [k1]
        for frac, kprev in ((0.5, 0), (0.5, 1), (1.0, 2)):
            q = p0 + frac * h * ks[kprev]
            k, ok = self.sample(np.where(live[:, None], q, 0.0))
            miss = live & ~ok
            st[miss] = np.where(np.isfinite(q[miss]).all(axis=1), HALO_MISS, NONFINITE)
            fail[miss] = q[miss]
            live &= ok
            bad = live & ~np.isfinite(k).all(axis=1)
            st[bad] = NONFINITE
            live &= ~bad
            ks.append(k)
        p1[live] = p0[live] + (h / 6.0) * (ks[0] + 2.0 * ks[1] + 2.0 * ks[2] + ks[3])[live]
        bad = live & ~np.isfinite(p1).all(axis=1)
        st[bad] = NONFINITE
        self._fail = fail
        return p1, st

    def inside_owned(self, x):
        return np.all((x >= self.lo) & (x < self.hi), axis=1)

    def trace(self, seeds, h, max_steps, eps=1e-6, t_birth=None, keep_verts=True):
        """Trace to termination, every vertex kept: dict of steps, code, final_pos, n_verts,
        verts [n][max+1][3] (NaN-padded), in_outbox, out_pos, out_dest."""
        P = np.asarray(seeds, np.float64).reshape(-1, 3).copy()
        n = len(P)
        m = np.broadcast_to(np.asarray(max_steps, np.int64), (n,)).copy()
        cap = int(m.max(initial=0)) + 2
        verts = np.full((n, cap, 3), np.nan) if keep_verts else None
        steps = np.zeros(n, np.int32)
        code = np.full(n, ACTIVE, np.int32)
        nv = np.ones(n, np.int64)
        if keep_verts:
            verts[:, 0] = P
        out_pos = np.full((n, 3), np.nan)
        out_dest = np.full(n, -1, np.int32)
        exit0 = ~self.inside_owned(P)
        code[exit0] = EXIT
        out_pos[exit0] = P[exit0]
        out_dest[exit0] = self.dest(P[exit0])
        while True:
            act = code == ACTIVE
            lim = act & (steps >= m)
            code[lim] = MAX_STEPS
            act &= ~lim
            idx = np.nonzero(act)[0]
            if len(idx) == 0:
                break
            p1, st = self.step(P[idx], h, eps)
            fail = self._fail
            miss = st == HALO_MISS
            code[idx[miss]] = HALO_MISS
            out_pos[idx[miss]] = P[idx[miss]]
            out_dest[idx[miss]] = self.dest(fail[miss])
            other = (st != ACTIVE) & ~miss
            code[idx[other]] = st[other]
            go = idx[st == ACTIVE]
            P[go] = p1[st == ACTIVE]
            steps[go] += 1
            if keep_verts:
                verts[go, nv[go]] = P[go]
            nv[go] += 1
            ex = go[~self.inside_owned(P[go])]
            code[ex] = EXIT
            out_pos[ex] = P[ex]
            out_dest[ex] = self.dest(P[ex])
        return dict(steps=steps, code=code, final_pos=P, n_verts=nv, verts=verts,
                    in_outbox=((code == EXIT) | (code == HALO_MISS)).astype(np.int8), out_pos=out_pos,
                    out_dest=out_dest)
