"""FP64 oracle of an unstructured hexahedral field -- TEST INFRASTRUCTURE.

Only tests/ may import it.  It shares no code with the GPU library.

The paper's second field type (Sec. 3.3) is an unstructured grid located by point
containment; its benchmark converts every voxel of a structured data set to a
hexahedron (Sec. 5).  Definitions, written out plainly (no acceleration structure:
every cell is tested):

  * cell c has 8 vertices in VTK hexahedron order; the corner with parametric
    coordinates (r, s, u) in {0,1}^3 is vertex VTK_OF_CORNER[r + 2s + 4u];
  * its trilinear map  X(r,s,u) = sum_corners w(r) w(s) w(u) X_corner  with
    w(0) = 1 - r, w(1) = r (and likewise for s, u);
  * x lies in c iff X(r,s,u) = x has a solution with r, s, u in [0, 1]
    (found by Newton's method from the cell centre, to FP64 convergence);
  * sample(x) = the same trilinear weights applied to the vertex values of the
    first such cell in cell order (every containing cell gives the same value
    on a conforming mesh: the interpolant is continuous across shared faces);
    undefined (False) when no cell contains x (Sec. 3.1.1: sample() fails);
  * destinationID, the owned bounds and the RK4 update with its termination
    rules are those of the structured oracle (Sec. 3.1.1, Sec. 3.1.2).
"""
from __future__ import annotations

import numpy as np

from . import ACTIVE, EXIT, HALO_MISS, MAX_STEPS, NONFINITE, STAGNANT

# VTK_HEXAHEDRON vertex order: 0 (0,0,0), 1 (1,0,0), 2 (1,1,0), 3 (0,1,0), 4 (0,0,1), 5 (1,0,1),
# 6 (1,1,1), 7 (0,1,1); corner index r + 2s + 4u -> VTK vertex
VTK_OF_CORNER = np.array([0, 1, 3, 2, 4, 5, 7, 6])
CORNER_BITS = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], np.float64)
INSIDE_TOL = 1e-12  # parametric slack for points on a cell face


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
    """A steady hexahedral field: vertices [nv, 3], values [nv, 3], cells [nc, 8] (VTK order),
    owned bounds [lo, hi) and a rank grid for destinationID."""

    def __init__(self, vertices, values, cells, lo, hi, rank_grid=(1, 1, 1), rank_coord=(0, 0, 0)):
        vertices = np.asarray(vertices, np.float64)
        values = np.asarray(values, np.float64)
        cells = np.asarray(cells, np.int64)
        self.X = vertices[cells[:, VTK_OF_CORNER]]  # [nc, 8, 3] corners by parametric index
        self.V = values[cells[:, VTK_OF_CORNER]]
        self.box_lo = self.X.min(axis=1)
        self.box_hi = self.X.max(axis=1)
        self.lo = np.asarray(lo, np.float64)
        self.hi = np.asarray(hi, np.float64)
        self.rank_grid = np.asarray(rank_grid, np.int64)
        self.rank_coord = np.asarray(rank_coord, np.int64)
        self.periodic = False

    # ------------------------------------------------------------ location
    def invert(self, cell, x, iters=60):
        """Parametric coordinates of x in each given cell (Newton from the centre); NaN rows
        where the iteration does not converge."""
        X = self.X[cell]
        rsu = np.full((len(cell), 3), 0.5)
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
            r = self.invert(ci, x[pi])
            ok = np.all((r >= -INSIDE_TOL) & (r <= 1 + INSIDE_TOL), axis=1)
            pi, ci, r = pi[ok], ci[ok], r[ok]
            first = np.unique(pi, return_index=True)[1]  # first containing cell per point
            cell[pi[first]] = ci[first]
            rsu[pi[first]] = np.clip(r[first], 0.0, 1.0)
        return cell, rsu

    def sample(self, x, t=None):
        """(values [n, 3], defined [n]) at points x."""
        cell, rsu = self.locate(x)
        ok = cell >= 0
        v = np.zeros((len(cell), 3))
        if ok.any():
            v[ok] = np.einsum("nk,nkc->nc", weights(rsu[ok]), self.V[cell[ok]])
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
