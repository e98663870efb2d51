// Unstructured field of hexahedra, tetrahedra, wedges and pyramids: point
// location and interpolation (Sec. 3.3: an unstructured grid located by a
// bounding volume hierarchy and point containment tests; Sec. 5 converts every
// voxel to a hexahedron).
//
// Every kind of cell maps parametric coordinates (r, s, u) to space with a
// polynomial in the monomials 1, r, s, rs, u, ru, su, rsu (its VTK linear
// shape functions written out): a tetrahedron's map is affine and its domain
// the simplex r, s, u >= 0, r + s + u <= 1; a wedge's has no rs and rsu terms
// and its domain is the triangle r, s >= 0, r + s <= 1 times 0 <= u <= 1; a
// pyramid's is the hexahedron's with the top face collapsed into the apex
// (domain [0,1]^3, singular at u = 1); a hexahedron's is trilinear.  The value
// map uses the same polynomial of the vertex values.
//
// Device blob of one field, addressed in 16-byte units from its start:
//   HexHeader (2 units) | BVH nodes (2 units each) | cell records (12 units each)
//   | face neighbours (2 units per record).
// A lane keeps the cell it sampled last; when a point leaves it, the Newton
// solution outside the cell names the face it left through, and the cell across
// that face is tried next (a particle moves a fraction of a cell per stage), for
// up to HEX_HOPS cells; only then does the BVH walk run.
// BVH: nodes in depth-first preorder, each with its box and `skip` (the index of
// the first node after its subtree), so a point query walks the array without a
// stack: a box that holds the point is entered (next node), one that does not
// is skipped.  A leaf names up to 8 consecutive cell records.
// Cell record (FP32): the trilinear position map and value map in monomial form
// over the parametric coordinates (r, s, u) in [0,1]^3, coefficients of
// 1, r, s, rs, u, ru, su, rsu, three components each (24 + 24 floats); the
// position map's constant term is the cell's first corner.
#pragma once
#include "device.h"

namespace streami {

struct alignas(16) HexHeader {
  unsigned n_nodes;
  unsigned n_cells;
  unsigned node_off;   // 16-byte units from the blob start
  unsigned cell_off;
  float tol;           // parametric slack of the containment test
  unsigned neigh_off;  // face neighbours: 2 units per record, 8 ints: the cells across the
                       // record's faces (hex_exit_face order; -1: none), each as
                       // (kind << 28) | record, then the record's own kind, then unused
  unsigned pad[2];
};
static_assert(sizeof(HexHeader) == 32, "hex header is two 16-byte units");

constexpr int HEX_REC_UNITS = 12;  // 16-byte units per cell record
constexpr int HEX_LEAF_MAX = 8;    // cells per BVH leaf
// kinds of cell (the record's own kind sits in slot 6 of its neighbour entry)
enum HexKind { HK_HEX = 0, HK_TETRA = 1, HK_WEDGE = 2, HK_PYRAMID = 3 };
constexpr int HEX_KIND_SHIFT = 28;
constexpr int HEX_REC_MASK = (1 << HEX_KIND_SHIFT) - 1;

// Containment of x in one cell: Newton's method on the position map, in FP32
// relative to the first vertex, from the centre of the kind's domain (a
// pyramid's r and s steps count times 1 - u: near the apex they move the point
// that much less).  A non-affine map can have a second root outside the
// domain, which the iteration may reach when x lies near a vertex of a warped
// cell: a first start that does not end inside is retried once from the
// parametric point of the vertex nearest to x, a fifth of the way to the
// centre, and the last start decides.  Returns 1 when it converges inside the
// domain widened by tol, 0 when it converges outside (rsu then locates x beyond
// the cell's faces), -1 when it does not converge.
__device__ __forceinline__ int hex_contains(const float4* rec, float3 x, float tol, int kind, float3& rsu) {
  const float4 q0 = rec[0], q1 = rec[1], q2 = rec[2], q3 = rec[3], q4 = rec[4], q5 = rec[5];
  // c[k][a] = coefficient k (1, r, s, rs, u, ru, su, rsu), component a
  const float c[8][3] = {{q0.x, q0.y, q0.z}, {q0.w, q1.x, q1.y}, {q1.z, q1.w, q2.x}, {q2.y, q2.z, q2.w},
                         {q3.x, q3.y, q3.z}, {q3.w, q4.x, q4.y}, {q4.z, q4.w, q5.x}, {q5.y, q5.z, q5.w}};
  const float d[3] = {x.x - c[0][0], x.y - c[0][1], x.z - c[0][2]};
  // an affine cell (no rs, ru, su, rsu terms: a tetrahedron, a parallelepiped such as a voxel)
  // has a constant Jacobian and one root, so the first Newton step is the solution
  bool affine = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) affine = affine && c[3][a] == 0.0f && c[5][a] == 0.0f && c[6][a] == 0.0f && c[7][a] == 0.0f;
  const float cr = kind == HK_TETRA ? 0.25f : kind == HK_WEDGE ? 1.0f / 3.0f : 0.5f;
  const float cu = kind == HK_TETRA ? 0.25f : 0.5f;
  const float lo = -tol, hi = 1.0f + tol;
  float r = cr, s = cr, u = cu;
  int result = -1;
#pragma unroll 1
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (attempt == 1) {
      if (result > 0 || affine) break;
      // the vertex nearest to x: X(vertex) - X(vertex 0) against d
      const int nv = kind == HK_HEX ? 8 : kind == HK_WEDGE ? 6 : 5;
      float best = INFINITY;
#pragma unroll 1
      for (int i = 0; i < nv; ++i) {
        float vr, vs, vu;
        if (kind == HK_HEX) {
          vr = (float)(i & 1); vs = (float)((i >> 1) & 1); vu = (float)(i >> 2);
        } else if (kind == HK_WEDGE) {
          vr = (float)(i % 3 == 1); vs = (float)(i % 3 == 2); vu = (float)(i / 3);
        } else {
          vr = i == 4 ? 0.5f : (float)(i == 1 || i == 2); vs = i == 4 ? 0.5f : (float)(i >= 2); vu = (float)(i == 4);
        }
        float dist = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float e = fmaf(c[1][a], vr, fmaf(c[2][a], vs, fmaf(c[3][a], vr * vs, fmaf(c[4][a], vu,
                          fmaf(c[5][a], vr * vu, fmaf(c[6][a], vs * vu, fmaf(c[7][a], vr * vs * vu, -d[a])))))));
          dist = fmaf(e, e, dist);
        }
        if (dist < best) {
          best = dist;
          r = fmaf(0.8f, vr, 0.2f * cr);
          s = fmaf(0.8f, vs, 0.2f * cr);
          u = fmaf(0.8f, vu, 0.2f * cu);
        }
      }
    }
    bool conv = false;
#pragma unroll 1
    for (int it = 0; it < 8; ++it) {
      const float rs = r * s, ru = r * u, su = s * u, rsu3 = rs * u;
      float F[3], Jr[3], Js[3], Ju[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        F[a] = fmaf(c[1][a], r, fmaf(c[2][a], s, fmaf(c[3][a], rs, fmaf(c[4][a], u, fmaf(c[5][a], ru,
                    fmaf(c[6][a], su, fmaf(c[7][a], rsu3, -d[a])))))));
        Jr[a] = fmaf(c[3][a], s, fmaf(c[5][a], u, fmaf(c[7][a], su, c[1][a])));
        Js[a] = fmaf(c[3][a], r, fmaf(c[6][a], u, fmaf(c[7][a], ru, c[2][a])));
        Ju[a] = fmaf(c[5][a], r, fmaf(c[6][a], s, fmaf(c[7][a], rs, c[4][a])));
      }
      // Cramer's rule for [Jr Js Ju] delta = F
      const float x0 = Js[1] * Ju[2] - Js[2] * Ju[1], x1 = Js[2] * Ju[0] - Js[0] * Ju[2],
                  x2 = Js[0] * Ju[1] - Js[1] * Ju[0];  // Js x Ju
      const float det = Jr[0] * x0 + Jr[1] * x1 + Jr[2] * x2;
      if (!(fabsf(det) > 0.0f)) break;  // degenerate cell (or NaN): contains nothing
      const float inv = 1.0f / det;
      const float y0 = F[1] * Ju[2] - F[2] * Ju[1], y1 = F[2] * Ju[0] - F[0] * Ju[2],
                  y2 = F[0] * Ju[1] - F[1] * Ju[0];  // F x Ju
      const float z0 = Js[1] * F[2] - Js[2] * F[1], z1 = Js[2] * F[0] - Js[0] * F[2],
                  z2 = Js[0] * F[1] - Js[1] * F[0];  // Js x F
      const float dr = (F[0] * x0 + F[1] * x1 + F[2] * x2) * inv;
      const float ds = (Jr[0] * y0 + Jr[1] * y1 + Jr[2] * y2) * inv;
      const float du = (Jr[0] * z0 + Jr[1] * z1 + Jr[2] * z2) * inv;
      r -= dr;
      s -= ds;
      u -= du;
      const float w = kind == HK_PYRAMID ? fabsf(1.0f - u) : 1.0f;
      if (affine || fmaxf(w * fmaxf(fabsf(dr), fabsf(ds)), fabsf(du)) <= 1e-5f) {
        conv = true;
        break;
      }
    }
    if (!conv) {
      result = -1;
      continue;
    }
    bool in = r >= lo && s >= lo && u >= lo;
    if (kind == HK_TETRA) in = in && r + s + u <= hi;
    else if (kind == HK_WEDGE) in = in && r + s <= hi && u <= hi;
    else in = in && r <= hi && s <= hi && u <= hi;
    result = in ? 1 : 0;
  }
  rsu = make_float3(r, s, u);
  return result;
}

// The face beyond which the parametric point lies farthest, numbered per kind:
//   hexahedron r=0, r=1, s=0, s=1, u=0, u=1;  tetrahedron r=0, s=0, u=0, r+s+u=1;
//   wedge r=0, s=0, r+s=1, u=0, u=1;  pyramid r=0, r=1, s=0, s=1, u=0.
__device__ __forceinline__ int hex_exit_face(int kind, float3 q) {
  float w = -q.x;
  int f = 0;
  if (kind == HK_TETRA) {
    if (-q.y > w) { w = -q.y; f = 1; }
    if (-q.z > w) { w = -q.z; f = 2; }
    if (q.x + q.y + q.z - 1.0f > w) { f = 3; }
    return f;
  }
  if (kind == HK_WEDGE) {
    if (-q.y > w) { w = -q.y; f = 1; }
    if (q.x + q.y - 1.0f > w) { w = q.x + q.y - 1.0f; f = 2; }
    if (-q.z > w) { w = -q.z; f = 3; }
    if (q.z - 1.0f > w) { f = 4; }
    return f;
  }
  if (q.x - 1.0f > w) { w = q.x - 1.0f; f = 1; }
  if (-q.y > w) { w = -q.y; f = 2; }
  if (q.y - 1.0f > w) { w = q.y - 1.0f; f = 3; }
  if (-q.z > w) { w = -q.z; f = 4; }
  if (kind == HK_HEX && q.z - 1.0f > w) { f = 5; }
  return f;
}

constexpr int HEX_HOPS = 3;  // neighbour cells tried before a BVH walk

// The value map of a record at parametric coordinates (7 fused multiply-adds per component).
__device__ __forceinline__ float3 hex_value(const float4* rec, float3 rsu) {
  const float4 q0 = rec[6], q1 = rec[7], q2 = rec[8], q3 = rec[9], q4 = rec[10], q5 = rec[11];
  const float k[8][3] = {{q0.x, q0.y, q0.z}, {q0.w, q1.x, q1.y}, {q1.z, q1.w, q2.x}, {q2.y, q2.z, q2.w},
                         {q3.x, q3.y, q3.z}, {q3.w, q4.x, q4.y}, {q4.z, q4.w, q5.x}, {q5.y, q5.z, q5.w}};
  float v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float a0 = fmaf(rsu.z, k[4][a], k[0][a]), a1 = fmaf(rsu.z, k[6][a], k[2][a]);
    const float a2 = fmaf(rsu.z, k[5][a], k[1][a]), a3 = fmaf(rsu.z, k[7][a], k[3][a]);
    v[a] = fmaf(rsu.x, fmaf(rsu.y, a3, a2), fmaf(rsu.y, a1, a0));
  }
  return make_float3(v[0], v[1], v[2]);
}

// sample() of an unstructured field: the record of the cell a lane sampled
// last stays in registers (a particle samples the same cell several times in a
// row), and is tested first; then up to HEX_HOPS neighbours across the faces
// the point lies beyond, each record loaded into the same registers; otherwise
// the BVH walk finds the first leaf cell (in preorder) holding x.  False where
// no cell holds x (Sec. 3.1.1).
struct HexSampler {
  int cell = -1;          // the cell whose record rc holds (-1: none)
  int kind = HK_HEX;      // its kind
  bool affine = false;    // its position map is affine: rc holds the inverse Jacobian (below)
  unsigned gathers = 0;   // BVH walks
  float4 rc[HEX_REC_UNITS];
  __device__ __forceinline__ void reset() { cell = -1; }
  // Load record c.  An affine map (no rs, ru, su, rsu terms: voxels, tetrahedra) is inverted
  // once here: its inverse Jacobian (rows), by Cramer's rule, takes the 12 zero slots of the
  // non-affine coefficients, so a cached sample locates x with 9 multiply-adds.
  __device__ __forceinline__ void load(const float4* recs, int c) {
    const float4* r = recs + (size_t)HEX_REC_UNITS * c;
#pragma unroll
    for (int i = 0; i < HEX_REC_UNITS; ++i) rc[i] = r[i];
    // c1 = (q0.w, q1.x, q1.y), c2 = (q1.z, q1.w, q2.x), c4 = (q3.x, q3.y, q3.z); the zero slots:
    // c3 = (q2.y, q2.z, q2.w), c5 = (q3.w, q4.x, q4.y), c6 = (q4.z, q4.w, q5.x), c7 = (q5.y, q5.z, q5.w)
    affine = rc[2].y == 0.0f && rc[2].z == 0.0f && rc[2].w == 0.0f && rc[3].w == 0.0f && rc[4].x == 0.0f &&
             rc[4].y == 0.0f && rc[4].z == 0.0f && rc[4].w == 0.0f && rc[5].x == 0.0f && rc[5].y == 0.0f &&
             rc[5].z == 0.0f && rc[5].w == 0.0f;
    if (affine) {
      const float a0 = rc[0].w, a1 = rc[1].x, a2 = rc[1].y;  // column r: c1
      const float b0 = rc[1].z, b1 = rc[1].w, b2 = rc[2].x;  // column s: c2
      const float e0 = rc[3].x, e1 = rc[3].y, e2 = rc[3].z;  // column u: c4
      // rows of the inverse: (b x e), (e x a), (a x b) over det
      const float x0 = b1 * e2 - b2 * e1, x1 = b2 * e0 - b0 * e2, x2 = b0 * e1 - b1 * e0;
      const float det = a0 * x0 + a1 * x1 + a2 * x2;
      if (!(fabsf(det) > 0.0f)) {
        affine = false;  // degenerate: the general path finds nothing
        return;
      }
      const float inv = 1.0f / det;
      const float y0 = e1 * a2 - e2 * a1, y1 = e2 * a0 - e0 * a2, y2 = e0 * a1 - e1 * a0;
      const float z0 = a1 * b2 - a2 * b1, z1 = a2 * b0 - a0 * b2, z2 = a0 * b1 - a1 * b0;
      rc[2].y = x0 * inv; rc[2].z = x1 * inv; rc[2].w = x2 * inv;
      rc[3].w = y0 * inv; rc[4].x = y1 * inv; rc[4].y = y2 * inv;
      rc[4].z = z0 * inv; rc[4].w = z1 * inv; rc[5].x = z2 * inv;
    }
  }
  // containment of x in the cached cell (hex_contains' contract)
  __device__ __forceinline__ int contains_cached(float3 x, float tol, float3& rsu) const {
    if (!affine) return hex_contains(rc, x, tol, kind, rsu);
    const float d0 = x.x - rc[0].x, d1 = x.y - rc[0].y, d2 = x.z - rc[0].z;
    const float r = fmaf(rc[2].y, d0, fmaf(rc[2].z, d1, rc[2].w * d2));
    const float s = fmaf(rc[3].w, d0, fmaf(rc[4].x, d1, rc[4].y * d2));
    const float u = fmaf(rc[4].z, d0, fmaf(rc[4].w, d1, rc[5].x * d2));
    rsu = make_float3(r, s, u);
    const float lo = -tol, hi = 1.0f + tol;
    bool in = r >= lo && s >= lo && u >= lo;
    if (kind == HK_TETRA) in = in && r + s + u <= hi;
    else if (kind == HK_WEDGE) in = in && r + s <= hi && u <= hi;
    else in = in && r <= hi && s <= hi && u <= hi;
    return in ? 1 : 0;
  }
  __device__ __forceinline__ bool sample(const BlockDev&, const char* base, float3 x, float, float3& v, bool = false) {
    const HexHeader& H = *reinterpret_cast<const HexHeader*>(base);
    const float4* blob = reinterpret_cast<const float4*>(base);
    const float4* recs = blob + H.cell_off;
    float3 rsu;
    bool found = false;
    if (cell >= 0) {
      int c = cell, k = kind;
#pragma unroll 1
      for (int hop = 0; hop <= HEX_HOPS; ++hop) {
        kind = k;
        const int st = contains_cached(x, H.tol, rsu);
        if (st > 0) {
          found = true;
          cell = c;
          kind = k;
          break;
        }
        if (st < 0 || hop == HEX_HOPS) break;
        const int* nb = reinterpret_cast<const int*>(blob + H.neigh_off + 2 * (size_t)c);
        const int e = nb[hex_exit_face(k, rsu)];
        if (e < 0) break;
        c = e & HEX_REC_MASK;
        k = e >> HEX_KIND_SHIFT;
        load(recs, c);
      }
      if (!found) cell = -1;  // rc holds the last cell tried
    }
    if (!found) {
      ++gathers;
      const float4* nodes = blob + H.node_off;
      unsigned i = 0;
      int hit = -1, hk = HK_HEX;
      while (i < H.n_nodes) {
        const float4 a = nodes[2 * (size_t)i], b = nodes[2 * (size_t)i + 1];
        const bool in = x.x >= a.x && x.x <= b.x && x.y >= a.y && x.y <= b.y && x.z >= a.z && x.z <= b.z;
        const unsigned skip = __float_as_uint(a.w);
        const int leaf = __float_as_int(b.w);
        if (!in) {
          i = skip;
        } else if (leaf < 0) {
          ++i;
        } else {
          const int first = leaf >> 3, cnt = (leaf & 7) + 1;
          for (int q = 0; q < cnt; ++q) {
            const int c = first + q;
            const int ck = reinterpret_cast<const int*>(blob + H.neigh_off + 2 * (size_t)c)[6];
            if (hex_contains(recs + (size_t)HEX_REC_UNITS * c, x, H.tol, ck, rsu) > 0) {
              hit = c;
              hk = ck;
              break;
            }
          }
          if (hit >= 0) break;
          i = skip;
        }
      }
      if (hit < 0) return false;
      cell = hit;
      kind = hk;
      load(recs, hit);
    }
    v = hex_value(rc, rsu);
    return true;
  }
};

}  // namespace streami
