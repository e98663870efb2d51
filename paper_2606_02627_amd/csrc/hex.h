// Unstructured hexahedral field: point location and interpolation (Sec. 3.3:
// an unstructured grid located by a bounding volume hierarchy and point
// containment tests; Sec. 5 converts every voxel to a hexahedron).
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
  unsigned neigh_off;  // face neighbours: 2 units per record, record indices of the cells across
                       // faces r=0, r=1, s=0, s=1, u=0, u=1 (-1: none), then 2 unused
  unsigned pad[2];
};
static_assert(sizeof(HexHeader) == 32, "hex header is two 16-byte units");

constexpr int HEX_REC_UNITS = 12;  // 16-byte units per cell record
constexpr int HEX_LEAF_MAX = 8;    // cells per BVH leaf

// Containment of x in one cell: Newton's method on the position map from the
// cell centre, in FP32 relative to the first corner.  Returns 1 when it
// converges inside [-tol, 1 + tol]^3, 0 when it converges outside (rsu then
// locates x beyond the cell's faces), -1 when it does not converge.
__device__ __forceinline__ int hex_contains(const float4* rec, float3 x, float tol, float3& rsu) {
  const float4 q0 = rec[0], q1 = rec[1], q2 = rec[2], q3 = rec[3], q4 = rec[4], q5 = rec[5];
  // c[k][a] = coefficient k (1, r, s, rs, u, ru, su, rsu), component a
  const float c[8][3] = {{q0.x, q0.y, q0.z}, {q0.w, q1.x, q1.y}, {q1.z, q1.w, q2.x}, {q2.y, q2.z, q2.w},
                         {q3.x, q3.y, q3.z}, {q3.w, q4.x, q4.y}, {q4.z, q4.w, q5.x}, {q5.y, q5.z, q5.w}};
  const float d[3] = {x.x - c[0][0], x.y - c[0][1], x.z - c[0][2]};
  // an affine cell (a parallelepiped: no rs, ru, su, rsu terms, e.g. a voxel) has a constant
  // Jacobian, so the first Newton step is the solution
  bool affine = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) affine = affine && c[3][a] == 0.0f && c[5][a] == 0.0f && c[6][a] == 0.0f && c[7][a] == 0.0f;
  float r = 0.5f, s = 0.5f, u = 0.5f;
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
    if (affine || fmaxf(fabsf(dr), fmaxf(fabsf(ds), fabsf(du))) <= 1e-5f) {
      conv = true;
      break;
    }
  }
  rsu = make_float3(r, s, u);
  const float lo = -tol, hi = 1.0f + tol;
  if (!conv) return -1;
  return (r >= lo && r <= hi && s >= lo && s <= hi && u >= lo && u <= hi) ? 1 : 0;
}

// The face (0: r=0, 1: r=1, 2: s=0, 3: s=1, 4: u=0, 5: u=1) beyond which the
// parametric point lies farthest.
__device__ __forceinline__ int hex_exit_face(float3 q) {
  float w = -q.x;
  int f = 0;
  if (q.x - 1.0f > w) { w = q.x - 1.0f; f = 1; }
  if (-q.y > w) { w = -q.y; f = 2; }
  if (q.y - 1.0f > w) { w = q.y - 1.0f; f = 3; }
  if (-q.z > w) { w = -q.z; f = 4; }
  if (q.z - 1.0f > w) { f = 5; }
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

// sample() of a hexahedral field: the cell a lane sampled last is tested
// first, then up to HEX_HOPS neighbours across the faces the point lies beyond;
// otherwise the BVH walk finds the first leaf cell (in preorder) holding x.
// False where no cell holds x (Sec. 3.1.1).
struct HexSampler {
  int cell = -1;
  unsigned gathers = 0;  // BVH walks
  __device__ __forceinline__ void reset() { cell = -1; }
  __device__ __forceinline__ bool sample(const BlockDev&, const char* base, float3 x, float, float3& v, bool = false) {
    const HexHeader& H = *reinterpret_cast<const HexHeader*>(base);
    const float4* blob = reinterpret_cast<const float4*>(base);
    const float4* recs = blob + H.cell_off;
    float3 rsu;
    int found = -1;
    if (cell >= 0) {
      int c = cell;
#pragma unroll 1
      for (int hop = 0; hop <= HEX_HOPS; ++hop) {
        const int st = hex_contains(recs + (size_t)HEX_REC_UNITS * c, x, H.tol, rsu);
        if (st > 0) {
          found = c;
          break;
        }
        if (st < 0 || hop == HEX_HOPS) break;
        const int* nb = reinterpret_cast<const int*>(blob + H.neigh_off + 2 * (size_t)c);
        c = nb[hex_exit_face(rsu)];
        if (c < 0) break;
      }
    }
    if (found < 0) {
      ++gathers;
      const float4* nodes = blob + H.node_off;
      unsigned i = 0;
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
          for (int k = 0; k < cnt; ++k)
            if (hex_contains(recs + (size_t)HEX_REC_UNITS * (first + k), x, H.tol, rsu) > 0) {
              found = first + k;
              break;
            }
          if (found >= 0) break;
          i = skip;
        }
      }
      if (found < 0) {
        cell = -1;
        return false;
      }
    }
    cell = found;
    v = hex_value(recs + (size_t)HEX_REC_UNITS * cell, rsu);
    return true;
  }
};

}  // namespace streami
