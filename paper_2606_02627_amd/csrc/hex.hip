// Host construction of an unstructured field's device blob (see hex.h): cell
// records in BVH leaf order and a depth-first BVH over the cells' boxes.
//
// BVH: top-down median split of the cell centroids along the longest axis of
// their bounds, leaves of at most 4 cells; each node's box is the union of its
// cells' boxes.  A cell's box holds the whole cell (a trilinear hexahedron lies
// in the convex hull of its corners), widened by the containment slack so that
// points the sampler accepts near a face are still found.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "hex.h"

namespace streami {

namespace {

// VTK cell types and this library's kinds (hex.h)
struct KindInfo {
  int vtk, kind, n_verts, n_faces;
  int face[6][4];  // VTK vertex indices of each face in hex_exit_face order (-1: triangle)
};
constexpr KindInfo KINDS[4] = {
    // hexahedron: faces r=0, r=1, s=0, s=1, u=0, u=1
    {12, HK_HEX, 8, 6, {{0, 3, 7, 4}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 2, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}}},
    // tetrahedron: r=0, s=0, u=0, r+s+u=1
    {10, HK_TETRA, 4, 4, {{0, 2, 3, -1}, {0, 1, 3, -1}, {0, 1, 2, -1}, {1, 2, 3, -1}}},
    // wedge: r=0, s=0, r+s=1, u=0, u=1
    {13, HK_WEDGE, 6, 5, {{0, 2, 5, 3}, {0, 1, 4, 3}, {1, 2, 5, 4}, {0, 1, 2, -1}, {3, 4, 5, -1}}},
    // pyramid: r=0, r=1, s=0, s=1, u=0
    {14, HK_PYRAMID, 5, 5, {{0, 3, 4, -1}, {1, 2, 4, -1}, {0, 1, 4, -1}, {3, 2, 4, -1}, {0, 1, 2, 3}}},
};
const KindInfo* kind_of_vtk(int vtk) {
  for (const KindInfo& k : KINDS)
    if (k.vtk == vtk) return &k;
  return nullptr;
}

// VTK_HEXAHEDRON vertex of the corner with parametric bits r + 2s + 4u
constexpr int VTK_OF_CORNER[8] = {0, 1, 3, 2, 4, 5, 7, 6};

// The cell across each face of every cell (-1 on the mesh boundary): another cell that holds
// all of the face's vertices, found among the cells incident to its smallest vertex.
void face_neighbours(const int* cells, const KindInfo* const* kinds, long long nv, long long nc,
                     std::vector<int>& nb) {
  std::vector<long long> start((size_t)nv + 1, 0);
  for (long long c = 0; c < nc; ++c)
    for (int i = 0; i < kinds[c]->n_verts; ++i) ++start[(size_t)cells[8 * c + i] + 1];
  for (long long v = 0; v < nv; ++v) start[v + 1] += start[v];
  std::vector<int> inc((size_t)start[nv]);
  {
    std::vector<long long> fill(start.begin(), start.end() - 1);
    for (long long c = 0; c < nc; ++c)
      for (int i = 0; i < kinds[c]->n_verts; ++i) inc[(size_t)fill[cells[8 * c + i]]++] = (int)c;
  }
  nb.assign(6 * (size_t)nc, -1);
  auto work = [&](long long b, long long e) {
    for (long long c = b; c < e; ++c) {
      const KindInfo& K = *kinds[c];
      for (int f = 0; f < K.n_faces; ++f) {
        int fv[4], n = 0;
        for (int i = 0; i < 4; ++i)
          if (K.face[f][i] >= 0) fv[n++] = cells[8 * c + K.face[f][i]];
        int vm = fv[0];
        for (int i = 1; i < n; ++i) vm = std::min(vm, fv[i]);
        for (long long k = start[vm]; k < start[vm + 1]; ++k) {
          const int q = inc[(size_t)k];
          if (q == c) continue;
          int hit = 0;
          for (int i = 0; i < n; ++i)
            for (int j = 0; j < kinds[q]->n_verts; ++j)
              if (cells[8 * (long long)q + j] == fv[i]) {
                ++hit;
                break;
              }
          if (hit == n) {
            nb[6 * c + f] = q;
            break;
          }
        }
      }
    }
  };
  const long long nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (long long t = 0; t < nt; ++t) th.emplace_back(work, nc * t / nt, nc * (t + 1) / nt);
  for (auto& t : th) t.join();
}
constexpr int LEAF_CELLS = 4;

struct Node {
  float lo[3], hi[3];
  unsigned skip;
  int leaf;  // -1 internal, else (first record << 3) | (count - 1)
};

struct Builder {
  const float* box;  // [nc][6]: lo xyz, hi xyz
  const float* cen;  // [nc][3]
  std::vector<int>& idx;
  std::vector<Node>& nodes;
  std::vector<int>& order;  // cells in leaf order

  void build(long long b, long long e) {
    const size_t me = nodes.size();
    nodes.push_back(Node());
    Node nd;
    for (int a = 0; a < 3; ++a) {
      nd.lo[a] = INFINITY;
      nd.hi[a] = -INFINITY;
    }
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long long k = b; k < e; ++k) {
      const int c = idx[k];
      for (int a = 0; a < 3; ++a) {
        nd.lo[a] = std::min(nd.lo[a], box[6 * (size_t)c + a]);
        nd.hi[a] = std::max(nd.hi[a], box[6 * (size_t)c + 3 + a]);
        clo[a] = std::min(clo[a], cen[3 * (size_t)c + a]);
        chi[a] = std::max(chi[a], cen[3 * (size_t)c + a]);
      }
    }
    if (e - b <= LEAF_CELLS) {
      nd.leaf = (int)((order.size() << 3) | (size_t)(e - b - 1));
      for (long long k = b; k < e; ++k) order.push_back(idx[k]);
      nd.skip = (unsigned)(me + 1);
    } else {
      int ax = 0;
      for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[ax] - clo[ax]) ax = a;
      const long long mid = (b + e) / 2;
      std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e,
                       [&](int p, int q) { return cen[3 * (size_t)p + ax] < cen[3 * (size_t)q + ax]; });
      build(b, mid);
      build(mid, e);
      nd.leaf = -1;
      nd.skip = (unsigned)nodes.size();
    }
    nodes[me] = nd;
  }
};

// The 8 monomial coefficients (1, r, s, rs, u, ru, su, rsu) of the trilinear
// map through corner values c[i] (i = r + 2s + 4u), per component, in FP64.
void monomial_coeffs(double c[8][3]) {
  for (int bit = 1; bit < 8; bit <<= 1)
    for (int i = 0; i < 8; ++i)
      if (i & bit)
        for (int a = 0; a < 3; ++a) c[i][a] -= c[i ^ bit][a];
}

// The monomial coefficients of a cell's map through its vertex data p[i] (VTK order), in FP64:
// the VTK linear shape functions of each kind written out in 1, r, s, rs, u, ru, su, rsu.
void kind_coeffs(int kind, const double p[8][3], double c[8][3]) {
  for (int i = 0; i < 8; ++i)
    for (int a = 0; a < 3; ++a) c[i][a] = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (kind == HK_HEX) {
      double q[8][3];
      for (int i = 0; i < 8; ++i)
        for (int b = 0; b < 3; ++b) q[i][b] = p[VTK_OF_CORNER[i]][b];
      monomial_coeffs(q);
      for (int i = 0; i < 8; ++i) c[i][a] = q[i][a];
    } else if (kind == HK_TETRA) {  // p0 + r (p1-p0) + s (p2-p0) + u (p3-p0)
      c[0][a] = p[0][a];
      c[1][a] = p[1][a] - p[0][a];
      c[2][a] = p[2][a] - p[0][a];
      c[4][a] = p[3][a] - p[0][a];
    } else if (kind == HK_WEDGE) {  // (1-u) (bottom triangle) + u (top triangle)
      c[0][a] = p[0][a];
      c[1][a] = p[1][a] - p[0][a];
      c[2][a] = p[2][a] - p[0][a];
      c[4][a] = p[3][a] - p[0][a];
      c[5][a] = (p[4][a] - p[3][a]) - (p[1][a] - p[0][a]);
      c[6][a] = (p[5][a] - p[3][a]) - (p[2][a] - p[0][a]);
    } else {  // pyramid: (1-u) Q(r,s) + u apex, Q bilinear through the base p0 p1 p2 p3
      const double q0 = p[0][a], q1 = p[1][a] - p[0][a], q2 = p[3][a] - p[0][a];
      const double q3 = (p[2][a] - p[1][a]) - (p[3][a] - p[0][a]);
      c[0][a] = q0;
      c[1][a] = q1;
      c[2][a] = q2;
      c[3][a] = q3;
      c[4][a] = p[4][a] - q0;
      c[5][a] = -q1;
      c[6][a] = -q2;
      c[7][a] = -q3;
    }
  }
}

}  // namespace

// Blob of an unstructured field (16-byte units: header, nodes, records) from
// host arrays; cells [nc][8] list each cell's vertices in VTK order, types [nc]
// are VTK codes (NULL: all hexahedra); types and vertex indices are checked.
// Returns an empty string or the error.
std::string build_hex_blob(const float* V, long long nv, const float* val, const int* cells,
                           const unsigned char* types, long long nc, float tol, std::vector<float>& blob,
                           unsigned& n_nodes) {
  std::vector<const KindInfo*> kinds((size_t)nc);
  for (long long c = 0; c < nc; ++c) {
    const int t = types ? (int)types[c] : 12;
    kinds[c] = kind_of_vtk(t);
    if (!kinds[c])
      return "cell " + std::to_string(c) + " has type " + std::to_string(t) +
             " (supported: 10 tetra, 12 hexahedron, 13 wedge, 14 pyramid)";
  }
  std::vector<float> box(6 * (size_t)nc), cen(3 * (size_t)nc);
  for (long long c = 0; c < nc; ++c) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float mag = 0.0f;
    for (int i = 0; i < kinds[c]->n_verts; ++i) {
      const int v = cells[8 * c + i];
      if (v < 0 || v >= nv) return "cell " + std::to_string(c) + " names vertex " + std::to_string(v) + " of " +
                                    std::to_string(nv);
      for (int a = 0; a < 3; ++a) {
        const float x = V[3 * (size_t)v + a];
        if (!std::isfinite(x)) return "vertex " + std::to_string(v) + " is not finite";
        lo[a] = std::min(lo[a], x);
        hi[a] = std::max(hi[a], x);
        mag = std::max(mag, std::fabs(x));
      }
    }
    const float ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    const float pad = 2.0f * tol * ext + 1e-6f * mag;
    for (int a = 0; a < 3; ++a) {
      box[6 * c + a] = lo[a] - pad;
      box[6 * c + 3 + a] = hi[a] + pad;
      cen[3 * c + a] = 0.5f * (lo[a] + hi[a]);
    }
  }
  std::vector<int> idx((size_t)nc), order;
  std::iota(idx.begin(), idx.end(), 0);
  order.reserve((size_t)nc);
  std::vector<Node> nodes;
  nodes.reserve(2 * (size_t)nc / LEAF_CELLS + 2);
  Builder bld{box.data(), cen.data(), idx, nodes, order};
  bld.build(0, nc);
  n_nodes = (unsigned)nodes.size();
  std::vector<int> nbc;
  face_neighbours(cells, kinds.data(), nv, nc, nbc);
  std::vector<int> rec_of((size_t)nc);
  for (size_t k = 0; k < order.size(); ++k) rec_of[(size_t)order[k]] = (int)k;
  const size_t node_off = 2, cell_off = node_off + 2 * nodes.size(), neigh_off = cell_off + (size_t)HEX_REC_UNITS * nc;
  blob.assign(4 * (neigh_off + 2 * (size_t)nc), 0.0f);
  HexHeader H;
  std::memset(&H, 0, sizeof H);
  H.n_nodes = n_nodes;
  H.n_cells = (unsigned)nc;
  H.node_off = (unsigned)node_off;
  H.cell_off = (unsigned)cell_off;
  H.tol = tol;
  H.neigh_off = (unsigned)neigh_off;
  std::memcpy(blob.data(), &H, sizeof H);
  for (size_t k = 0; k < nodes.size(); ++k) {
    float* q = blob.data() + 4 * (node_off + 2 * k);
    const Node& nd = nodes[k];
    q[0] = nd.lo[0]; q[1] = nd.lo[1]; q[2] = nd.lo[2];
    std::memcpy(&q[3], &nd.skip, 4);
    q[4] = nd.hi[0]; q[5] = nd.hi[1]; q[6] = nd.hi[2];
    std::memcpy(&q[7], &nd.leaf, 4);
  }
  for (size_t k = 0; k < order.size(); ++k) {
    const long long c = order[k];
    const KindInfo& K = *kinds[c];
    double P[8][3] = {}, Pv[8][3] = {}, X[8][3], W[8][3];
    for (int i = 0; i < K.n_verts; ++i) {
      const int v = cells[8 * c + i];
      for (int a = 0; a < 3; ++a) {
        P[i][a] = V[3 * (size_t)v + a];
        Pv[i][a] = val[3 * (size_t)v + a];
      }
    }
    kind_coeffs(K.kind, P, X);
    kind_coeffs(K.kind, Pv, W);
    float* q = blob.data() + 4 * (cell_off + (size_t)HEX_REC_UNITS * k);
    for (int i = 0; i < 8; ++i)
      for (int a = 0; a < 3; ++a) {
        q[3 * i + a] = (float)X[i][a];
        q[24 + 3 * i + a] = (float)W[i][a];
      }
    int nbr[8] = {-1, -1, -1, -1, -1, -1, K.kind, -1};
    for (int f = 0; f < K.n_faces; ++f) {
      const int o = nbc[6 * (size_t)c + f];
      nbr[f] = o >= 0 ? (kinds[(size_t)o]->kind << HEX_KIND_SHIFT) | rec_of[(size_t)o] : -1;
    }
    std::memcpy(blob.data() + 4 * (neigh_off + 2 * k), nbr, sizeof nbr);
  }
  return "";
}

}  // namespace streami
