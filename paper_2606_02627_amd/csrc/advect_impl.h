// RK4 particle advection through one or many vector-field blocks (gfx950).
//
// Per particle and step (the paper's update kernel, Sec. 3.1.2): four samples
// of the field -- each a cell location plus a trilinear vec3 interpolation
// (Sec. 2: the update step is dominated by cell location and interpolation;
// Sec. 3.3: a structured field addressed by offset computation) -- the RK4
// combination, then the destination test against the owned bounds; particles
// that leave go to the outbox with destinationID() of their new position
// (Sec. 3.1.1), others append a polyline vertex (Sec. 3.2, assembleOutput).
//
// gfx950 design (measured: a lane's step is a chain of dependent instructions
// and cell-cache refills, so instruction count and latency are what matter;
// the 16-bit kernels at 512^3 keep the VALU busy, the FP32 one does not):
//  * one lane per particle, persistent grid; a wave refills its free lanes
//    from per-XCD work queues over a spatially sorted order, with one atomic
//    per refill (ballot + mbcnt), so long and short trajectories share waves;
//  * each lane keeps the cell it sampled last in registers -- for steady
//    fields its trilinear coefficients in monomial form, for unsteady 16-bit
//    fields the packed corners of the two bracketing slices; a particle moves
//    ~0.1-0.3 cells per step, so most samples re-use them and only a cell
//    change issues the gather;
//  * FP32 fields are stored by default as one 96-byte record of coefficients
//    per cell (the cell layout), so a refill is six 16-byte loads and no
//    arithmetic; node rows hold FP32 (12 B) or FP16/BF16 nodes padded to 8 B;
//  * addresses are 32-bit byte offsets from a per-block base (uniform for a
//    single block), the byte offset of the cell's first corner (or record)
//    doubles as the cache key, and cell location is branch-free (med3 domain
//    test and clamp), skipped for whole steps that start deep inside a block;
//  * vertices go to a log in wave-aggregated runs inside 8192-record chunks,
//    outbox records with one atomic per wave and event.
#pragma once
#include <type_traits>

#include "device.h"
#include "hex.h"

namespace streami {

// SM_LDS: SM_CACHED with each lane's cell record kept in LDS instead of
// registers (steady cell records of one block; an A/B choice, bit-identical).
enum SampleMode { SM_CACHED = 0, SM_UNCACHED = 1, SM_UNSTEADY = 2, SM_UNSTEADY_UNCACHED = 3, SM_LDS = 4 };

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ bool finite3(float3 v) {
  return __builtin_isfinite(v.x) && __builtin_isfinite(v.y) && __builtin_isfinite(v.z);
}

// x/6 correctly rounded via one correction step of x*(1/6): exact whenever
// x/6 is representable (keeps dyadic straight lines bit-exact).
__device__ __forceinline__ float div6(float x) {
  const float r = 1.0f / 6.0f;
  float q = x * r;
  float e = fmaf(-q, 6.0f, x);
  return fmaf(e, r, q);
}

template <int FMT>
struct NodeBytes { static constexpr unsigned v = 8; };
template <>
struct NodeBytes<FMT_F32> { static constexpr unsigned v = 12; };

template <int FMT>
__device__ __forceinline__ float3 load_node(const char* p);

template <>
__device__ __forceinline__ float3 load_node<FMT_F32>(const char* p) {
  const float* q = reinterpret_cast<const float*>(p);
  return make_float3(q[0], q[1], q[2]);
}

template <>
__device__ __forceinline__ float3 load_node<FMT_F16>(const char* p) {
  const uint2 w = *reinterpret_cast<const uint2*>(p);
  _Float16 a = __builtin_bit_cast(_Float16, (unsigned short)(w.x & 0xffffu));
  _Float16 b = __builtin_bit_cast(_Float16, (unsigned short)(w.x >> 16));
  _Float16 c = __builtin_bit_cast(_Float16, (unsigned short)(w.y & 0xffffu));
  return make_float3((float)a, (float)b, (float)c);
}

template <>
__device__ __forceinline__ float3 load_node<FMT_BF16>(const char* p) {
  const uint2 w = *reinterpret_cast<const uint2*>(p);
  return make_float3(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u),
                     __uint_as_float(w.y << 16));
}

// Byte offsets of node index i/j/k within one slice of a block (CELL: of the
// record of the cell whose lowest corner is node i/j/k).
template <int LAYOUT, unsigned NB>
__device__ __forceinline__ unsigned off_x(int i) {
  constexpr int S = brick_shift(LAYOUT), M = (1 << S) - 1;
  if (S) return __umul24((unsigned)(((i >> S) << (3 * S)) + (i & M)), NB);
  if (LAYOUT == LAYOUT_CELL) return __umul24((unsigned)i, 96u);
  return __umul24((unsigned)i, NB);
}
template <int LAYOUT, unsigned NB>
__device__ __forceinline__ unsigned off_y(const BlockDev& B, int j) {
  constexpr int S = brick_shift(LAYOUT), M = (1 << S) - 1;
  if (S) return __umul24((unsigned)(j >> S), B.ys) + (unsigned)(j & M) * ((1u << S) * NB);
  return __umul24((unsigned)j, B.ys);
}
template <int LAYOUT, unsigned NB>
__device__ __forceinline__ unsigned off_z(const BlockDev& B, int k) {
  constexpr int S = brick_shift(LAYOUT), M = (1 << S) - 1;
  if (S) return __umul24((unsigned)(k >> S), B.zs) + (unsigned)(k & M) * ((1u << (2 * S)) * NB);
  return __umul24((unsigned)k, B.zs);
}

// Cell location along one axis, without branches.  Block: defined iff
// 0 <= s <= n-1 (closed); i0 = min(floor(s), n-2), f = s - i0.  Periodic:
// i0 = floor(s) mod n (exact in float for |s| < 2^24), i1 = (i0+1) mod n.
// Undefined coordinates still produce in-range indices.  Without CHECK the
// caller guarantees 0 <= s < n-1 (a step deep inside the block), where the
// test and the clamp change nothing.
template <bool PERIODIC, bool CHECK = true>
__device__ __forceinline__ void locate_axis(float x, float scale, float offs, float fn, float inv_fn,
                                            int& i0, int& i1, float& f, bool& ok) {
  const float s = fmaf(x, scale, offs);
  if (!PERIODIC && !CHECK) {
    const float fl = floorf(s);
    f = s - fl;
    i0 = (int)fl;
    i1 = i0 + 1;
  } else if (PERIODIC) {
    ok = ok && (__builtin_fabsf(s) < 8388608.0f);
    const float fl = floorf(s);
    f = s - fl;
    const float q = floorf(fl * inv_fn);
    float w = fmaf(-q, fn, fl);
    w = (w < 0.0f) ? w + fn : w;
    w = (w >= fn) ? w - fn : w;
    w = __builtin_amdgcn_fmed3f(w, 0.0f, fn - 1.0f);
    i0 = (int)w;
    i1 = (w + 1.0f >= fn) ? 0 : i0 + 1;
  } else {
    ok = ok && (s == __builtin_amdgcn_fmed3f(s, 0.0f, fn - 1.0f));
    // fn >= 2 (validated), so the clamp to [0, fn-2] is one med3
    const float fl = __builtin_amdgcn_fmed3f(floorf(s), 0.0f, fn - 2.0f);
    f = s - fl;
    i0 = (int)fl;
    i1 = i0 + 1;
  }
}

__device__ __forceinline__ float3 trilinear(const float3 c[8], float fx, float fy, float fz) {
  float3 v;
  v.x = lerpf(lerpf(lerpf(c[0].x, c[1].x, fx), lerpf(c[2].x, c[3].x, fx), fy),
              lerpf(lerpf(c[4].x, c[5].x, fx), lerpf(c[6].x, c[7].x, fx), fy), fz);
  v.y = lerpf(lerpf(lerpf(c[0].y, c[1].y, fx), lerpf(c[2].y, c[3].y, fx), fy),
              lerpf(lerpf(c[4].y, c[5].y, fx), lerpf(c[6].y, c[7].y, fx), fy), fz);
  v.z = lerpf(lerpf(lerpf(c[0].z, c[1].z, fx), lerpf(c[2].z, c[3].z, fx), fy),
              lerpf(lerpf(c[4].z, c[5].z, fx), lerpf(c[6].z, c[7].z, fx), fy), fz);
  return v;
}

// A sample from monomial coefficients (to_monomial): 7 fused multiply-adds
// per component.
__device__ __forceinline__ float mono1(float k0, float k1, float k2, float k3, float k4, float k5, float k6, float k7,
                                       float fx, float fy, float fz) {
  const float a0 = fmaf(fz, k4, k0), a1 = fmaf(fz, k6, k2), a2 = fmaf(fz, k5, k1), a3 = fmaf(fz, k7, k3);
  return fmaf(fx, fmaf(fy, a3, a2), fmaf(fy, a1, a0));
}
__device__ __forceinline__ float3 monomial(const float3 k[8], float fx, float fy, float fz) {
  float3 v;
  v.x = mono1(k[0].x, k[1].x, k[2].x, k[3].x, k[4].x, k[5].x, k[6].x, k[7].x, fx, fy, fz);
  v.y = mono1(k[0].y, k[1].y, k[2].y, k[3].y, k[4].y, k[5].y, k[6].y, k[7].y, fx, fy, fz);
  v.z = mono1(k[0].z, k[1].z, k[2].z, k[3].z, k[4].z, k[5].z, k[6].z, k[7].z, fx, fy, fz);
  return v;
}

// sample(): the field value at (x, t); false where the block holds no data
// for x (Sec. 3.1.1).
template <int FMT, int LAYOUT, bool PERIODIC, int MODE>
struct Sampler {
  static constexpr unsigned NB = NodeBytes<FMT>::v;
  unsigned key;
  unsigned gathers = 0;  // cell-cache refills of this lane (a time-sliced refill reads two slices)
  float3 c[8];

  __device__ __forceinline__ void reset() { key = 0xffffffffu; }

  __device__ __forceinline__ void gather(const BlockDev& B, const char* base, unsigned o000, int x0, int x1,
                                         int y0, int y1, int z0, int z1, float3 d[8]) {
    if constexpr (LAYOUT == LAYOUT_CELL) {
      // the record already holds the coefficients (periodic wrap included)
      const float4* q = reinterpret_cast<const float4*>(base + o000);
      const float4 a = q[0], b = q[1], c = q[2], e = q[3], g = q[4], k = q[5];
      d[0] = make_float3(a.x, a.y, a.z);
      d[1] = make_float3(a.w, b.x, b.y);
      d[2] = make_float3(b.z, b.w, c.x);
      d[3] = make_float3(c.y, c.z, c.w);
      d[4] = make_float3(e.x, e.y, e.z);
      d[5] = make_float3(e.w, g.x, g.y);
      d[6] = make_float3(g.z, g.w, k.x);
      d[7] = make_float3(k.y, k.z, k.w);
      return;
    }
    // signed deltas: a periodic wrap steps back to index 0 (a slice is < 2 GiB,
    // so every byte offset and delta fits in int)
    int dx, r10, r01;
    if (PERIODIC || brick_shift(LAYOUT)) {
      dx = (int)off_x<LAYOUT, NB>(x1) - (int)off_x<LAYOUT, NB>(x0);
      r10 = (int)off_y<LAYOUT, NB>(B, y1) - (int)off_y<LAYOUT, NB>(B, y0);
      r01 = (int)off_z<LAYOUT, NB>(B, z1) - (int)off_z<LAYOUT, NB>(B, z0);
    } else {
      dx = (int)NB;
      r10 = (int)B.ys;
      r01 = (int)B.zs;
    }
    // row offsets in 32 bits from the block's (wave-uniform) base, so every
    // load takes the scalar-base + 32-bit-offset form (2-7% faster measured
    // than 64-bit row pointers, once scalar registers do not spill)
    const unsigned o10 = o000 + (unsigned)r10, o01 = o000 + (unsigned)r01, o11 = o01 + (unsigned)r10;
    const char* p00 = base + o000;
    const char* p10 = base + o10;
    const char* p01 = base + o01;
    const char* p11 = base + o11;
    d[0] = load_node<FMT>(p00);
    d[1] = load_node<FMT>(p00 + dx);
    d[2] = load_node<FMT>(p10);
    d[3] = load_node<FMT>(p10 + dx);
    d[4] = load_node<FMT>(p01);
    d[5] = load_node<FMT>(p01 + dx);
    d[6] = load_node<FMT>(p11);
    d[7] = load_node<FMT>(p11 + dx);
  }

  // inner (wave-uniform): every sample of this step is known to lie inside
  __device__ __forceinline__ bool sample(const BlockDev& B, const char* base, float3 x, float t, float3& v,
                                         bool inner = false) {
    bool ok = true;
    int x0, x1, y0, y1, z0, z1;
    float fx, fy, fz;
    if (!PERIODIC && inner) {
      locate_axis<false, false>(x.x, B.scale[0], B.offs[0], B.fn[0], B.inv_fn[0], x0, x1, fx, ok);
      locate_axis<false, false>(x.y, B.scale[1], B.offs[1], B.fn[1], B.inv_fn[1], y0, y1, fy, ok);
      locate_axis<false, false>(x.z, B.scale[2], B.offs[2], B.fn[2], B.inv_fn[2], z0, z1, fz, ok);
    } else {
      locate_axis<PERIODIC>(x.x, B.scale[0], B.offs[0], B.fn[0], B.inv_fn[0], x0, x1, fx, ok);
      locate_axis<PERIODIC>(x.y, B.scale[1], B.offs[1], B.fn[1], B.inv_fn[1], y0, y1, fy, ok);
      locate_axis<PERIODIC>(x.z, B.scale[2], B.offs[2], B.fn[2], B.inv_fn[2], z0, z1, fz, ok);
    }
    const unsigned o000 = off_x<LAYOUT, NB>(x0) + off_y<LAYOUT, NB>(B, y0) + off_z<LAYOUT, NB>(B, z0);
    if (MODE == SM_CACHED) {
      if (ok && o000 != key) {
        gather(B, base, o000, x0, x1, y0, y1, z0, z1, c);
        if (LAYOUT != LAYOUT_CELL) to_monomial(c);
        key = o000;
        ++gathers;
      }
      v = monomial(c, fx, fy, fz);
    } else if (MODE == SM_LDS) {
      // slot threadIdx.x of a 256-lane workgroup: six 16-byte words, word-major,
      // so a wave's lanes touch consecutive words (no bank conflicts)
      __shared__ float4 g_cell_lds[6][256];
      const unsigned tid = threadIdx.x;
      if (ok && o000 != key) {
        const float4* q = reinterpret_cast<const float4*>(base + o000);
        const float4 w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3], w4 = q[4], w5 = q[5];
        g_cell_lds[0][tid] = w0;
        g_cell_lds[1][tid] = w1;
        g_cell_lds[2][tid] = w2;
        g_cell_lds[3][tid] = w3;
        g_cell_lds[4][tid] = w4;
        g_cell_lds[5][tid] = w5;
        key = o000;
        ++gathers;
      }
      const float4 a = g_cell_lds[0][tid], b = g_cell_lds[1][tid], cc = g_cell_lds[2][tid];
      const float4 e = g_cell_lds[3][tid], g = g_cell_lds[4][tid], k = g_cell_lds[5][tid];
      float3 d[8];
      d[0] = make_float3(a.x, a.y, a.z);
      d[1] = make_float3(a.w, b.x, b.y);
      d[2] = make_float3(b.z, b.w, cc.x);
      d[3] = make_float3(cc.y, cc.z, cc.w);
      d[4] = make_float3(e.x, e.y, e.z);
      d[5] = make_float3(e.w, g.x, g.y);
      d[6] = make_float3(g.z, g.w, k.x);
      d[7] = make_float3(k.y, k.z, k.w);
      v = monomial(d, fx, fy, fz);
    } else if (MODE == SM_UNCACHED) {
      if (ok) {
        gather(B, base, o000, x0, x1, y0, y1, z0, z1, c);
        if (LAYOUT != LAYOUT_CELL) to_monomial(c);
        ++gathers;
      }
      v = monomial(c, fx, fy, fz);
    } else {
      // linear blend of the two slices bracketing t, clamped at the ends
      float3 d[8];
      if (ok) {
        ++gathers;
        int s = 0;
        float al = 0.0f;
        if (B.n_slices > 1) {
          const float u = (t - B.t0) * B.inv_sdt;
          const float fs = fminf(fmaxf(floorf(u), 0.0f), (float)(B.n_slices - 2));
          s = (int)fs;
          al = fminf(fmaxf(u - fs, 0.0f), 1.0f);
        }
        const char* b0 = base + (size_t)s * B.slice_bytes;
        gather(B, b0, o000, x0, x1, y0, y1, z0, z1, d);
        float3 v0 = LAYOUT == LAYOUT_CELL ? monomial(d, fx, fy, fz) : trilinear(d, fx, fy, fz);
        if (B.n_slices > 1) {
          gather(B, b0 + B.slice_bytes, o000, x0, x1, y0, y1, z0, z1, d);
          const float3 v1 = LAYOUT == LAYOUT_CELL ? monomial(d, fx, fy, fz) : trilinear(d, fx, fy, fz);
          v0.x = lerpf(v0.x, v1.x, al);
          v0.y = lerpf(v0.y, v1.y, al);
          v0.z = lerpf(v0.z, v1.z, al);
        }
        v = v0;
      } else {
        v = make_float3(0.f, 0.f, 0.f);
      }
    }
    return ok;
  }
};

// Unsteady 16-bit nodes: the corners of the two slices that bracket t are
// cached packed (x|y<<16 per corner, z pairs), 24 VGPRs instead of 48 as
// FP32, and widened at each sample (key: cell and slice).
template <int FMT>
__device__ __forceinline__ float lo16(unsigned w);
template <>
__device__ __forceinline__ float lo16<FMT_BF16>(unsigned w) { return __uint_as_float(w << 16); }
template <>
__device__ __forceinline__ float lo16<FMT_F16>(unsigned w) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
}
template <int FMT>
__device__ __forceinline__ float hi16(unsigned w);
template <>
__device__ __forceinline__ float hi16<FMT_BF16>(unsigned w) { return __uint_as_float(w & 0xffff0000u); }
template <>
__device__ __forceinline__ float hi16<FMT_F16>(unsigned w) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}

template <int FMT, int LAYOUT, bool PERIODIC>
struct PackedSlicesSampler {
  static constexpr unsigned NB = 8;
  static constexpr int NS = 2;
  unsigned key, skey;
  unsigned gathers = 0;  // cell-cache refills of this lane (a time-sliced refill reads two slices)
  unsigned xy[NS][8];  // corner c: x | y << 16
  unsigned zz[NS][4];  // corners 2i, 2i+1: z | z << 16

  __device__ __forceinline__ void reset() { key = 0xffffffffu; skey = 0xffffffffu; }

  __device__ __forceinline__ void gather(const BlockDev& B, const char* base, unsigned o000, int x0, int x1, int y0,
                                         int y1, int z0, int z1, unsigned* xyo, unsigned* zzo) {
    int dx, r10, r01;
    if (PERIODIC || brick_shift(LAYOUT)) {
      dx = (int)off_x<LAYOUT, NB>(x1) - (int)off_x<LAYOUT, NB>(x0);
      r10 = (int)off_y<LAYOUT, NB>(B, y1) - (int)off_y<LAYOUT, NB>(B, y0);
      r01 = (int)off_z<LAYOUT, NB>(B, z1) - (int)off_z<LAYOUT, NB>(B, z0);
    } else {
      dx = (int)NB;
      r10 = (int)B.ys;
      r01 = (int)B.zs;
    }
    const char* p00 = base + o000;
    const char* p10 = p00 + r10;
    const char* p01 = p00 + r01;
    const char* p11 = p01 + r10;
    const uint2 w0 = *reinterpret_cast<const uint2*>(p00), w1 = *reinterpret_cast<const uint2*>(p00 + dx);
    const uint2 w2 = *reinterpret_cast<const uint2*>(p10), w3 = *reinterpret_cast<const uint2*>(p10 + dx);
    const uint2 w4 = *reinterpret_cast<const uint2*>(p01), w5 = *reinterpret_cast<const uint2*>(p01 + dx);
    const uint2 w6 = *reinterpret_cast<const uint2*>(p11), w7 = *reinterpret_cast<const uint2*>(p11 + dx);
    xyo[0] = w0.x; xyo[1] = w1.x; xyo[2] = w2.x; xyo[3] = w3.x;
    xyo[4] = w4.x; xyo[5] = w5.x; xyo[6] = w6.x; xyo[7] = w7.x;
    zzo[0] = (w0.y & 0xffffu) | (w1.y << 16);
    zzo[1] = (w2.y & 0xffffu) | (w3.y << 16);
    zzo[2] = (w4.y & 0xffffu) | (w5.y << 16);
    zzo[3] = (w6.y & 0xffffu) | (w7.y << 16);
  }

  // one component at a time, so only 8 widened values are live at once
  __device__ __forceinline__ static float tri1(float c0, float c1, float c2, float c3, float c4, float c5,
                                               float c6, float c7, float fx, float fy, float fz) {
    return lerpf(lerpf(lerpf(c0, c1, fx), lerpf(c2, c3, fx), fy), lerpf(lerpf(c4, c5, fx), lerpf(c6, c7, fx), fy),
                 fz);
  }
  __device__ __forceinline__ float3 interp(int sl, float fx, float fy, float fz) const {
    const unsigned* a = xy[sl];
    const unsigned* b = zz[sl];
    float3 v;
    v.x = tri1(lo16<FMT>(a[0]), lo16<FMT>(a[1]), lo16<FMT>(a[2]), lo16<FMT>(a[3]), lo16<FMT>(a[4]),
               lo16<FMT>(a[5]), lo16<FMT>(a[6]), lo16<FMT>(a[7]), fx, fy, fz);
    v.y = tri1(hi16<FMT>(a[0]), hi16<FMT>(a[1]), hi16<FMT>(a[2]), hi16<FMT>(a[3]), hi16<FMT>(a[4]),
               hi16<FMT>(a[5]), hi16<FMT>(a[6]), hi16<FMT>(a[7]), fx, fy, fz);
    v.z = tri1(lo16<FMT>(b[0]), hi16<FMT>(b[0]), lo16<FMT>(b[1]), hi16<FMT>(b[1]), lo16<FMT>(b[2]),
               hi16<FMT>(b[2]), lo16<FMT>(b[3]), hi16<FMT>(b[3]), fx, fy, fz);
    return v;
  }

  // inner (wave-uniform): every sample of this step is known to lie inside
  __device__ __forceinline__ bool sample(const BlockDev& B, const char* base, float3 x, float t, float3& v,
                                         bool inner = false) {
    bool ok = true;
    int x0, x1, y0, y1, z0, z1;
    float fx, fy, fz;
    if (!PERIODIC && inner) {
      locate_axis<false, false>(x.x, B.scale[0], B.offs[0], B.fn[0], B.inv_fn[0], x0, x1, fx, ok);
      locate_axis<false, false>(x.y, B.scale[1], B.offs[1], B.fn[1], B.inv_fn[1], y0, y1, fy, ok);
      locate_axis<false, false>(x.z, B.scale[2], B.offs[2], B.fn[2], B.inv_fn[2], z0, z1, fz, ok);
    } else {
      locate_axis<PERIODIC>(x.x, B.scale[0], B.offs[0], B.fn[0], B.inv_fn[0], x0, x1, fx, ok);
      locate_axis<PERIODIC>(x.y, B.scale[1], B.offs[1], B.fn[1], B.inv_fn[1], y0, y1, fy, ok);
      locate_axis<PERIODIC>(x.z, B.scale[2], B.offs[2], B.fn[2], B.inv_fn[2], z0, z1, fz, ok);
    }
    const unsigned o000 = off_x<LAYOUT, NB>(x0) + off_y<LAYOUT, NB>(B, y0) + off_z<LAYOUT, NB>(B, z0);
    int s = 0;
    float al = 0.0f;
    if (B.n_slices > 1) {
      const float u = (t - B.t0) * B.inv_sdt;
      const float fs = fminf(fmaxf(floorf(u), 0.0f), (float)(B.n_slices - 2));
      s = (int)fs;
      al = fminf(fmaxf(u - fs, 0.0f), 1.0f);
    }
    const bool refill = ok && (o000 != key || (unsigned)s != skey);
    gathers += refill ? 1u : 0u;  // counted outside the branch: inside it costs 17 registers here
    if (refill) {
      const char* b0 = base + (size_t)s * B.slice_bytes;
      gather(B, b0, o000, x0, x1, y0, y1, z0, z1, xy[0], zz[0]);
      if (B.n_slices > 1) gather(B, b0 + B.slice_bytes, o000, x0, x1, y0, y1, z0, z1, xy[1], zz[1]);
      key = o000;
      skey = (unsigned)s;
    }
    float3 v0 = interp(0, fx, fy, fz);
    if (B.n_slices > 1) {
      const float3 v1 = interp(1, fx, fy, fz);
      v0.x = lerpf(v0.x, v1.x, al);
      v0.y = lerpf(v0.y, v1.y, al);
      v0.z = lerpf(v0.z, v1.z, al);
    }
    v = v0;
    return ok;
  }
};

// The sampler each (format, mode) uses: the FP32 register cache of the cell's
// monomial coefficients for steady fields (every format), the packed two-slice
// cache for unsteady 16-bit fields, or no cache.  FP32 unsteady sampling is
// uncached (two slices of FP32 corners would not fit the register budget), and
// SM_UNSTEADY_UNCACHED is that plain form for every format.
template <int FMT, int LAYOUT, bool PERIODIC, int MODE>
struct SamplerFor {
  using type = Sampler<FMT, LAYOUT, PERIODIC, MODE == SM_UNSTEADY_UNCACHED ? SM_UNSTEADY : MODE>;
};
template <int MODE>
struct SamplerFor<FMT_F32, LAYOUT_HEX, false, MODE> {
  using type = HexSampler;
};
template <int LAYOUT, bool PERIODIC>
struct SamplerFor<FMT_F16, LAYOUT, PERIODIC, SM_UNSTEADY> {
  using type = PackedSlicesSampler<FMT_F16, LAYOUT, PERIODIC>;
};
template <int LAYOUT, bool PERIODIC>
struct SamplerFor<FMT_BF16, LAYOUT, PERIODIC, SM_UNSTEADY> {
  using type = PackedSlicesSampler<FMT_BF16, LAYOUT, PERIODIC>;
};

// One classical RK4 update from (P, t).  Returns ACTIVE when the step was
// taken (P1 set) or the termination code; for HALO_MISS `fail` is the stage
// point whose sample was undefined.  A non-finite k makes the next stage point
// (or, for k4, the new position) non-finite, so NONFINITE is detected where an
// undefined stage point is non-finite, or the new position is.
template <class S>
__device__ __forceinline__ int rk4_step(S& smp, const BlockDev& B, const char* base, float3 P, float t,
                                        float h, float eps2, float3& P1, float3& fail, bool inner = false) {
  float3 k, q, sum;
  if (!smp.sample(B, base, P, t, k, inner)) { fail = P; return HALO_MISS; }
  if (fmaf(k.x, k.x, fmaf(k.y, k.y, k.z * k.z)) < eps2) return STAGNANT;
  const float hh = 0.5f * h;
  sum = k;  // k1 + 2 k2 + 2 k3 + k4, accumulated as the stages come in
  q = make_float3(fmaf(hh, k.x, P.x), fmaf(hh, k.y, P.y), fmaf(hh, k.z, P.z));
  if (!smp.sample(B, base, q, t + hh, k, inner)) { fail = q; return finite3(q) ? HALO_MISS : NONFINITE; }
  sum = make_float3(fmaf(2.0f, k.x, sum.x), fmaf(2.0f, k.y, sum.y), fmaf(2.0f, k.z, sum.z));
  q = make_float3(fmaf(hh, k.x, P.x), fmaf(hh, k.y, P.y), fmaf(hh, k.z, P.z));
  if (!smp.sample(B, base, q, t + hh, k, inner)) { fail = q; return finite3(q) ? HALO_MISS : NONFINITE; }
  sum = make_float3(fmaf(2.0f, k.x, sum.x), fmaf(2.0f, k.y, sum.y), fmaf(2.0f, k.z, sum.z));
  q = make_float3(fmaf(h, k.x, P.x), fmaf(h, k.y, P.y), fmaf(h, k.z, P.z));
  if (!smp.sample(B, base, q, t + h, k, inner)) { fail = q; return finite3(q) ? HALO_MISS : NONFINITE; }
  sum = make_float3(sum.x + k.x, sum.y + k.y, sum.z + k.z);
  P1 = make_float3(P.x + div6(h * sum.x), P.y + div6(h * sum.y), P.z + div6(h * sum.z));
  if (!finite3(P1)) return NONFINITE;
  return ACTIVE;
}

// destinationID(): flat macrocell id of x, -1 outside the macrocell grid.  The
// advection kernel passes the block descriptor in memory (LDS or global), not
// its register copy: the rank-grid fields are read only at an exit, and keeping
// them in scalar registers for the whole loop would spill others.
__device__ __forceinline__ int dest_id(const BlockDev& B, float3 x) {
  int r0 = B.rcoord[0] + (int)floorf((x.x - B.lo[0]) * B.inv_ext[0]);
  int r1 = B.rcoord[1] + (int)floorf((x.y - B.lo[1]) * B.inv_ext[1]);
  int r2 = B.rcoord[2] + (int)floorf((x.z - B.lo[2]) * B.inv_ext[2]);
  if (r0 < 0 || r0 >= B.rgrid[0] || r1 < 0 || r1 >= B.rgrid[1] || r2 < 0 || r2 >= B.rgrid[2]) return -1;
  return r0 + B.rgrid[0] * (r1 + B.rgrid[1] * r2);
}

__device__ __forceinline__ bool inside(const BlockDev& B, float3 x) {
  return x.x >= B.lo[0] && x.x < B.hi[0] && x.y >= B.lo[1] && x.y < B.hi[1] && x.z >= B.lo[2] &&
         x.z < B.hi[2];
}

// A value every lane holds the same copy of, moved to scalar registers so that
// addresses built from it use the scalar-base form of the memory instructions.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

extern __shared__ BlockDev g_lds_blocks[];

template <int FMT, int LAYOUT, bool PERIODIC, int MODE, bool BATCHED>
__device__ __forceinline__ void advect_body(const AdvectArgs& A) {
  // The log and outbox counters are addressed from A.ctr (they follow the
  // per-call counters), and the rank-grid fields are read from memory at an
  // exit: every 64-bit pointer or field kept in scalar registers for the whole
  // loop spills others, and each spill reload is a VALU instruction.
  constexpr unsigned NB = NodeBytes<FMT>::v;
  BlockDev B0;
  const char* base0 = nullptr;
  if constexpr (BATCHED) {
    for (int i = threadIdx.x; i < A.n_blocks; i += blockDim.x) g_lds_blocks[i] = A.blocks[i];
    __syncthreads();
  } else {
    B0 = A.blocks[0];
    base0 = reinterpret_cast<const char*>(A.nodes) + (size_t)B0.base * NB;
  }
  // interior of a single non-periodic block: a step that starts with its
  // storage coordinates in [ilo, ihi] on every axis samples only where the
  // field is defined and below the last node, so its samples skip the domain
  // test and the clamp (bit-identical results); NaN bounds disable it.  Only
  // the cell layout has the registers for the second path: with node rows
  // it would cost a wave per SIMD (96 -> 100 VGPRs), more than it saves.
  constexpr bool INTERIOR = !BATCHED && !PERIODIC && LAYOUT == LAYOUT_CELL;
  float ilo[3], ihi[3];
  if constexpr (INTERIOR) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float mg = fmaf(fabsf(A.h), B0.vs[a], B0.sl[a]);
      ilo[a] = A.checked ? INFINITY : mg;
      ihi[a] = B0.fn[a] - 1.0f - mg;
    }
  }
  const int lane = __lane_id();
  int p = -1;  // particle index (< 2^31, enforced at seeding)
  float3 P = make_float3(0.f, 0.f, 0.f);
  float tb = 0.f;
  int n = 0, m = 0, nv = 0, stride = 1, blk = 0, left = 0, until_rec = 0;
  const char* lbase = base0;
  // this wave's current log chunk [cpos, cend) (wave-uniform)
  unsigned long long cpos = 0, cend = 0;
  bool log_ok = true;
  unsigned my_steps = 0, my_verts = 0;
  typename SamplerFor<FMT, LAYOUT, PERIODIC, MODE>::type smp;
  smp.reset();
  bool queue_done = false;  // wave-uniform
  const unsigned long long all = __ballot(1);
  int q = (int)(blockIdx.x % (unsigned)A.n_queues), tries = 0;

  while (true) {
    const unsigned long long dead = __ballot(p < 0);
    if (!queue_done && dead != 0 && (__popcll(dead) >= A.refill || dead == all)) {
      const int cnt = __popcll(dead);
      const int leader = __ffsll((long long)dead) - 1;
      // queue q: its range of every class (qn positions); the slots claimed here
      // belong to this queue even when q moves on below
      const int qc = q;
      const unsigned* qrow = A.order ? A.qtab + qc * QTAB_STRIDE : nullptr;
      const long long qn = A.order ? (long long)qrow[0] : A.n_particles;
      unsigned long long qbase = 0;
      if (lane == leader) qbase = atomicAdd(&A.qctr[q * QCTR_STRIDE], (unsigned long long)cnt);
      qbase = __shfl(qbase, leader, 64);
      const long long first = (long long)qbase;
      if (first + cnt >= qn) {  // this queue is used up: continue with the next one
        q = (q + 1 == A.n_queues) ? 0 : q + 1;
        if (++tries == A.n_queues) queue_done = true;
      }
      if (p < 0) {
        const long long k = first + (long long)lanes_below(dead);
        if (k < qn) {
          long long slot = k;
          if (A.order) {  // the queue's range in each class in turn
            unsigned kk = (unsigned)k;
            for (int c = 0; c < A.n_classes; ++c) {
              const unsigned len = qrow[2 + 2 * c];
              if (kk < len) {
                slot = (long long)(qrow[1 + 2 * c] + kk);
                break;
              }
              kk -= len;
            }
          }
          const long long my = A.order ? (long long)A.order[slot] : slot;
          const int4 mt = A.meta[my];
          const float4 ps = A.pos[my];
          if (mt.z == ACTIVE && (!A.windowed || fmaf((float)mt.x, A.h, ps.w) < A.t_end)) {
            p = (int)my;
            P = make_float3(ps.x, ps.y, ps.z);
            tb = ps.w;
            n = mt.x; m = mt.y; nv = mt.w;
            const int4 m2 = A.meta2[my];
            stride = m2.x; blk = m2.y;
            until_rec = stride - n % stride;
            left = A.budget > 0 ? A.budget : 0x7fffffff;
            if constexpr (BATCHED)
              lbase = reinterpret_cast<const char*>(A.nodes) + (size_t)g_lds_blocks[blk].base * NB;
            smp.reset();
          }
        }
      }
    }
    if (queue_done && __ballot(p < 0) == all) break;

    // an outbox record takes P: the new position after an exit, the unchanged
    // one after a halo miss
    int term = ACTIVE;
    int dest = -1;
    bool rec = false;  // a vertex (P, index nv) to append this iteration
    if (p >= 0) {
      const BlockDev& B = BATCHED ? g_lds_blocks[blk] : B0;
      const float t = fmaf((float)n, A.h, tb);
      if (n >= m) {
        term = MAX_STEPS;
      } else if (A.windowed && !(t < A.t_end)) {
        left = 0;  // the window ends here: park the particle, still ACTIVE
      } else {
        float3 P1, fail;
        int st;
        bool inner = false;
        if constexpr (INTERIOR) {
          bool in = true;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float sa = fmaf(a == 0 ? P.x : a == 1 ? P.y : P.z, B0.scale[a], B0.offs[a]);
            in = in && sa >= ilo[a] && sa <= ihi[a];
          }
          inner = __ballot(!in) == 0;  // the lanes taking a step, all inside: a uniform branch
        }
        st = rk4_step(smp, B, lbase, P, t, A.h, A.eps2, P1, fail, inner);
        if (st == ACTIVE) {
          P = P1;
          ++n;
          --left;
          ++my_steps;
          const bool out = !PERIODIC && !inside(B, P);
          const bool on_stride = --until_rec == 0;
          if (on_stride) until_rec = stride;
          rec = out || n == m || on_stride;
          if (out) {
            term = EXIT;
            dest = dest_id(BATCHED ? g_lds_blocks[blk] : A.blocks[0], P);
          } else if (n == m) {
            term = MAX_STEPS;
          }
        } else {
          term = st;
          if (st == HALO_MISS) dest = dest_id(BATCHED ? g_lds_blocks[blk] : A.blocks[0], fail);
          rec = until_rec != stride;  // the final vertex is always kept
        }
      }
    }
    // wave-aggregated vertex append into this wave's log chunk (assembleOutput)
    const unsigned long long vm = __ballot(rec);
    if (vm != 0) {
      const unsigned cnt = (unsigned)__popcll(vm);
      if (cpos + cnt > cend) {
        // mark the unused tail of the old chunk (< 64 records) so fetches skip it
        if (log_ok && cpos + lane < cend) A.log.v[cpos + lane] = make_float4(0.f, 0.f, 0.f, __uint_as_float(LOG_UNUSED));
        unsigned long long nb = 0;
        if (lane == 0) nb = atomicAdd(A.ctr + CTR_N + PER_LOG, (unsigned long long)A.log_chunk);
        nb = uniform_u64(__shfl(nb, 0, 64));
        if (nb + A.log_chunk > (unsigned long long)A.log.cap) {
          log_ok = false;  // cannot happen when the host sized the log; never write past it
          if (lane == 0) atomicOr(&A.ctr[CTR_OVERFLOW], 1ull);
        }
        cpos = nb;
        cend = nb + A.log_chunk;
      }
      if (rec && log_ok) {
        // wave-uniform chunk base (scalar address) + a 32-bit lane offset
        const unsigned k = lanes_below(vm);
        const unsigned long long cu = uniform_u64(cpos);
        float4* vb = A.log.v + cu;
        vb[k] = make_float4(P.x, P.y, P.z, __uint_as_float((unsigned)p));
      }
      if (rec) {
        ++nv;
        ++my_verts;
      }
      cpos += cnt;
    }
    // wave-aggregated outbox append (emitOutgoing)
    const bool emit = (term == EXIT || term == HALO_MISS);
    const unsigned long long em = __ballot(emit);
    if (em != 0) {
      const int leader = __ffsll((long long)em) - 1;
      unsigned long long obase = 0;
      // with segments, each XCD's waves reserve from their own counter (one shared by every
      // wave with an exit cost 4% of the 256^3 launch in contention).  Compiled into the batched
      // and cell-record kernels only: the single-block node-row kernels (few exits per step,
      // VALU-bound at 16 bits) lost 1.4% to the scalar registers the path takes; their segments
      // stay empty
      constexpr bool OB_SEG = BATCHED || LAYOUT == LAYOUT_CELL;
      if (lane == leader) {
        const unsigned long long cnt = (unsigned long long)__popcll(em);
        bool direct = true;
        if (OB_SEG && A.ob_seg_cap > 0) {
          const unsigned seg = blockIdx.x & (OB_SEGS - 1);
          const unsigned long long cap = (unsigned long long)A.ob_seg_cap;
          unsigned long long* sc = A.qctr + (size_t)(MAX_QUEUES + seg) * QCTR_STRIDE;
          const unsigned long long o = atomicAdd(sc, cnt);
          if (o + cnt <= cap) {
            obase = (unsigned long long)A.ob_seg_base + seg * cap + o;
            direct = false;
          } else if (o < cap) {
            sc[1] = o + 1;  // the one reservation that crosses the end: the segment's records stop at o
          }
        }
        if (direct) obase = atomicAdd(A.ctr + CTR_N + PER_OUTBOX, cnt);
      }
      obase = __shfl(obase, leader, 64);
      if (emit) {
        OutRec r;
        r.id = A.ids[p];
        r.pos[0] = P.x; r.pos[1] = P.y; r.pos[2] = P.z;
        r.steps = n;
        r.dest = dest;
        r.code = (short)term;
        r.block = (short)blk;
        A.outbox[obase + lanes_below(em)] = r;
        A.outbox_src[obase + lanes_below(em)] = p;
      }
    }
    if (p >= 0 && (term != ACTIVE || left <= 0)) {
      A.pos[p] = make_float4(P.x, P.y, P.z, tb);
      A.meta[p] = make_int4(n, m, term, nv);
      p = -1;
    }
  }
  // mark the unused tail of this wave's last chunk
  if (log_ok)
    for (unsigned long long r = cpos + lane; r < cend; r += 64)
      A.log.v[r] = make_float4(0.f, 0.f, 0.f, __uint_as_float(LOG_UNUSED));
  const unsigned long long s = wave_sum((unsigned long long)my_steps), v = wave_sum((unsigned long long)my_verts);
  const unsigned long long g = wave_sum((unsigned long long)smp.gathers);
  if (lane == 0) {
    if (s) atomicAdd(&A.ctr[CTR_STEPS], s);
    if (g) atomicAdd(&A.ctr[CTR_GATHERS], g);
    if (v) {
      atomicAdd(&A.ctr[CTR_VERTS], v);
      atomicAdd(A.ctr + CTR_N + PER_LOG_REAL, v);
    }
  }
}

// ---------------------------------------------------------------- surrogate jumps
// Pre-pass of the commutation residual: xh = one plain RK4 step from x.
template <int FMT, int LAYOUT, bool PERIODIC>
__global__ void __launch_bounds__(256) k_sur_pre(SurrogateArgs S) {
  constexpr unsigned NB = NodeBytes<FMT>::v;
  const AdvectArgs& A = S.a;
  const BlockDev B = A.blocks[0];
  const char* base = reinterpret_cast<const char*>(A.nodes) + (size_t)B.base * NB;
  typename SamplerFor<FMT, LAYOUT, PERIODIC, SM_CACHED>::type smp;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < A.n_particles;
       q += (long long)gridDim.x * blockDim.x) {
    if (A.meta[q].z != ACTIVE) continue;
    smp.reset();
    const float4 ps = A.pos[q];
    float3 P1 = make_float3(ps.x, ps.y, ps.z), fail;
    const int4 mt = A.meta[q];
    const float t = fmaf((float)mt.x, A.h, ps.w);
    if (rk4_step(smp, B, base, make_float3(ps.x, ps.y, ps.z), t, A.h, A.eps2, P1, fail) != ACTIVE)
      P1 = make_float3(ps.x, ps.y, ps.z);
    S.xh[3 * q] = P1.x;
    S.xh[3 * q + 1] = P1.y;
    S.xh[3 * q + 2] = P1.z;
  }
}

// Accept the network's jump when its residual is within tol, else advance by
// plain RK4 steps; particles whose step count is not a multiple of the jump,
// or that have fewer than a jump's steps left, take plain steps to the next
// multiple.  One vertex per particle per call at most (record strides are
// multiples of the jump), appended with one atomic per wave.
template <int FMT, int LAYOUT, bool PERIODIC>
__global__ void __launch_bounds__(256) k_sur_apply(SurrogateArgs S) {
  constexpr unsigned NB = NodeBytes<FMT>::v;
  const AdvectArgs& A = S.a;
  const BlockDev B = A.blocks[0];
  const char* base = reinterpret_cast<const char*>(A.nodes) + (size_t)B.base * NB;
  const int lane = __lane_id();
  typename SamplerFor<FMT, LAYOUT, PERIODIC, SM_CACHED>::type smp;
  unsigned my_steps = 0, acc = 0, fb = 0;
  for (long long q0 = blockIdx.x * (long long)blockDim.x; q0 < A.n_particles; q0 += (long long)gridDim.x * blockDim.x) {
    const long long q = q0 + threadIdx.x;
    int term = ACTIVE, dest = -1;
    bool rec = false, active = false;
    float3 P = make_float3(0.f, 0.f, 0.f), opos = P;
    int4 mt = make_int4(0, 0, 0, 0);
    int stride = 1;
    float tb = 0.f;
    if (q < A.n_particles) {
      mt = A.meta[q];
      active = mt.z == ACTIVE;
    }
    if (active) {
      smp.reset();
      const float4 ps = A.pos[q];
      P = make_float3(ps.x, ps.y, ps.z);
      opos = P;
      tb = ps.w;
      stride = A.meta2[q].x;
      int n = mt.x;
      const int m = mt.y;
      int target = ((n / S.jump) + 1) * S.jump;
      if (target > m) target = m;
      bool plain = (n % S.jump) != 0 || m - n < S.jump;
      if (n >= m) {
        term = MAX_STEPS;
      } else if (!plain) {
        const float3 d = make_float3(S.dhat[3 * q], S.dhat[3 * q + 1], S.dhat[3 * q + 2]);
        const float3 Y = make_float3(P.x + d.x, P.y + d.y, P.z + d.z);
        float3 ref, fail;
        float r = 3.0e38f;
        const float t = fmaf((float)n, A.h, tb);
        if (S.kind == 1) {
          if (rk4_step(smp, B, base, P, t, S.jump * A.h, A.eps2, ref, fail) == ACTIVE)
            r = fmaxf(fabsf(Y.x - ref.x), fmaxf(fabsf(Y.y - ref.y), fabsf(Y.z - ref.z)));
        } else {
          const float3 d2 = make_float3(S.dhat2[3 * q], S.dhat2[3 * q + 1], S.dhat2[3 * q + 2]);
          const float3 xh = make_float3(S.xh[3 * q], S.xh[3 * q + 1], S.xh[3 * q + 2]);
          if (rk4_step(smp, B, base, Y, t + S.jump * A.h, A.h, A.eps2, ref, fail) == ACTIVE)
            r = fmaxf(fabsf(xh.x + d2.x - ref.x), fmaxf(fabsf(xh.y + d2.y - ref.y), fabsf(xh.z + d2.z - ref.z)));
        }
        if (r <= S.tol && __builtin_isfinite(Y.x + Y.y + Y.z)) {
          P = Y;
          n += S.jump;
          my_steps += S.jump;
          ++acc;
          if (!PERIODIC && !inside(B, P)) {
            term = EXIT;
            dest = dest_id(B, P);
            opos = P;
          } else if (n == m) {
            term = MAX_STEPS;
          }
          rec = term != ACTIVE || n % stride == 0;
        } else {
          plain = true;
          ++fb;
        }
      }
      if (plain && term == ACTIVE) {
        smp.reset();
        while (n < target) {
          float3 P1, fail;
          const float t = fmaf((float)n, A.h, tb);
          const int st = rk4_step(smp, B, base, P, t, A.h, A.eps2, P1, fail);
          if (st != ACTIVE) {
            term = st;
            if (st == HALO_MISS) {
              dest = dest_id(B, fail);
              opos = P;
            }
            break;
          }
          P = P1;
          ++n;
          ++my_steps;
          if (!PERIODIC && !inside(B, P)) {
            term = EXIT;
            dest = dest_id(B, P);
            opos = P;
            break;
          }
        }
        if (term == ACTIVE && n == m) term = MAX_STEPS;
        rec = term != ACTIVE || n % stride == 0;
      }
      mt.x = n;
    }
    // one log record per recording lane (exact reservation, one atomic per wave)
    const unsigned long long vm = __ballot(rec);
    if (vm) {
      unsigned long long b = 0;
      const int leader = __ffsll((long long)vm) - 1;
      if (lane == leader) b = atomicAdd(A.log.count, (unsigned long long)__popcll(vm));
      b = __shfl(b, leader, 64);
      if (rec) {
        const unsigned long long r = b + lanes_below(vm);
        if (r < (unsigned long long)A.log.cap) {
          A.log.v[r] = make_float4(P.x, P.y, P.z, __uint_as_float((unsigned)q));
        }
        ++mt.w;
      }
      if (lane == leader) {
        atomicAdd(A.log.real, (unsigned long long)__popcll(vm));
        // a record past the reserved log is lost: the call reports it as an error
        if (b + __popcll(vm) > (unsigned long long)A.log.cap) atomicOr(&A.ctr[CTR_OVERFLOW], 1ull);
      }
    }
    const bool emit = term == EXIT || term == HALO_MISS;
    const unsigned long long em = __ballot(emit);
    if (em) {
      const int leader = __ffsll((long long)em) - 1;
      unsigned long long ob = 0;
      if (lane == leader) ob = atomicAdd(A.outbox_count, (unsigned long long)__popcll(em));
      ob = __shfl(ob, leader, 64);
      if (emit) {
        OutRec rr;
        rr.id = A.ids[q];
        rr.pos[0] = opos.x; rr.pos[1] = opos.y; rr.pos[2] = opos.z;
        rr.steps = mt.x;
        rr.dest = dest;
        rr.code = (short)term;
        rr.block = 0;
        A.outbox[ob + lanes_below(em)] = rr;
        A.outbox_src[ob + lanes_below(em)] = (int)q;
      }
    }
    if (active) {
      A.pos[q] = make_float4(P.x, P.y, P.z, tb);
      A.meta[q] = make_int4(mt.x, mt.y, term, mt.w);
    }
  }
  const unsigned long long s = wave_sum(my_steps), a1 = wave_sum(acc), f1 = wave_sum(fb);
  if (lane == 0) {
    if (s) atomicAdd(&A.ctr[CTR_STEPS], s);
    if (a1) atomicAdd(&A.ctr[CTR_ACCEPT], a1);
    if (f1) atomicAdd(&A.ctr[CTR_FALLBACK], f1);
  }
}

template <int FMT>
int launch_surrogate_fmt(const SurrogateArgs& s, int layout, bool periodic, bool pre, int grid, hipStream_t st) {
#define STREAMI_S(LAY, PER)                                                                        if (pre) hipLaunchKernelGGL((k_sur_pre<FMT, LAY, PER>), dim3(grid), dim3(256), 0, st, s);        else hipLaunchKernelGGL((k_sur_apply<FMT, LAY, PER>), dim3(grid), dim3(256), 0, st, s);          return 0;
  if constexpr (FMT == FMT_F32) {
    if (layout == LAYOUT_CELL) {
      if (periodic) { STREAMI_S(LAYOUT_CELL, true) } else { STREAMI_S(LAYOUT_CELL, false) }
    }
  } else {
    if (layout == LAYOUT_CELL) return -1;
  }
  if (layout == LAYOUT_BRICK4) {
    if (periodic) { STREAMI_S(LAYOUT_BRICK4, true) } else { STREAMI_S(LAYOUT_BRICK4, false) }
  } else if (layout == LAYOUT_BRICK8) {
    if (periodic) { STREAMI_S(LAYOUT_BRICK8, true) } else { STREAMI_S(LAYOUT_BRICK8, false) }
  } else {
    if (periodic) { STREAMI_S(LAYOUT_LINEAR, true) } else { STREAMI_S(LAYOUT_LINEAR, false) }
  }
#undef STREAMI_S
}

// With the cell cache in LDS (24 KB per workgroup) at most 6 workgroups fit a CU:
// those kernels are held to 6 waves per SIMD.
template <int FMT, int LAYOUT, bool PERIODIC, int MODE, bool BATCHED>
__global__ void __launch_bounds__(256, MODE == SM_LDS ? 6 : 1) k_advect(AdvectArgs A) {
  advect_body<FMT, LAYOUT, PERIODIC, MODE, BATCHED>(A);
}

template <int FMT, int LAYOUT, bool PERIODIC, int MODE, bool BATCHED>
static void launch_variant(const AdvectArgs& a, int grid, hipStream_t st) {
  const size_t lds = BATCHED ? sizeof(BlockDev) * (size_t)a.n_blocks : 0;
  hipLaunchKernelGGL((k_advect<FMT, LAYOUT, PERIODIC, MODE, BATCHED>), dim3(grid), dim3(256), lds, st, a);
}

// All variants of one storage format.  Periodic blocks are supported for a
// single steady block (the batched and unsteady kernels assume BLOCK boundaries).
template <int FMT>
int launch_advect_fmt(const AdvectArgs& a, int layout, bool periodic, int mode, bool batched, int grid,
                      hipStream_t st) {
#define STREAMI_L(LAY)                                                                              \
  if (batched) {                                                                                    \
    if (periodic) return -1;                                                                        \
    if (mode == SM_CACHED) launch_variant<FMT, LAY, false, SM_CACHED, true>(a, grid, st);           \
    else if (mode == SM_UNCACHED) launch_variant<FMT, LAY, false, SM_UNCACHED, true>(a, grid, st);  \
    else if (mode == SM_UNSTEADY) launch_variant<FMT, LAY, false, SM_UNSTEADY, true>(a, grid, st);  \
    else launch_variant<FMT, LAY, false, SM_UNSTEADY_UNCACHED, true>(a, grid, st);                 \
  } else if (periodic) {                                                                            \
    if (mode == SM_CACHED) launch_variant<FMT, LAY, true, SM_CACHED, false>(a, grid, st);           \
    else if (mode == SM_UNCACHED) launch_variant<FMT, LAY, true, SM_UNCACHED, false>(a, grid, st);  \
    else return -1;                                                                                 \
  } else {                                                                                          \
    if (mode == SM_CACHED) launch_variant<FMT, LAY, false, SM_CACHED, false>(a, grid, st);          \
    else if (mode == SM_UNCACHED) launch_variant<FMT, LAY, false, SM_UNCACHED, false>(a, grid, st); \
    else if (mode == SM_UNSTEADY) launch_variant<FMT, LAY, false, SM_UNSTEADY, false>(a, grid, st); \
    else launch_variant<FMT, LAY, false, SM_UNSTEADY_UNCACHED, false>(a, grid, st);                \
  }                                                                                                 \
  return 0;
  if (FMT == FMT_F32 && mode == SM_UNSTEADY_UNCACHED) mode = SM_UNSTEADY;  // the same sampler
  if constexpr (FMT == FMT_F32) {
    if (layout == LAYOUT_CELL && mode == SM_LDS) {
      if (batched) return -1;
      if (periodic) launch_variant<FMT, LAYOUT_CELL, true, SM_LDS, false>(a, grid, st);
      else launch_variant<FMT, LAYOUT_CELL, false, SM_LDS, false>(a, grid, st);
      return 0;
    }
    if (layout == LAYOUT_CELL) { STREAMI_L(LAYOUT_CELL) }
    if (layout == LAYOUT_HEX) {  // one steady block; the sampler keeps its own cell cache
      if (batched || periodic || mode >= SM_UNSTEADY) return -1;
      launch_variant<FMT, LAYOUT_HEX, false, SM_CACHED, false>(a, grid, st);
      return 0;
    }
  } else {
    if (layout == LAYOUT_CELL || layout == LAYOUT_HEX) return -1;
  }
  if (layout == LAYOUT_BRICK4) {
    STREAMI_L(LAYOUT_BRICK4)
  } else if (layout == LAYOUT_BRICK8) {
    STREAMI_L(LAYOUT_BRICK8)
  } else {
    STREAMI_L(LAYOUT_LINEAR)
  }
#undef STREAMI_L
}

}  // namespace streami
