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
// gfx950 design:
//  * one lane per particle, persistent grid; a wave refills its free lanes
//    from a global work counter with one atomic per refill (ballot + mbcnt),
//    so long and short trajectories share waves without idling;
//  * each lane keeps the 8 corner vectors of the cell it sampled last in
//    registers; a particle moves ~0.1-0.3 cells per step, so most of the four
//    samples of a step re-use them and only a cell change issues the gather;
//  * the outbox append is wave-aggregated (one atomic per wave and event);
//  * nodes are FP32 (12 B) or FP16/BF16 padded to 8 B, so a node is one
//    aligned load; 16-bit values are widened in registers, all arithmetic FP32;
//  * layouts: x-fastest rows, or 4x4x4-node bricks (a cell's 8 corners then
//    span 2-3 cache lines instead of 4-5).
#include "device.h"

namespace streami {

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ bool finite3(float3 v) {
  return __builtin_isfinite(v.x) && __builtin_isfinite(v.y) && __builtin_isfinite(v.z);
}

// x/6 correctly rounded via one Newton-style correction of x*(1/6): exact
// whenever x/6 is representable (keeps dyadic straight lines bit-exact).
__device__ __forceinline__ float div6(float x) {
  const float r = 1.0f / 6.0f;
  float q = x * r;
  float e = fmaf(-q, 6.0f, x);
  return fmaf(e, r, q);
}

template <int FMT>
__device__ __forceinline__ float3 load_node(const void* nodes, long long idx);

template <>
__device__ __forceinline__ float3 load_node<FMT_F32>(const void* nodes, long long idx) {
  const float* p = reinterpret_cast<const float*>(nodes) + idx * 3;
  return make_float3(p[0], p[1], p[2]);
}

template <>
__device__ __forceinline__ float3 load_node<FMT_F16>(const void* nodes, long long idx) {
  uint2 w = reinterpret_cast<const uint2*>(nodes)[idx];
  _Float16 a = __builtin_bit_cast(_Float16, (unsigned short)(w.x & 0xffffu));
  _Float16 b = __builtin_bit_cast(_Float16, (unsigned short)(w.x >> 16));
  _Float16 c = __builtin_bit_cast(_Float16, (unsigned short)(w.y & 0xffffu));
  return make_float3((float)a, (float)b, (float)c);
}

template <>
__device__ __forceinline__ float3 load_node<FMT_BF16>(const void* nodes, long long idx) {
  uint2 w = reinterpret_cast<const uint2*>(nodes)[idx];
  return make_float3(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u),
                     __uint_as_float(w.y << 16));
}

// Cell location along one axis.  Block: defined iff 0 <= s <= n-1 (closed),
// i0 = min(floor(s), n-2), f = s - i0.  Periodic: i0 = floor(s) mod n.
__device__ __forceinline__ bool locate_axis(bool periodic, float x, float scale, float offs, int n,
                                            int& i0, int& i1, float& f) {
  if (periodic) {
    float s = fmaf(x, scale, offs);
    if (!__builtin_isfinite(s)) return false;
    float fl = floorf(s);
    f = s - fl;
    int k = (int)fl % n;
    k += (k < 0) ? n : 0;
    i0 = k;
    i1 = (k + 1 == n) ? 0 : k + 1;
    return true;
  }
  float s = fmaf(x, scale, offs);
  if (!(s >= 0.0f && s <= (float)(n - 1))) return false;
  int k = min((int)s, n - 2);
  i0 = k;
  i1 = k + 1;
  f = s - (float)k;
  return true;
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

template <int FMT, int LAYOUT>
__device__ __forceinline__ void gather8(const BlockDev& B, const void* nodes, long long sbase, int x0,
                                        int x1, int y0, int y1, int z0, int z1, float3 c[8]) {
  const int a0 = ax_off<LAYOUT>(B, x0), a1 = ax_off<LAYOUT>(B, x1);
  const int b0 = ay_off<LAYOUT>(B, y0), b1 = ay_off<LAYOUT>(B, y1);
  const int e0 = az_off<LAYOUT>(B, z0), e1 = az_off<LAYOUT>(B, z1);
  const long long base = B.base + sbase;
  const long long r00 = base + b0 + e0, r10 = base + b1 + e0, r01 = base + b0 + e1, r11 = base + b1 + e1;
  c[0] = load_node<FMT>(nodes, r00 + a0);
  c[1] = load_node<FMT>(nodes, r00 + a1);
  c[2] = load_node<FMT>(nodes, r10 + a0);
  c[3] = load_node<FMT>(nodes, r10 + a1);
  c[4] = load_node<FMT>(nodes, r01 + a0);
  c[5] = load_node<FMT>(nodes, r01 + a1);
  c[6] = load_node<FMT>(nodes, r11 + a0);
  c[7] = load_node<FMT>(nodes, r11 + a1);
}

// sample(): the field value at (x, t), false where the block holds no data
// for x (Sec. 3.1.1).
template <int FMT, int LAYOUT, bool UNSTEADY, bool CACHE>
struct Sampler {
  int key;
  float3 c[8];

  __device__ __forceinline__ void reset() { key = -1; }

  __device__ __forceinline__ bool operator()(const BlockDev& B, const void* nodes, float3 x, float t,
                                             float3& v) {
    int x0, x1, y0, y1, z0, z1;
    float fx, fy, fz;
    const bool per = B.periodic != 0;
    if (!locate_axis(per, x.x, B.scale[0], B.offs[0], B.nst[0], x0, x1, fx)) return false;
    if (!locate_axis(per, x.y, B.scale[1], B.offs[1], B.nst[1], y0, y1, fy)) return false;
    if (!locate_axis(per, x.z, B.scale[2], B.offs[2], B.nst[2], z0, z1, fz)) return false;
    if (!UNSTEADY) {
      const int k = x0 + B.nst[0] * (y0 + B.nst[1] * z0);
      if (!CACHE || k != key) {
        gather8<FMT, LAYOUT>(B, nodes, 0, x0, x1, y0, y1, z0, z1, c);
        key = k;
      }
      v = trilinear(c, fx, fy, fz);
      return true;
    } else {
      // linear blend of the two slices bracketing t, clamped at the ends
      int s = 0;
      float al = 0.0f;
      if (B.n_slices > 1) {
        float u = (t - B.t0) * B.inv_sdt;
        float fs = fminf(fmaxf(floorf(u), 0.0f), (float)(B.n_slices - 2));
        s = (int)fs;
        al = fminf(fmaxf(u - fs, 0.0f), 1.0f);
      }
      float3 d[8];
      gather8<FMT, LAYOUT>(B, nodes, (long long)s * B.slice_nodes, x0, x1, y0, y1, z0, z1, d);
      float3 v0 = trilinear(d, fx, fy, fz);
      if (B.n_slices > 1) {
        gather8<FMT, LAYOUT>(B, nodes, (long long)(s + 1) * B.slice_nodes, x0, x1, y0, y1, z0, z1, d);
        float3 v1 = trilinear(d, fx, fy, fz);
        v0.x = lerpf(v0.x, v1.x, al);
        v0.y = lerpf(v0.y, v1.y, al);
        v0.z = lerpf(v0.z, v1.z, al);
      }
      v = v0;
      return true;
    }
  }
};

// One classical RK4 update from (P, t).  Returns ACTIVE when the step was
// taken (P1 set) or the termination code; for HALO_MISS `fail` is the stage
// point whose sample was undefined.
template <class S>
__device__ __forceinline__ int rk4_step(S& smp, const BlockDev& B, const void* nodes, float3 P,
                                        float t, float h, float eps2, float3& P1, float3& fail) {
  float3 k1, k2, k3, k4, q;
  if (!smp(B, nodes, P, t, k1)) { fail = P; return HALO_MISS; }
  if (!finite3(k1)) return NONFINITE;
  if (fmaf(k1.x, k1.x, fmaf(k1.y, k1.y, k1.z * k1.z)) < eps2) return STAGNANT;
  const float hh = 0.5f * h;
  q = make_float3(fmaf(hh, k1.x, P.x), fmaf(hh, k1.y, P.y), fmaf(hh, k1.z, P.z));
  if (!smp(B, nodes, q, t + hh, k2)) { fail = q; return HALO_MISS; }
  if (!finite3(k2)) return NONFINITE;
  q = make_float3(fmaf(hh, k2.x, P.x), fmaf(hh, k2.y, P.y), fmaf(hh, k2.z, P.z));
  if (!smp(B, nodes, q, t + hh, k3)) { fail = q; return HALO_MISS; }
  if (!finite3(k3)) return NONFINITE;
  q = make_float3(fmaf(h, k3.x, P.x), fmaf(h, k3.y, P.y), fmaf(h, k3.z, P.z));
  if (!smp(B, nodes, q, t + h, k4)) { fail = q; return HALO_MISS; }
  if (!finite3(k4)) return NONFINITE;
  float sx = fmaf(2.0f, k3.x, fmaf(2.0f, k2.x, k1.x)) + k4.x;
  float sy = fmaf(2.0f, k3.y, fmaf(2.0f, k2.y, k1.y)) + k4.y;
  float sz = fmaf(2.0f, k3.z, fmaf(2.0f, k2.z, k1.z)) + k4.z;
  P1 = make_float3(P.x + div6(h * sx), P.y + div6(h * sy), P.z + div6(h * sz));
  if (!finite3(P1)) return NONFINITE;
  return ACTIVE;
}

// destinationID(): flat macrocell id of x, -1 outside the macrocell grid.
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

__device__ __forceinline__ unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

extern __shared__ BlockDev g_lds_blocks[];

template <int FMT, int LAYOUT, bool UNSTEADY, bool CACHE, bool BATCHED>
__global__ void __launch_bounds__(256) k_advect(AdvectArgs A) {
  BlockDev B0;
  if constexpr (BATCHED) {
    for (int i = threadIdx.x; i < A.n_blocks; i += blockDim.x) g_lds_blocks[i] = A.blocks[i];
    __syncthreads();
  } else {
    B0 = A.blocks[0];
  }
  const int lane = __lane_id();
  long long p = -1;
  float3 P = make_float3(0.f, 0.f, 0.f);
  float tb = 0.f;
  int n = 0, m = 0, nv = 0, stride = 1, vcap = 0, blk = 0, left = 0;
  long long vb = 0;
  unsigned long long my_steps = 0, my_verts = 0;
  Sampler<FMT, LAYOUT, UNSTEADY, CACHE> smp;
  smp.reset();
  bool queue_done = false;  // wave-uniform
  const unsigned long long all = __ballot(1);

  while (true) {
    const unsigned long long dead = __ballot(p < 0);
    if (!queue_done && dead != 0 && (__popcll(dead) >= A.refill || dead == all)) {
      const int cnt = __popcll(dead);
      const int leader = __ffsll((long long)dead) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(&A.ctr[CTR_QUEUE], (unsigned long long)cnt);
      base = __shfl(base, leader, 64);
      if (base + cnt >= (unsigned long long)A.n_particles) queue_done = true;
      if (p < 0) {
        const long long my = (long long)(base + lanes_below(dead));
        if (my < A.n_particles) {
          const int4 mt = A.meta[my];
          if (mt.z == ACTIVE) {
            p = my;
            const float4 ps = A.pos[my];
            P = make_float3(ps.x, ps.y, ps.z);
            tb = ps.w;
            n = mt.x; m = mt.y; nv = mt.w;
            const int4 m2 = A.meta2[my];
            stride = m2.x; blk = m2.y; vcap = m2.z;
            vb = A.vbase[my];
            left = A.budget > 0 ? A.budget : 0x7fffffff;
            smp.reset();
          }
        }
      }
    }
    if (queue_done && __ballot(p < 0) == all) break;

    int term = ACTIVE;
    int dest = -1;
    float3 opos = P;
    if (p >= 0) {
      const BlockDev& B = BATCHED ? g_lds_blocks[blk] : B0;
      if (n >= m) {
        term = MAX_STEPS;
      } else {
        float3 P1, fail;
        const float t = fmaf((float)n, A.h, tb);
        const int st = rk4_step(smp, B, A.nodes, P, t, A.h, A.eps2, P1, fail);
        if (st == ACTIVE) {
          P = P1;
          ++n;
          --left;
          ++my_steps;
          const bool out = !B.periodic && !inside(B, P);
          if (out || n == m || (n % stride) == 0) {
            if (nv < vcap) {
              float* w = A.verts + (vb + nv) * 3;
              w[0] = P.x; w[1] = P.y; w[2] = P.z;
            }
            ++nv;
            ++my_verts;
          }
          if (out) {
            term = EXIT;
            dest = dest_id(B, P);
            opos = P;
          } else if (n == m) {
            term = MAX_STEPS;
          }
        } else {
          term = st;
          if (st == HALO_MISS) {
            dest = dest_id(B, fail);
            opos = P;
          }
          if (n % stride != 0) {  // the final vertex is always kept
            if (nv < vcap) {
              float* w = A.verts + (vb + nv) * 3;
              w[0] = P.x; w[1] = P.y; w[2] = P.z;
            }
            ++nv;
            ++my_verts;
          }
        }
      }
    }
    // wave-aggregated outbox append (emitOutgoing)
    const bool emit = (term == EXIT || term == HALO_MISS);
    const unsigned long long em = __ballot(emit);
    if (em != 0) {
      const int leader = __ffsll((long long)em) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(A.outbox_count, (unsigned long long)__popcll(em));
      base = __shfl(base, leader, 64);
      if (emit) {
        OutRec r;
        r.id = A.ids[p];
        r.pos[0] = opos.x; r.pos[1] = opos.y; r.pos[2] = opos.z;
        r.steps = n;
        r.dest = dest;
        r.code = (short)term;
        r.block = (short)blk;
        A.outbox[base + lanes_below(em)] = r;
      }
    }
    if (p >= 0 && (term != ACTIVE || left <= 0)) {
      A.pos[p] = make_float4(P.x, P.y, P.z, tb);
      A.meta[p] = make_int4(n, m, term, nv);
      p = -1;
    }
  }
  const unsigned long long s = wave_sum(my_steps), v = wave_sum(my_verts);
  if (lane == 0) {
    if (s) atomicAdd(&A.ctr[CTR_STEPS], s);
    if (v) atomicAdd(&A.ctr[CTR_VERTS], v);
  }
}

// ---------------------------------------------------------------- dispatch
typedef void (*AdvectFn)(AdvectArgs);

template <int FMT, int LAYOUT, bool UNSTEADY, bool CACHE, bool BATCHED>
static void launch_one(const AdvectArgs& a, int grid, hipStream_t st) {
  size_t lds = BATCHED ? sizeof(BlockDev) * (size_t)a.n_blocks : 0;
  hipLaunchKernelGGL((k_advect<FMT, LAYOUT, UNSTEADY, CACHE, BATCHED>), dim3(grid), dim3(256), lds, st, a);
}

template <int FMT, int LAYOUT>
static int launch_fl(const AdvectArgs& a, bool unsteady, bool cache, bool batched, int grid, hipStream_t st) {
  if (unsteady) {
    if (batched) launch_one<FMT, LAYOUT, true, false, true>(a, grid, st);
    else launch_one<FMT, LAYOUT, true, false, false>(a, grid, st);
  } else if (cache) {
    if (batched) launch_one<FMT, LAYOUT, false, true, true>(a, grid, st);
    else launch_one<FMT, LAYOUT, false, true, false>(a, grid, st);
  } else {
    if (batched) launch_one<FMT, LAYOUT, false, false, true>(a, grid, st);
    else launch_one<FMT, LAYOUT, false, false, false>(a, grid, st);
  }
  return 0;
}

int launch_advect(const AdvectArgs& a, int fmt, int layout, bool unsteady, bool cache, bool batched,
                  int grid, hipStream_t st) {
  if (fmt == FMT_F32) {
    if (layout == LAYOUT_BRICK4) return launch_fl<FMT_F32, LAYOUT_BRICK4>(a, unsteady, cache, batched, grid, st);
    return launch_fl<FMT_F32, LAYOUT_LINEAR>(a, unsteady, cache, batched, grid, st);
  } else if (fmt == FMT_F16) {
    if (layout == LAYOUT_BRICK4) return launch_fl<FMT_F16, LAYOUT_BRICK4>(a, unsteady, cache, batched, grid, st);
    return launch_fl<FMT_F16, LAYOUT_LINEAR>(a, unsteady, cache, batched, grid, st);
  } else {
    if (layout == LAYOUT_BRICK4) return launch_fl<FMT_BF16, LAYOUT_BRICK4>(a, unsteady, cache, batched, grid, st);
    return launch_fl<FMT_BF16, LAYOUT_LINEAR>(a, unsteady, cache, batched, grid, st);
  }
}

}  // namespace streami
