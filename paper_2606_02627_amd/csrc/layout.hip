// Field ingest (node re-layout), particle seeding, line packing and small fill
// kernels.  Ingest copies the caller's x-fastest node array into the library's
// node pool in the handle's layout (or, for the cell layout, computes each
// cell's interpolation coefficients); 16-bit nodes are padded to 8 bytes so a
// node is one aligned 64-bit load in the advection kernel.
#include <algorithm>

#include "device.h"
#include "seed.h"

namespace streami {

template <int FMT, int LAYOUT>
__global__ void k_ingest(const void* src, void* pool, BlockDev B, int nx, int ny, int nz, int n_slices) {
  const long long per_slice = (long long)nx * ny * nz;
  const long long total = per_slice * n_slices;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long s = t / per_slice;
    long long r = t - s * per_slice;
    const int k = (int)(r / ((long long)nx * ny));
    r -= (long long)k * nx * ny;
    const int j = (int)(r / nx);
    const int i = (int)(r - (long long)j * nx);
    const long long dst = B.base + s * B.slice_nodes + ax_off<LAYOUT>(B, i) + ay_off<LAYOUT>(B, j) +
                          az_off<LAYOUT>(B, k);
    if (FMT == FMT_F32) {
      const float* a = reinterpret_cast<const float*>(src) + t * 3;
      float* b = reinterpret_cast<float*>(pool) + dst * 3;
      b[0] = a[0]; b[1] = a[1]; b[2] = a[2];
    } else {
      const unsigned short* a = reinterpret_cast<const unsigned short*>(src) + t * 3;
      uint2 w;
      w.x = (unsigned)a[0] | ((unsigned)a[1] << 16);
      w.y = (unsigned)a[2];
      reinterpret_cast<uint2*>(pool)[dst] = w;
    }
  }
}

// Cell layout (FP32): the record of cell (i, j, k) of slice s holds the
// monomial coefficients of the trilinear interpolant over its 8 corner nodes
// (corner index a + 2b + 4c for node (i+a, j+b, k+c), wrapped on a periodic
// block), 24 floats in corner-major, xyz-minor order.
__global__ void k_ingest_cell(const float* src, float4* pool, BlockDev B, int nx, int ny, int nz, int n_slices) {
  const int per = B.periodic;
  const int cx = per ? nx : nx - 1, cy = per ? ny : ny - 1, cz = per ? nz : nz - 1;
  const long long per_slice = (long long)cx * cy * cz;
  const long long total = per_slice * n_slices;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long s = t / per_slice;
    long long r = t - s * per_slice;
    const int k = (int)(r / ((long long)cx * cy));
    const long long rk = r - (long long)k * cx * cy;
    const int j = (int)(rk / cx);
    const int i = (int)(rk - (long long)j * cx);
    float3 c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int ii = i + (q & 1), jj = j + ((q >> 1) & 1), kk = k + (q >> 2);
      if (ii == nx) ii = 0;
      if (jj == ny) jj = 0;
      if (kk == nz) kk = 0;
      const float* a = src + 3 * (((s * nz + kk) * ny + jj) * (long long)nx + ii);
      c[q] = make_float3(a[0], a[1], a[2]);
    }
    to_monomial(c);
    // B.base and B.slice_nodes count 12-byte units: 8 per 96-byte record
    float4* o = pool + (B.base + s * B.slice_nodes) * 3 / 4 + r * 6;
    o[0] = make_float4(c[0].x, c[0].y, c[0].z, c[1].x);
    o[1] = make_float4(c[1].y, c[1].z, c[2].x, c[2].y);
    o[2] = make_float4(c[2].z, c[3].x, c[3].y, c[3].z);
    o[3] = make_float4(c[4].x, c[4].y, c[4].z, c[5].x);
    o[4] = make_float4(c[5].y, c[5].z, c[6].x, c[6].y);
    o[5] = make_float4(c[6].z, c[7].x, c[7].y, c[7].z);
  }
}

// max |v_a| per component over n nodes of the caller's array (xyz per node,
// FP32 or 16-bit), as the bit pattern of a non-negative float so that an
// unsigned max orders it; a NaN node wins (its pattern exceeds Inf's), so a
// field with a NaN never passes the interior test
__global__ void k_max_abs(const void* src, int fmt, long long n, unsigned* out) {
  unsigned m[3] = {0u, 0u, 0u};
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float v;
      if (fmt == FMT_F32) {
        v = reinterpret_cast<const float*>(src)[3 * t + a];
      } else {
        const unsigned short u = reinterpret_cast<const unsigned short*>(src)[3 * t + a];
        v = fmt == FMT_F16 ? (float)__builtin_bit_cast(_Float16, u) : __uint_as_float((unsigned)u << 16);
      }
      const unsigned b = __float_as_uint(v) & 0x7fffffffu;
      m[a] = b > m[a] ? b : m[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    unsigned w = m[a];
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned o = __shfl_xor(w, off, 64);
      w = o > w ? o : w;
    }
    if (__lane_id() == 0 && w) atomicMax(out + a, w);
  }
}

int launch_max_abs(const void* src, int fmt, long long n, unsigned* out, hipStream_t st) {
  int grid = (int)((n + 255) / 256);
  if (grid > 512) grid = 512;  // grid-stride: few waves, so few atomics on the three maxima
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_max_abs, dim3(grid), dim3(256), 0, st, src, fmt, n, out);
  return 0;
}

int launch_ingest(const void* src, void* pool, const BlockDev& B, int fmt, int layout, int nx, int ny,
                  int nz, int n_slices, hipStream_t st) {
  const long long total = (long long)nx * ny * nz * n_slices;
  int grid = (int)((total + 255) / 256);
  if (grid > 65536) grid = 65536;
  if (grid < 1) grid = 1;
#define STREAMI_INGEST(F, L) hipLaunchKernelGGL((k_ingest<F, L>), dim3(grid), dim3(256), 0, st, src, pool, B, nx, ny, nz, n_slices)
  if (layout == LAYOUT_CELL) {
    if (fmt != FMT_F32) return -1;
    hipLaunchKernelGGL(k_ingest_cell, dim3(grid), dim3(256), 0, st, reinterpret_cast<const float*>(src),
                       reinterpret_cast<float4*>(pool), B, nx, ny, nz, n_slices);
  } else if (layout == LAYOUT_BRICK4) {
    if (fmt == FMT_F32) STREAMI_INGEST(FMT_F32, LAYOUT_BRICK4); else STREAMI_INGEST(FMT_F16, LAYOUT_BRICK4);
  } else if (layout == LAYOUT_BRICK8) {
    if (fmt == FMT_F32) STREAMI_INGEST(FMT_F32, LAYOUT_BRICK8); else STREAMI_INGEST(FMT_F16, LAYOUT_BRICK8);
  } else {
    if (fmt == FMT_F32) STREAMI_INGEST(FMT_F32, LAYOUT_LINEAR); else STREAMI_INGEST(FMT_F16, LAYOUT_LINEAR);
  }
#undef STREAMI_INGEST
  return 0;
}

// Initialise n particles at [first, first+n): positions, ids, limits; append
// the seed as vertex 0 of its line to the vertex log (one atomic per wave); a
// seed outside the owned bounds of a non-periodic block ends at once (EXIT,
// 0 steps) and goes to the outbox.
constexpr int SEED_THREADS = 1024;  // one log reservation per 16 waves

// Initialise the particles of up to SEED_JOBS batches in one launch: each
// batch (job) owns a run of workgroups starting at wg0, and its particle i
// goes to slot first + i: positions, ids, limits; the seed is vertex 0 of its
// line in the vertex log (one reservation per workgroup); a seed outside the
// owned bounds of a non-periodic block ends at once (EXIT, 0 steps) and goes
// to the outbox.
__global__ void __launch_bounds__(SEED_THREADS) k_seed(SeedJobs J, const BlockDev* blocks, float4* pos,
                                                       int4* meta, int4* meta2, unsigned long long* pid,
                                                       VertexLog log, OutRec* outbox, int* outbox_src,
                                                       unsigned long long* outbox_count) {
  int jb = 0;  // the job of this workgroup (uniform): the last one starting at or before it
  for (int j = 1; j < J.n_jobs; ++j)
    if (J.j[j].wg0 <= blockIdx.x) jb = j;
  const SeedJob& S = J.j[jb];
  const long long i = (long long)(blockIdx.x - S.wg0) * blockDim.x + threadIdx.x;
  const long long n = S.n;
  const int blk = S.blk;
  const BlockDev& B = blocks[blk];
  bool emit = false;
  const long long q = S.first + i;
  float3 x = make_float3(0.f, 0.f, 0.f);
  unsigned long long id = 0;
  if (i < n) {
    x = make_float3(S.xyz[3 * i], S.xyz[3 * i + 1], S.xyz[3 * i + 2]);
    id = S.ids ? S.ids[i] : S.auto_id0 + (unsigned long long)i;
    const int m = S.max_steps ? S.max_steps[i] : J.default_max;
    bool out = false;
    if (!B.periodic)
      out = !(x.x >= B.lo[0] && x.x < B.hi[0] && x.y >= B.lo[1] && x.y < B.hi[1] && x.z >= B.lo[2] &&
              x.z < B.hi[2]);
    pos[q] = make_float4(x.x, x.y, x.z, S.t_births ? S.t_births[i] : J.t_birth);
    meta[q] = make_int4(0, m, out ? EXIT : ACTIVE, 1);
    meta2[q] = make_int4(J.stride, blk, m / J.stride + 2, 0);
    pid[q] = id;
    emit = out;
  }
  // vertex 0 of every new line (the host sized the log for it): one
  // reservation per workgroup, so that a million seeds do not serialise on
  // the log counter
  __shared__ unsigned s_cnt[SEED_THREADS / 64];
  __shared__ unsigned long long s_base;
  const unsigned long long vm = __ballot(i < n);
  const int wv = threadIdx.x >> 6, lane = __lane_id();
  if (lane == 0) s_cnt[wv] = (unsigned)__popcll(vm);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += s_cnt[w];
    s_base = tot ? atomicAdd(log.count, (unsigned long long)tot) : 0ull;
    if (blockIdx.x == S.wg0) atomicAdd(log.real, (unsigned long long)n);  // once per job
  }
  __syncthreads();
  if (i < n) {
    unsigned long long r = s_base;
    for (int w = 0; w < wv; ++w) r += s_cnt[w];
    r += __builtin_amdgcn_mbcnt_hi((unsigned)(vm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)vm, 0u));
    if (r < (unsigned long long)log.cap) {
      log.v[r] = make_float4(x.x, x.y, x.z, __uint_as_float((unsigned)q));
    }
  }
  const unsigned long long em = __ballot(emit);
  if (em) {
    const int lane = __lane_id();
    const int leader = __ffsll((long long)em) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(outbox_count, (unsigned long long)__popcll(em));
    base = __shfl(base, leader, 64);
    if (emit) {
      const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(em >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)em, 0u));
      int r0 = B.rcoord[0] + (int)floorf((x.x - B.lo[0]) * B.inv_ext[0]);
      int r1 = B.rcoord[1] + (int)floorf((x.y - B.lo[1]) * B.inv_ext[1]);
      int r2 = B.rcoord[2] + (int)floorf((x.z - B.lo[2]) * B.inv_ext[2]);
      int dest = (r0 < 0 || r0 >= B.rgrid[0] || r1 < 0 || r1 >= B.rgrid[1] || r2 < 0 || r2 >= B.rgrid[2])
                     ? -1 : r0 + B.rgrid[0] * (r1 + B.rgrid[1] * r2);
      OutRec r;
      r.id = id;
      r.pos[0] = x.x; r.pos[1] = x.y; r.pos[2] = x.z;
      r.steps = 0;
      r.dest = dest;
      r.code = (short)EXIT;
      r.block = (short)blk;
      outbox[base + below] = r;
      outbox_src[base + below] = (int)q;
    }
  }
}

int launch_seed(const SeedJobs& J, unsigned n_wg, const BlockDev* blocks, float4* pos, int4* meta, int4* meta2,
                unsigned long long* pid, const VertexLog& log, OutRec* outbox, int* outbox_src,
                unsigned long long* outbox_count, hipStream_t st) {
  if (J.n_jobs <= 0 || n_wg == 0) return 0;
  hipLaunchKernelGGL(k_seed, dim3(n_wg), dim3(SEED_THREADS), 0, st, J, blocks, pos, meta, meta2, pid, log, outbox,
                     outbox_src, outbox_count);
  return 0;
}

// row_of[idx[r]] = r for the requested rows (row_of was filled with -1).
__global__ void k_mark_rows(const long long* idx, long long count, int* row_of) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < count;
       r += (long long)gridDim.x * blockDim.x)
    row_of[idx[r]] = (int)r;
}

int launch_mark_rows(const long long* idx, long long count, int* row_of, hipStream_t st) {
  if (count <= 0) return 0;
  long long grid = (count + 255) / 256;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_mark_rows, dim3((unsigned)grid), dim3(256), 0, st, idx, count, row_of);
  return 0;
}

__global__ void k_fill_u32(unsigned* p, long long n, unsigned v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

int launch_fill_u32(unsigned* p, long long n, unsigned v, hipStream_t st) {
  if (n <= 0) return 0;
  long long grid = (n + 255) / 256;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)grid), dim3(256), 0, st, p, n, v);
  return 0;
}

__global__ void k_fill_u64(unsigned long long* p, long long n, unsigned long long v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

int launch_fill_u64(unsigned long long* p, long long n, unsigned long long v, hipStream_t st);

// Vertex bound of the jobs' device step limits: sum of m/stride + 2, the
// largest m, and a flag for a negative m, accumulated into out[0..2] (the
// caller clears it); grid-stride over every job in turn
__global__ void k_seed_bound(SeedJobs J, unsigned long long* out) {
  unsigned long long s = 0, mx = 0, neg = 0, mn = ~0ull;
  const long long t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x, dt = (long long)gridDim.x * blockDim.x;
  for (int j = 0; j < J.n_jobs; ++j) {
    const int* ms = J.j[j].max_steps;
    for (long long i = t0; i < J.j[j].n; i += dt) {
      const int m = ms[i];
      if (m < 0) {
        neg = 1;
      } else {
        s += (unsigned long long)(m / J.stride + 2);
        mx = mx > (unsigned long long)m ? mx : (unsigned long long)m;
        mn = mn < (unsigned long long)m ? mn : (unsigned long long)m;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    const unsigned long long m2 = __shfl_xor(mx, o, 64);
    mx = mx > m2 ? mx : m2;
    const unsigned long long m3 = __shfl_xor(mn, o, 64);
    mn = mn < m3 ? mn : m3;
    neg |= __shfl_xor(neg, o, 64);
  }
  if (__lane_id() == 0) {
    if (s) atomicAdd(&out[0], s);
    if (mx) atomicMax(&out[1], mx);
    if (mn != ~0ull) atomicMin(&out[3], mn);
    if (neg) atomicOr(&out[2], neg);
  }
}

// at most 64 workgroups, so the three result atomics do not serialise
// Seed points on a control shape (Sec. 3.1.2's convenience seeding): point (i, j), i fastest,
// of an nu x nv midpoint grid on the parallelogram o + s u + t v, s = (2i+1)/(2nu),
// t = (2j+1)/(2nv); a line segment is the case nv = 1, v = 0.  FP32: the parameters are
// correctly rounded quotients and each coordinate is two fused multiply-adds.
__global__ void k_seed_shape(float ox, float oy, float oz, float ux, float uy, float uz, float vx, float vy, float vz,
                             long long nu, long long nv, float* out) {
  const long long n = nu * nv;
  const float du = (float)(2 * nu), dv = (float)(2 * nv);
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
    const long long i = k % nu, j = k / nu;
    const float s = (float)(2 * i + 1) / du, t = (float)(2 * j + 1) / dv;
    out[3 * k + 0] = fmaf(s, ux, fmaf(t, vx, ox));
    out[3 * k + 1] = fmaf(s, uy, fmaf(t, vy, oy));
    out[3 * k + 2] = fmaf(s, uz, fmaf(t, vz, oz));
  }
}

int launch_seed_shape(const double o[3], const double u[3], const double v[3], long long nu, long long nv, float* out,
                      hipStream_t st) {
  const long long n = nu * nv;
  if (n <= 0) return 0;
  const long long grid = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_seed_shape, dim3((unsigned)grid), dim3(256), 0, st, (float)o[0], (float)o[1], (float)o[2],
                     (float)u[0], (float)u[1], (float)u[2], (float)v[0], (float)v[1], (float)v[2], nu, nv, out);
  return 0;
}

int launch_seed_bound(const SeedJobs& J, long long total, unsigned long long* out, hipStream_t st) {
  long long grid = (total + 255) / 256;
  if (grid > 64) grid = 64;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_seed_bound, dim3((unsigned)grid), dim3(256), 0, st, J, out);
  return 0;
}

int launch_fill_u64(unsigned long long* p, long long n, unsigned long long v, hipStream_t st) {
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, st, p, n, v);
  return 0;
}

// Per-particle line metadata of a range: n_verts (clamped to capacity), steps, codes, ids.
__global__ void k_gather_meta(const long long* idx, long long count, const int4* meta, const int4* meta2,
                              const unsigned long long* pid, long long* nverts, int* steps, int* codes,
                              unsigned long long* ids) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < count;
       r += (long long)gridDim.x * blockDim.x) {
    const long long q = idx[r];
    const int4 mt = meta[q];
    const int vcap = meta2[q].z;
    nverts[r] = mt.w < vcap ? mt.w : vcap;
    steps[r] = mt.x;
    codes[r] = mt.z;
    ids[r] = pid[q];
  }
}

int launch_gather_meta(const long long* idx, long long count, const int4* meta, const int4* meta2,
                       const unsigned long long* pid, long long* nverts, int* steps, int* codes,
                       unsigned long long* ids, hipStream_t st) {
  if (count <= 0) return 0;
  int grid = (int)((count + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_gather_meta, dim3(grid), dim3(256), 0, st, idx, count, meta, meta2, pid, nverts, steps,
                     codes, ids);
  return 0;
}

// Per-code particle counts (stats), wave-aggregated atomics.
// Particles per termination code.  Reduced per wave (shuffles), then per
// workgroup (LDS), so one launch issues at most 6 atomics per workgroup: with
// one atomic per wave and code, ~50k same-address atomics serialised at the L2
// and took 0.2 ms for 1M particles, called once per exchange round.
__global__ void __launch_bounds__(256) k_count_codes(const int4* meta, long long n, unsigned long long* counts) {
  __shared__ unsigned long long part[6][4];
  unsigned c[6] = {0, 0, 0, 0, 0, 0};
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int z = meta[i].z;
    if (z >= 0 && z < 6) c[z]++;
  }
  const int wave = threadIdx.x >> 6;
  for (int k = 0; k < 6; ++k) {
    unsigned long long v = c[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (__lane_id() == 0) part[k][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const unsigned long long v = part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] + part[threadIdx.x][3];
    if (v) atomicAdd(&counts[threadIdx.x], v);
  }
}

// The outbox records of the last launch, from the per-XCD segments (behind the
// outbox proper, from index seg_base) to the end of the outbox, segment after
// segment.  Records of segment s: its counter, capped at seg_cap, or the mark
// of the reservation that did not fit (o + 1 in the counter's next word).
__device__ __forceinline__ unsigned long long seg_records(const unsigned long long* seg_ctr, int s,
                                                          unsigned long long cap) {
  const unsigned long long* c = seg_ctr + (size_t)s * QCTR_STRIDE;
  return c[1] ? c[1] - 1 : (c[0] < cap ? c[0] : cap);
}

__global__ void k_ob_concat(OutRec* outbox, int* outbox_src, long long seg_base, long long seg_cap,
                            const unsigned long long* seg_ctr, const unsigned long long* outbox_count) {
  unsigned long long off[OB_SEGS + 1];
  off[0] = 0;
#pragma unroll
  for (int s = 0; s < OB_SEGS; ++s) off[s + 1] = off[s] + seg_records(seg_ctr, s, (unsigned long long)seg_cap);
  const unsigned long long base = *outbox_count;
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < off[OB_SEGS];
       i += (unsigned long long)gridDim.x * blockDim.x) {
    int s = 0;
    while (i >= off[s + 1]) ++s;
    const size_t j = (size_t)seg_base + (size_t)s * (size_t)seg_cap + (size_t)(i - off[s]);
    outbox[base + i] = outbox[j];
    outbox_src[base + i] = outbox_src[j];
  }
}

// After k_ob_concat (a separate launch, so that no workgroup reads the old count late).
__global__ void k_ob_commit(const unsigned long long* seg_ctr, long long seg_cap, unsigned long long* outbox_count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int s = 0; s < OB_SEGS; ++s) t += seg_records(seg_ctr, s, (unsigned long long)seg_cap);
    *outbox_count += t;
  }
}

int launch_ob_concat(OutRec* outbox, int* outbox_src, long long seg_base, long long seg_cap,
                     const unsigned long long* seg_ctr, unsigned long long* outbox_count, hipStream_t st) {
  int grid = (int)std::min<long long>((OB_SEGS * seg_cap + 255) / 256, 1024);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_ob_concat, dim3(grid), dim3(256), 0, st, outbox, outbox_src, seg_base, seg_cap, seg_ctr,
                     outbox_count);
  hipLaunchKernelGGL(k_ob_commit, dim3(1), dim3(64), 0, st, seg_ctr, seg_cap, outbox_count);
  return 0;
}

int launch_count_codes(const int4* meta, long long n, unsigned long long* counts, hipStream_t st) {
  // about 16 particles per thread (4096 per workgroup), at most 256 workgroups
  int grid = (int)((n + 4095) / 4096);
  if (grid > 256) grid = 256;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_count_codes, dim3(grid), dim3(256), 0, st, meta, n, counts);
  return 0;
}

}  // namespace streami

namespace streami {

// ---------------------------------------------------------------- work order
// Active particles whose next step lies inside the time window are bucketed by
// (class of the steps they may still take, longest first; block; Morton index
// of a coarse brick of their position): particles that may run longest start
// first, so that the launch does not end waiting for a long trajectory started
// late, and lanes of a wave work on nearby cells.  The others (terminated, or
// waiting for a later window) get the last key and no slot in the order.
// The order only decides which lane advances which particle, never what is
// computed, so results do not depend on it.

__device__ __forceinline__ unsigned spread3(unsigned v) {  // 5 bits -> every third bit
  v &= 0x1f;
  v = (v | (v << 8)) & 0x0f00f;
  v = (v | (v << 4)) & 0xc30c3;
  v = (v | (v << 2)) & 0x249249;
  return v;
}

// n_classes classes of the remaining steps min(max_steps - steps, span) in [0, span]
__global__ void k_order_keys(const float4* pos, const int4* meta, const int4* meta2, const BlockDev* blocks,
                             long long n, int bits, unsigned n_buckets, int n_classes, int span, float h, float t_end,
                             unsigned* key, unsigned* hist) {
  const unsigned n_spatial = (n_buckets - 1) / (unsigned)n_classes;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    unsigned k = n_buckets - 1;
    const int4 mt = meta[i];
    const float4 p = pos[i];
    // work = active particles whose next step starts inside the time window
    if (mt.z == ACTIVE && fmaf((float)mt.x, h, p.w) < t_end) {
      const int blk = meta2[i].y;
      const BlockDev& B = blocks[blk];
      const float side = (float)(1 << bits);
      const float xs[3] = {p.x, p.y, p.z};
      unsigned c[3];
      for (int a = 0; a < 3; ++a) {
        const float s = fmaf(xs[a], B.scale[a], B.offs[a]) * (side / B.fn[a]);
        float w = floorf(s);
        if (B.periodic) w -= side * floorf(w / side);
        c[a] = (unsigned)__builtin_amdgcn_fmed3f(w, 0.0f, side - 1.0f);
      }
      const int rem = min(mt.y - mt.x, span);
      const int cls = min(n_classes - 1, (int)((long long)max(rem, 0) * n_classes / ((long long)span + 1)));
      k = (unsigned)(n_classes - 1 - cls) * n_spatial + (unsigned)blk * (1u << (3 * bits)) +
          (spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2));
    }
    key[i] = k;
    // idle particles (terminated, or outside the window) take no slot: only the
    // counted entries of the order are read, and one shared bucket would
    // serialise millions of atomics on one address
    if (k != n_buckets - 1) atomicAdd(&hist[k], 1u);
  }
}

// Exclusive scan of hist[0..nb) into cursor[] over SCAN_WG workgroups, each
// owning a contiguous range of the buckets: k_scan_part sums each range,
// k_scan_apply scans its range in tiles of SCAN_T from the sum of the ranges
// before it.  The class starts (each class's first bucket's prefix; the last
// entry, the idle bucket's prefix, is the number of particles counted) go to
// cls[]; k_scan_qtab then gives queue q the range [start + n q / Q,
// start + n (q+1) / Q) of each class of n particles (Q = MAX_QUEUES).
constexpr unsigned SCAN_WG = ORDER_SCAN_WG, SCAN_T = 256;

__device__ __forceinline__ unsigned block_sum(unsigned v, unsigned* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const unsigned w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  unsigned t = 0;
  for (unsigned i = 0; i < SCAN_T / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// exclusive prefix of v over the workgroup's threads; total = the workgroup's sum
__device__ __forceinline__ unsigned block_exclusive(unsigned v, unsigned* sh, unsigned& total) {
  const unsigned w = threadIdx.x >> 6, l = threadIdx.x & 63;
  unsigned incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned u = __shfl_up(incl, (unsigned)o, 64);
    if (l >= (unsigned)o) incl += u;
  }
  if (l == 63) sh[w] = incl;
  __syncthreads();
  unsigned off = 0;
  total = 0;
  for (unsigned i = 0; i < SCAN_T / 64; ++i) {
    if (i < w) off += sh[i];
    total += sh[i];
  }
  __syncthreads();
  return off + incl - v;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_part(const unsigned* hist, unsigned nb, unsigned* part) {
  __shared__ unsigned sh[SCAN_T / 64];
  const unsigned per = (nb + SCAN_WG - 1) / SCAN_WG;
  const unsigned b0 = blockIdx.x * per, b1 = min(nb, b0 + per);
  unsigned s = 0;
  for (unsigned b = b0 + threadIdx.x; b < b1; b += SCAN_T) s += hist[b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const unsigned* hist, unsigned nb, unsigned n_classes,
                                                       const unsigned* part, unsigned* cursor, unsigned* cls) {
  __shared__ unsigned sh[SCAN_T / 64];
  const unsigned per = (nb + SCAN_WG - 1) / SCAN_WG;
  const unsigned b0 = blockIdx.x * per, b1 = min(nb, b0 + per);
  const unsigned n_spatial = (nb - 1) / n_classes;
  unsigned o = 0;
  for (unsigned i = threadIdx.x; i < blockIdx.x; i += SCAN_T) o += part[i];
  unsigned run = block_sum(o, sh);  // the buckets before this range
  for (unsigned t0 = b0; t0 < b1; t0 += SCAN_T) {
    const unsigned b = t0 + threadIdx.x;
    const unsigned h = b < b1 ? hist[b] : 0u;
    unsigned tot;
    const unsigned ex = run + block_exclusive(h, sh, tot);
    if (b < b1) {
      cursor[b] = ex;
      if (b == nb - 1) cls[n_classes] = ex;
      else if (b % n_spatial == 0) cls[b / n_spatial] = ex;
    }
    run += tot;
  }
}

__global__ void k_scan_qtab(const unsigned* cls, unsigned n_classes, unsigned* qtab) {
  const unsigned t = threadIdx.x;
  if (t >= (unsigned)MAX_QUEUES) return;
  unsigned* row = qtab + t * QTAB_STRIDE;
  unsigned total = 0;
  for (unsigned c = 0; c < n_classes; ++c) {
    const unsigned long long n = cls[c + 1] - cls[c];
    const unsigned lo = cls[c] + (unsigned)(n * t / MAX_QUEUES), hi = cls[c] + (unsigned)(n * (t + 1) / MAX_QUEUES);
    row[1 + 2 * c] = lo;
    row[2 + 2 * c] = hi - lo;
    total += hi - lo;
  }
  row[0] = total;
}

__global__ void k_order_scatter(const unsigned* key, long long n, unsigned idle, unsigned* cursor, int* order) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const unsigned k = key[i];
    if (k == idle) continue;
    const unsigned slot = atomicAdd(&cursor[k], 1u);
    order[slot] = (int)i;
  }
}

int launch_work_order(const float4* pos, const int4* meta, const int4* meta2, const BlockDev* blocks, long long n,
                      int bits, unsigned n_buckets, int n_classes, int span, float h, float t_end, unsigned* key,
                      unsigned* hist, unsigned* cursor, int* order, unsigned* qtab, hipStream_t st) {
  if (n <= 0) return 0;
  long long grid = (n + 255) / 256;
  if (grid > 16384) grid = 16384;
  launch_fill_u32(hist, n_buckets, 0u, st);
  hipLaunchKernelGGL(k_order_keys, dim3((unsigned)grid), dim3(256), 0, st, pos, meta, meta2, blocks, n, bits,
                     n_buckets, n_classes, span, h, t_end, key, hist);
  // qtab's buffer also holds the class starts and the range sums after the table
  unsigned* cls = qtab + MAX_QUEUES * QTAB_STRIDE;
  unsigned* part = cls + ORDER_CLASSES + 1;
  hipLaunchKernelGGL(k_scan_part, dim3(SCAN_WG), dim3(SCAN_T), 0, st, hist, n_buckets, part);
  hipLaunchKernelGGL(k_scan_apply, dim3(SCAN_WG), dim3(SCAN_T), 0, st, hist, n_buckets, (unsigned)n_classes, part,
                     cursor, cls);
  hipLaunchKernelGGL(k_scan_qtab, dim3(1), dim3(64), 0, st, cls, (unsigned)n_classes, qtab);
  hipLaunchKernelGGL(k_order_scatter, dim3((unsigned)grid), dim3(256), 0, st, key, n, n_buckets - 1, cursor, order);
  return 0;
}

}  // namespace streami
