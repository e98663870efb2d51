// Memory-level probe behind streami_probe_gather (include/streami_probe.h):
// random record gathers over a buffer of a chosen footprint, to measure the
// gather rate each level of the memory hierarchy sustains (L2 for a few
// hundred KB, the Infinity Cache for ~200 MB, HBM beyond).  It is measurement
// support for the advection kernel's gather roofline, not part of the method.
#include <hip/hip_runtime.h>

#include "../../include/streami.h"
#include "../../include/streami_probe.h"

namespace streami {
int set_error(int code, const char* msg);
}

namespace {

// 32-bit integer mix (xorshift-multiply, "lowbias32" constants by C. Wellons):
// a counter-based stream of record indices, cheap next to a memory access.
__device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Each lane reads `per_lane` records of R16 x 16 bytes at record-aligned
// offsets r * R16 * 16, r uniform in [0, n_recs) (n_recs < 2^32), and writes
// the XOR of everything it read to sink[lane] so no load can be dropped.
// U records are in flight per lane at a time (per_lane is a multiple of U).
template <int R16, int U>
__global__ void __launch_bounds__(256) k_probe_gather(const uint4* __restrict__ buf, unsigned n_recs, int per_lane,
                                                      unsigned seed, unsigned* __restrict__ sink) {
  const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned acc = 0;
  const unsigned ctr = mix32(tid ^ seed);
  for (int i = 0; i < per_lane; i += U) {
    uint4 v[U][R16];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned r = __umulhi(mix32(ctr + (unsigned)(i + u) * 0x9e3779b9u), n_recs);
      const uint4* q = buf + (size_t)r * R16;
#pragma unroll
      for (int k = 0; k < R16; ++k) v[u][k] = q[k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < R16; ++k) acc ^= v[u][k].x ^ v[u][k].y ^ v[u][k].z ^ v[u][k].w;
  }
  sink[tid] = acc;
}

// VALU issue rate: 8 independent chains per lane of one instruction kind
// (0: v_fma_f32, a VOP3 encoding; 1: v_add_u32, VOP2; 2: v_exp_f32 of a
// negated operand; 3: v_rcp_f32), 16 x 8 per iteration.  The float chains
// start in [0.5, 0.51] and stay finite (2^-x maps [0.5, 1] into itself, 1/x
// alternates between two values).
template <int KIND>
__global__ void __launch_bounds__(256) k_probe_valu(unsigned* __restrict__ sink, int iters) {
  unsigned x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c)
    x[c] = KIND >= 2 ? __float_as_uint(0.5f + 0.001f * (float)c + 0.00001f * (float)(threadIdx.x & 63))
                     : threadIdx.x * 2654435761u + (unsigned)c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (KIND == 0) x[c] = __float_as_uint(fmaf(__uint_as_float(x[c]), 0.999f, 0.5f));
        else if (KIND == 1) x[c] = x[c] + x[(c + 1) & 7];
        else if (KIND == 2) x[c] = __float_as_uint(__builtin_amdgcn_exp2f(-__uint_as_float(x[c])));
        else x[c] = __float_as_uint(__builtin_amdgcn_rcpf(__uint_as_float(x[c])));
      }
  }
  unsigned acc = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) acc ^= x[c];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

int perr(int code, const char* msg) { return streami::set_error(code, msg); }

template <int R16>
void launch_probe(int in_flight, unsigned grid, hipStream_t st, const uint4* b, unsigned nr, int per_lane,
                  unsigned seed, unsigned* sink) {
  if (in_flight == 1)
    hipLaunchKernelGGL((k_probe_gather<R16, 1>), dim3(grid), dim3(256), 0, st, b, nr, per_lane, seed, sink);
  else if (in_flight == 2)
    hipLaunchKernelGGL((k_probe_gather<R16, 2>), dim3(grid), dim3(256), 0, st, b, nr, per_lane, seed, sink);
  else if (in_flight == 4)
    hipLaunchKernelGGL((k_probe_gather<R16, 4>), dim3(grid), dim3(256), 0, st, b, nr, per_lane, seed, sink);
  else
    hipLaunchKernelGGL((k_probe_gather<R16, 8>), dim3(grid), dim3(256), 0, st, b, nr, per_lane, seed, sink);
}

}  // namespace

extern "C" int streami_probe_gather(const void* buf, int64_t bytes, int32_t record_bytes, int32_t loads_per_lane,
                                    int32_t in_flight, int32_t waves_per_cu, void* hip_stream, float* ms,
                                    int64_t* records_read) {
  if (!buf || !ms) return perr(STREAMI_E_ARG, "buf and ms must not be NULL");
  if (record_bytes != 16 && record_bytes != 96 && record_bytes != 128)
    return perr(STREAMI_E_ARG, "record_bytes must be 16, 96 or 128");
  if (in_flight != 1 && in_flight != 2 && in_flight != 4 && in_flight != 8)
    return perr(STREAMI_E_ARG, "in_flight must be 1, 2, 4 or 8");
  if (loads_per_lane < in_flight || loads_per_lane % in_flight != 0 || loads_per_lane > (1 << 20))
    return perr(STREAMI_E_ARG, "loads_per_lane must be a multiple of in_flight in [in_flight, 2^20]");
  if (waves_per_cu < 1 || waves_per_cu > 64) return perr(STREAMI_E_ARG, "waves_per_cu must be in [1, 64]");
  const long long n_recs = bytes / record_bytes;
  if (bytes < 0 || n_recs < 1 || n_recs >= (1LL << 32))
    return perr(STREAMI_E_ARG, "bytes must hold 1 to 2^32-1 records");
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return perr(STREAMI_E_DEVICE, "no HIP device");
  const unsigned grid = (unsigned)n_cu * (unsigned)waves_per_cu / 4;
  const size_t lanes = (size_t)grid * 256;
  unsigned* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc(&sink, lanes * sizeof(unsigned)) != hipSuccess) {
    (void)hipGetLastError();
    return perr(STREAMI_E_NOMEM, "probe sink allocation failed");
  }
  int rc = STREAMI_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = perr(STREAMI_E_DEVICE, "event creation failed");
  } else {
    const uint4* b = reinterpret_cast<const uint4*>(buf);
    const unsigned nr = (unsigned)n_recs;
    // one untimed launch (caches and TLB warm), then the timed one
    for (int rep = 0; rep < 2 && rc == STREAMI_OK; ++rep) {
      if (rep == 1) (void)hipEventRecord(e0, st);
      const unsigned seed = 0x5eed0000u + (unsigned)rep;
      if (record_bytes == 16)
        launch_probe<1>(in_flight, grid, st, b, nr, loads_per_lane, seed, sink);
      else if (record_bytes == 96)
        launch_probe<6>(in_flight, grid, st, b, nr, loads_per_lane, seed, sink);
      else
        launch_probe<8>(in_flight, grid, st, b, nr, loads_per_lane, seed, sink);
      if (hipGetLastError() != hipSuccess) rc = perr(STREAMI_E_DEVICE, "probe launch failed");
      if (rep == 1) (void)hipEventRecord(e1, st);
    }
    if (rc == STREAMI_OK) {
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess)
        rc = perr(STREAMI_E_DEVICE, "probe timing failed");
      else if (records_read)
        *records_read = (int64_t)lanes * loads_per_lane;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(sink);
  return rc;
}

extern "C" int streami_probe_valu(int32_t kind, int32_t waves_per_cu, void* hip_stream, float* ms,
                                  int64_t* instructions) {
  if (!ms) return perr(STREAMI_E_ARG, "ms must not be NULL");
  if (kind < 0 || kind > 3)
    return perr(STREAMI_E_ARG, "kind must be 0 (v_fma_f32), 1 (v_add_u32), 2 (v_exp_f32) or 3 (v_rcp_f32)");
  if (waves_per_cu < 4 || waves_per_cu > 64 || waves_per_cu % 4 != 0)
    return perr(STREAMI_E_ARG, "waves_per_cu must be a multiple of 4 in [4, 64]");
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return perr(STREAMI_E_DEVICE, "no HIP device");
  const unsigned grid = (unsigned)n_cu * (unsigned)waves_per_cu / 4;
  const int iters = 1024;
  unsigned* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc(&sink, (size_t)grid * 256 * sizeof(unsigned)) != hipSuccess) {
    (void)hipGetLastError();
    return perr(STREAMI_E_NOMEM, "probe sink allocation failed");
  }
  int rc = STREAMI_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = perr(STREAMI_E_DEVICE, "event creation failed");
  } else {
    for (int rep = 0; rep < 2 && rc == STREAMI_OK; ++rep) {
      if (rep == 1) (void)hipEventRecord(e0, st);
      if (kind == 0)
        hipLaunchKernelGGL(k_probe_valu<0>, dim3(grid), dim3(256), 0, st, sink, iters);
      else if (kind == 1)
        hipLaunchKernelGGL(k_probe_valu<1>, dim3(grid), dim3(256), 0, st, sink, iters);
      else if (kind == 2)
        hipLaunchKernelGGL(k_probe_valu<2>, dim3(grid), dim3(256), 0, st, sink, iters);
      else
        hipLaunchKernelGGL(k_probe_valu<3>, dim3(grid), dim3(256), 0, st, sink, iters);
      if (hipGetLastError() != hipSuccess) rc = perr(STREAMI_E_DEVICE, "probe launch failed");
      if (rep == 1) (void)hipEventRecord(e1, st);
    }
    if (rc == STREAMI_OK) {
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess)
        rc = perr(STREAMI_E_DEVICE, "probe timing failed");
      else if (instructions)
        *instructions = (int64_t)grid * 4 * iters * 16 * 8;  // wave-level instructions of the chains
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(sink);
  return rc;
}
