// Line assembly at fetch (Sec. 3.2, getLines()): the vertex log holds one
// 16-byte record (x, y, z, particle index) per recorded vertex, and a
// particle's records enter the log in step order (its seed vertex at seeding,
// then each wave appends its lanes' vertices in order into chunks taken from a
// monotonic counter; later launches, jumps and forwarded segments append after
// earlier ones).  So the records of the requested particles, kept in log order
// and sorted stably by their output row, are the CSR lines: selection and a
// stable radix sort on the device, then a gather.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "device.h"

namespace streami {

namespace {

// flag[r] = 1 for the records of requested particles (row_of[p] >= 0)
__global__ void k_flag_records(const float4* v, long long n_rec, long long n_particles, const int* row_of,
                               unsigned char* flag) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n_rec; r += (long long)gridDim.x * blockDim.x) {
    const unsigned p = __float_as_uint(v[r].w);
    flag[r] = ((long long)p < n_particles && row_of[p] >= 0) ? 1 : 0;
  }
}

// key[i] = output row of selected record sel[i]
template <class I>
__global__ void k_row_keys(const float4* v, const I* sel, long long m, const int* row_of, unsigned* key) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x)
    key[i] = (unsigned)row_of[__float_as_uint(v[sel[i]].w)];
}

// out[i] = x, y, z of record rec[i]
template <class I>
__global__ void k_gather_xyz(const float4* v, const I* rec, long long m, float* out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x) {
    const float4 q = v[rec[i]];
    out[3 * i + 0] = q.x;
    out[3 * i + 1] = q.y;
    out[3 * i + 2] = q.z;
  }
}

unsigned grid_of(long long n) {
  long long g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

int bits_for(long long rows) {
  int b = 1;
  while (b < 32 && (1LL << b) <= rows) ++b;
  return b;
}

template <class I>
int assemble(const VertexLog& log, long long n_rec, long long n_particles, const int* row_of, long long rows,
             long long n_vertices, float* out, hipStream_t st, void* (*alloc)(size_t, void*), void (*release)(void*, void*),
             void* ctx) {
  // scratch: flags, the selected record indices (two buffers for the sort), keys (two), count, sort temp
  unsigned char* flag = (unsigned char*)alloc((size_t)n_rec, ctx);
  I* sel = (I*)alloc(sizeof(I) * (size_t)n_vertices, ctx);
  I* sel2 = (I*)alloc(sizeof(I) * (size_t)n_vertices, ctx);
  unsigned* key = (unsigned*)alloc(4 * (size_t)n_vertices, ctx);
  unsigned* key2 = (unsigned*)alloc(4 * (size_t)n_vertices, ctx);
  long long* d_count = (long long*)alloc(sizeof(long long), ctx);
  int rc = 0;
  void* tmp = nullptr;
  if (!flag || !sel || !sel2 || !key || !key2 || !d_count) {
    rc = 2;
  } else {
    hipLaunchKernelGGL(k_flag_records, dim3(grid_of(n_rec)), dim3(256), 0, st, log.v, n_rec, n_particles, row_of, flag);
    hipcub::CountingInputIterator<I> idx((I)0);
    size_t b1 = 0, b2 = 0;
    hipcub::DoubleBuffer<unsigned> kb(key, key2);
    hipcub::DoubleBuffer<I> vb(sel, sel2);
    if (hipcub::DeviceSelect::Flagged(nullptr, b1, idx, flag, sel, d_count, n_rec, st) != hipSuccess ||
        hipcub::DeviceRadixSort::SortPairs(nullptr, b2, kb, vb, n_vertices, 0, bits_for(rows), st) != hipSuccess)
      rc = 3;
    if (!rc) {
      tmp = alloc(std::max(b1, b2), ctx);
      if (!tmp) rc = 2;
    }
    long long got = -1;
    if (!rc && (hipcub::DeviceSelect::Flagged(tmp, b1, idx, flag, sel, d_count, n_rec, st) != hipSuccess ||
                hipMemcpyAsync(&got, d_count, sizeof got, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess))
      rc = 3;
    if (!rc && got != n_vertices) rc = 4;  // the log and the particles' vertex counts disagree
    if (!rc) {
      hipLaunchKernelGGL(k_row_keys<I>, dim3(grid_of(n_vertices)), dim3(256), 0, st, log.v, sel, n_vertices, row_of, key);
      b2 = std::max(b1, b2);
      if (hipcub::DeviceRadixSort::SortPairs(tmp, b2, kb, vb, n_vertices, 0, bits_for(rows), st) != hipSuccess) rc = 3;
    }
    if (!rc) {
      hipLaunchKernelGGL(k_gather_xyz<I>, dim3(grid_of(n_vertices)), dim3(256), 0, st, log.v, vb.Current(), n_vertices,
                         out);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) rc = 3;
    }
  }
  for (void* q : {(void*)flag, (void*)sel, (void*)sel2, (void*)key, (void*)key2, (void*)d_count, tmp})
    if (q) release(q, ctx);
  return rc;
}

}  // namespace

// The CSR lines of the requested rows (row_of[p] = row of particle p or -1;
// n_vertices = the rows' total) written to out (device, n_vertices x 3).
// Scratch comes from alloc/release.  Returns 0, 2 (no memory), 3 (a device
// call failed) or 4 (the log's records of the requested particles do not
// number n_vertices).
int assemble_lines(const VertexLog& log, long long n_rec, long long n_particles, const int* row_of, long long rows,
                   long long n_vertices, float* out, hipStream_t st, void* (*alloc)(size_t, void*),
                   void (*release)(void*, void*), void* ctx) {
  if (n_vertices <= 0) return 0;
  if (n_rec < (1LL << 32))
    return assemble<unsigned>(log, n_rec, n_particles, row_of, rows, n_vertices, out, st, alloc, release, ctx);
  return assemble<unsigned long long>(log, n_rec, n_particles, row_of, rows, n_vertices, out, st, alloc, release, ctx);
}

}  // namespace streami
