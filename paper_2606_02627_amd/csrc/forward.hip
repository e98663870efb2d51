// Loopback forwarding between the blocks of one handle: the single-GPU form of
// the paper's exchange of outgoing particles (rafi_forwardParticles in the
// step() listing of Sec. 3.2, emitOutgoing in Sec. 3.1.2).  An outbox record
// whose destination macrocell (destinationID, Sec. 3.1.1) is a block of the
// same handle becomes a new particle of that block: the same id, step count,
// step limit, birth time and record stride, starting at the record's
// position, which is vertex 0 of its new line segment.  Records for
// macrocells outside the handle stay in the outbox.
//
// An exchange looks only at the records appended since the last one (from
// `first` on): a record that stays is final, so the records before `first`
// are not read again.  k_fwd_count counts the new records per destination
// block and the vertex records their segments may still write; the host then
// places each block's new particles in one contiguous range after the
// existing ones, k_fwd_write initialises them and compacts the new records
// that stay into a scratch buffer, and k_fwd_settle copies those back behind
// the settled ones.  Counting goes through LDS histograms, so a workgroup
// issues one global atomic per destination block.
#include <hip/hip_runtime.h>

#include "forward.h"

namespace streami {

constexpr int FWD_THREADS = 256;

// Destination block of record r, or -1 when it stays in the outbox.  A halo
// miss is not sent back to the block it came from (its owner could not take
// the step either).
__device__ __forceinline__ int fwd_target(const FwdArgs& a, const OutRec& rec) {
  if (rec.code != EXIT && rec.code != HALO_MISS) return -1;
  if (rec.dest < 0 || rec.dest >= a.n_ranks) return -1;
  const int b = a.rank_map[rec.dest];
  if (b < 0 || (rec.code == HALO_MISS && b == rec.block)) return -1;
  return b;
}

// counts[b] += records going to block b; counts[n_blocks] += vertex records
// their segments may write (remaining steps / stride + 2 each).
__global__ void __launch_bounds__(FWD_THREADS) k_fwd_count(FwdArgs a, unsigned long long* counts) {
  __shared__ unsigned hist[FWD_MAX_BLOCKS];
  for (int i = threadIdx.x; i < a.n_blocks; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const long long n = (long long)*a.outbox_count;
  unsigned long long bound = 0;
  for (long long r = a.first + blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x) {
    const OutRec rec = a.outbox[r];
    const int b = fwd_target(a, rec);
    if (b < 0) continue;
    const int src = a.outbox_src[r];
    const int m = a.meta[src].y, stride = a.meta2[src].x;
    atomicAdd(&hist[b], 1u);
    bound += (unsigned long long)((m - rec.steps) / stride + 2);
  }
  for (int o = 32; o > 0; o >>= 1) bound += __shfl_xor(bound, o, 64);
  if (__lane_id() == 0 && bound) atomicAdd(&counts[a.n_blocks], bound);
  __syncthreads();
  for (int i = threadIdx.x; i < a.n_blocks; i += blockDim.x)
    if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
}

__global__ void __launch_bounds__(FWD_THREADS) k_fwd_write(FwdArgs a, FwdOut o) {
  __shared__ unsigned hist[FWD_MAX_BLOCKS];
  __shared__ unsigned long long wg_base[FWD_MAX_BLOCKS];
  const long long n = (long long)*a.outbox_count;
  const long long stride_all = (long long)gridDim.x * blockDim.x;
  // every workgroup walks its records in rounds of blockDim.x, so that the
  // LDS histogram of one round fits the slots it reserves
  for (long long r0 = a.first + blockIdx.x * (long long)blockDim.x; r0 < n; r0 += stride_all) {
    for (int i = threadIdx.x; i < a.n_blocks; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const long long r = r0 + threadIdx.x;
    OutRec rec;
    int b = -1, src = -1;
    unsigned local = 0;
    if (r < n) {
      rec = a.outbox[r];
      src = a.outbox_src[r];
      b = fwd_target(a, rec);
      if (b >= 0) local = atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.n_blocks; i += blockDim.x)
      wg_base[i] = hist[i] ? atomicAdd(&o.cursor[i], (unsigned long long)hist[i]) : 0ull;
    __syncthreads();
    const int lane = __lane_id();
    // new particles and vertex 0 of their segments (one log reservation per wave)
    const unsigned long long fm = __ballot(b >= 0);
    if (fm) {
      const int leader = __ffsll((long long)fm) - 1;
      unsigned long long lb = 0;
      if (lane == leader) {
        lb = atomicAdd(o.log.count, (unsigned long long)__popcll(fm));
        atomicAdd(o.log.real, (unsigned long long)__popcll(fm));
      }
      lb = __shfl(lb, leader, 64);
      if (b >= 0) {
        const long long q = o.base[b] + (long long)wg_base[b] + local;
        const int4 mt = a.meta[src];
        const int4 m2 = a.meta2[src];
        const float tb = a.pos[src].w;
        o.pos[q] = make_float4(rec.pos[0], rec.pos[1], rec.pos[2], tb);
        o.meta[q] = make_int4(rec.steps, mt.y, ACTIVE, 1);
        o.meta2[q] = make_int4(m2.x, b, (mt.y - rec.steps) / m2.x + 2, 0);
        o.ids[q] = rec.id;
        const unsigned long long lr = lb + __builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
        if (lr < (unsigned long long)o.log.cap) {
          o.log.v[lr] = make_float4(rec.pos[0], rec.pos[1], rec.pos[2], __uint_as_float((unsigned)q));
        }
      }
    }
    // records that stay, compacted (order unspecified, like the outbox itself)
    const bool keep = r < n && b < 0;
    const unsigned long long km = __ballot(keep);
    if (km) {
      const int leader = __ffsll((long long)km) - 1;
      unsigned long long kb = 0;
      if (lane == leader) kb = atomicAdd(o.n_kept, (unsigned long long)__popcll(km));
      kb = __shfl(kb, leader, 64);
      if (keep) {
        const unsigned long long k =
            kb + __builtin_amdgcn_mbcnt_hi((unsigned)(km >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)km, 0u));
        o.kept[k] = rec;
        o.kept_src[k] = src;
      }
    }
    __syncthreads();  // hist and wg_base are reused by the next round
  }
}

// The new records that stay, from the scratch buffer back to the outbox at
// `first`, and the outbox count.
__global__ void k_fwd_settle(const OutRec* kept, const int* kept_src, const unsigned long long* n_kept, OutRec* outbox,
                             int* outbox_src, long long first, unsigned long long* outbox_count) {
  const long long k = (long long)*n_kept;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < k; i += (long long)gridDim.x * blockDim.x) {
    outbox[first + i] = kept[i];
    outbox_src[first + i] = kept_src[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *outbox_count = (unsigned long long)(first + k);
}

int launch_fwd_count(const FwdArgs& a, unsigned long long* counts, long long max_records, hipStream_t st) {
  if (a.n_blocks > FWD_MAX_BLOCKS) return -1;
  long long g = (max_records + FWD_THREADS - 1) / FWD_THREADS;
  g = g < 1 ? 1 : (g > 2048 ? 2048 : g);
  hipLaunchKernelGGL(k_fwd_count, dim3((unsigned)g), dim3(FWD_THREADS), 0, st, a, counts);
  return 0;
}

int launch_fwd_write(const FwdArgs& a, const FwdOut& o, long long max_records, hipStream_t st) {
  if (a.n_blocks > FWD_MAX_BLOCKS) return -1;
  long long g = (max_records + FWD_THREADS - 1) / FWD_THREADS;
  g = g < 1 ? 1 : (g > 2048 ? 2048 : g);
  hipLaunchKernelGGL(k_fwd_write, dim3((unsigned)g), dim3(FWD_THREADS), 0, st, a, o);
  return 0;
}

int launch_fwd_settle(const OutRec* kept, const int* kept_src, const unsigned long long* n_kept, OutRec* outbox,
                      int* outbox_src, long long first, unsigned long long* outbox_count, long long max_records,
                      hipStream_t st) {
  long long g = (max_records + FWD_THREADS - 1) / FWD_THREADS;
  g = g < 1 ? 1 : (g > 1024 ? 1024 : g);
  hipLaunchKernelGGL(k_fwd_settle, dim3((unsigned)g), dim3(FWD_THREADS), 0, st, kept, kept_src, n_kept, outbox,
                     outbox_src, first, outbox_count);
  return 0;
}

}  // namespace streami
