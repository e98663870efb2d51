// Argument blocks of the loopback forwarding kernels (forward.hip), shared
// with the host side.
#pragma once
#include "device.h"

namespace streami {

constexpr int FWD_MAX_BLOCKS = 1024;  // LDS histogram size (a handle holds fewer blocks)

struct FwdArgs {
  const OutRec* outbox;
  const int* outbox_src;
  const unsigned long long* outbox_count;
  long long first;  // records before it stayed in an earlier exchange and are not looked at again
  const int* rank_map;  // macrocell id -> block of this handle, or -1
  int n_ranks;
  int n_blocks;
  const float4* pos;
  const int4* meta;
  const int4* meta2;
};

struct FwdOut {
  const long long* base;     // first new particle slot per block
  unsigned long long* cursor;  // per block, zeroed: slots taken so far
  float4* pos;
  int4* meta;
  int4* meta2;
  unsigned long long* ids;
  VertexLog log;
  OutRec* kept;                 // records that stay
  int* kept_src;
  unsigned long long* n_kept;   // zeroed
};

int launch_fwd_count(const FwdArgs& a, unsigned long long* counts, long long max_records, hipStream_t st);
int launch_fwd_write(const FwdArgs& a, const FwdOut& o, long long max_records, hipStream_t st);
int launch_fwd_settle(const OutRec* kept, const int* kept_src, const unsigned long long* n_kept, OutRec* outbox,
                      int* outbox_src, long long first, unsigned long long* outbox_count, long long max_records,
                      hipStream_t st);

}  // namespace streami
