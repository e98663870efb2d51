// Device-side data structures shared by the library's kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace streami {

enum Fmt { FMT_F32 = 0, FMT_F16 = 1, FMT_BF16 = 2 };
// LINEAR: x-fastest node rows.  BRICK4 / BRICK8: 4x4x4- / 8x8x8-node bricks
// (nodes x-fastest inside a brick, bricks x-fastest).  CELL (FP32 only):
// one 96-byte record per cell holding its trilinear interpolant's monomial
// coefficients, so a cell-cache miss is six aligned 16-byte loads and no
// arithmetic (8x the node bytes; `base` and `slice_nodes` then count 12-byte
// units, 8 per cell).
// HEX (FP32 only): an unstructured hexahedral field (BVH + cell records, hex.h).
enum Layout { LAYOUT_LINEAR = 1, LAYOUT_BRICK4 = 2, LAYOUT_CELL = 3, LAYOUT_HEX = 4, LAYOUT_BRICK8 = 5 };
// log2 of a brick layout's edge (0: not a brick layout)
__host__ __device__ constexpr int brick_shift(int layout) {
  return layout == LAYOUT_BRICK4 ? 2 : layout == LAYOUT_BRICK8 ? 3 : 0;
}
enum Code { ACTIVE = 0, MAX_STEPS = 1, EXIT = 2, STAGNANT = 3, HALO_MISS = 4, NONFINITE = 5 };

// One block as the kernels see it.  Storage coordinate along an axis:
// s = x*scale + offs  (= (x - origin)/spacing + ghost).
struct alignas(16) BlockDev {
  float scale[3];
  float offs[3];
  int nst[3];        // stored nodes per axis (periodic: interior nodes)
  int periodic;
  float lo[3];
  float hi[3];
  float inv_ext[3];  // 1/(hi - lo) for destinationID
  int rgrid[3];
  int rcoord[3];
  int n_slices;
  float t0;
  float inv_sdt;     // 1/slice_dt
  int nb[3];         // bricks per axis (brick layout)
  int pad0;
  long long base;    // node index of slice 0 of this block in the node pool
  long long slice_nodes;  // pool units per slice (nodes; CELL: 8 per cell)
  // byte-offset geometry used by the advection kernel (all < 2^32)
  unsigned ys, zs;       // linear: bytes per y row / z plane; brick4: per brick row / plane; cell: per cell row / plane
  unsigned slice_bytes;  // bytes per time slice
  unsigned pad1;
  float fn[3];           // stored nodes per axis as float
  float inv_fn[3];       // 1/fn (periodic wrap)
  // interior test: a step's stage points lie within |h| vs[a] storage units of
  // its start along axis a (the interpolant is a convex combination of node
  // values), up to sl[a] units of rounding; vs = max |v_a| over the stored
  // nodes x scale x (1 + 2^-10), NaN or Inf when a node is not finite
  float vs[3];
  float sl[3];
};

// Outbox record, 32 bytes (same layout as streami_outbox_rec).
struct alignas(8) OutRec {
  unsigned long long id;
  float pos[3];
  int steps;
  int dest;
  short code;
  short block;
};
static_assert(sizeof(OutRec) == 32, "outbox record must be 32 bytes");

// Per-call counters (zeroed by a fill kernel before each advect launch).
enum Counter {
  CTR_QUEUE = 0, CTR_STEPS = 1, CTR_VERTS = 2, CTR_ACCEPT = 3, CTR_FALLBACK = 4, CTR_OVERFLOW = 5,
  CTR_GATHERS = 6, CTR_N = 8
};

// Persistent counters (survive across advect calls; reset by streami_clear).
enum Persist { PER_OUTBOX = 0, PER_LOG = 1, PER_LOG_REAL = 2, PER_N = 4 };

// Vertex log: a wave appends the vertices its lanes produce in one step as a
// contiguous run (ballot + mbcnt) inside a chunk it reserved with one atomic,
// so every store is part of a full, coalesced line.  A record is one 16-byte
// store (x, y, z, particle index).  A particle's records enter the log in step
// order (a particle stays in its lane for a launch, a wave's chunks come from a
// monotonic counter, and later launches append after earlier ones), so fetching
// sorts the requested particles' records stably by row to get their lines.
// Records per wave reservation.  Every wave reserves from one counter, so the
// chunk is large: at 1024 records the contended atomic cost a third of a pass.
// A launch sizes its chunks to the records a wave is expected to write (at most
// LOG_CHUNK): short launches (a step budget of a few steps) would otherwise
// abandon most of every chunk.
constexpr int LOG_CHUNK = 8192;
constexpr int LOG_CHUNK_MIN = 64;
constexpr unsigned LOG_UNUSED = 0xffffffffu;  // particle index of an unused record

struct VertexLog {
  float4* v;                       // x, y, z, particle index (as bits)
  unsigned long long* count;       // records reserved (incl. unused chunk tails)
  unsigned long long* real;        // records written
  long long cap;                   // records the buffers hold
};

struct AdvectArgs {
  const BlockDev* blocks;   // [n_blocks]
  int n_blocks;
  const void* nodes;        // node pool (format and layout fixed per handle)
  float4* pos;              // x, y, z, t_birth
  int4* meta;               // steps, max_steps, code, n_verts
  const int4* meta2;        // stride, block, vcap, 0
  const unsigned long long* ids;
  VertexLog log;
  OutRec* outbox;
  int* outbox_src;                   // particle index of each outbox record (for forwarding)
  unsigned long long* outbox_count;  // persistent across calls
  unsigned long long* ctr;           // per-call counters
  long long n_particles;
  // work order: particles are claimed in the order of `order` (NULL: index
  // order, one queue), which holds n_classes classes of remaining work, longest
  // first.  Each class is split into MAX_QUEUES contiguous ranges, one per queue
  // and XCD (workgroups are dispatched to the XCDs round-robin); queue q runs
  // its range of every class in turn, so each XCD starts with long work on a
  // compact part of the field.  qtab holds, per queue, the total count and then
  // (start, length) of its range in each class (QTAB_STRIDE unsigned per queue).
  // A wave that empties its queue steals from the next.
  const int* order;
  const unsigned* qtab;
  int n_classes;
  unsigned long long* qctr;  // n_queues counters, QCTR_STRIDE apart
  int n_queues;
  float h;
  float eps2;               // stagnation_eps^2
  int budget;               // 0 = unlimited
  int refill;               // free lanes that trigger a refill
  float t_end;              // with `windowed`, a step starts only at t < t_end
  int windowed;             // 0: no time window (the time is then only the sampler's)
  int checked;              // 1: test every sample's domain even deep inside the block
  unsigned log_chunk;       // records per log reservation of a wave (LOG_CHUNK_MIN .. LOG_CHUNK)
  // per-XCD outbox segments (ob_seg_cap > 0): segment s holds ob_seg_cap records from index
  // ob_seg_base + s * ob_seg_cap of outbox/outbox_src (behind the outbox proper); its counter is
  // qctr[(MAX_QUEUES + s) * QCTR_STRIDE], and the next word marks where a full segment's records
  // end (o + 1).  A reservation that does not fit goes straight to the outbox.  The segments are
  // appended to the outbox after the launch.  0: every record straight to the outbox.
  long long ob_seg_base;
  long long ob_seg_cap;
};

// One surrogate jump (16 plain steps) for every active particle of a single
// steady block.  dhat = network displacement at x; for the commutation
// residual (kind 0) xh = one plain step from x and dhat2 = network at xh.
struct SurrogateArgs {
  AdvectArgs a;
  const float* dhat;    // [n x 3]
  const float* dhat2;   // [n x 3] (kind 0)
  float* xh;            // [n x 3] (kind 0; written by the pre-pass)
  float tol;            // residual tolerance in world units
  int kind;             // 0 commutation, 1 one big RK4 step
  int jump;             // steps per jump (16)
};

// Trilinear interpolant in monomial form: corners c[i] (i = x + 2y + 4z) are
// turned in place into the coefficients of 1, x, y, xy, z, xz, yz, xyz
// (three FP32 difference stages, always in this order, so the cell layout's
// stored coefficients equal those computed from gathered corners bit for bit).
// The coefficients of a constant field are exactly 0 beyond the first.
__device__ __forceinline__ void to_monomial(float3 c[8]) {
#pragma unroll
  for (int b = 1; b < 8; b <<= 1)
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i & b) {
        c[i].x -= c[i ^ b].x;
        c[i].y -= c[i ^ b].y;
        c[i].z -= c[i ^ b].z;
      }
}

constexpr int QCTR_STRIDE = 16;  // one 128-byte line per queue counter
constexpr int OB_SEGS = 8;       // outbox segments, one per XCD (workgroup index mod 8)
constexpr int MAX_QUEUES = 8;
constexpr int ORDER_CLASSES = 8;  // classes of remaining steps in the spatial work order
constexpr int QTAB_STRIDE = 1 + 2 * ORDER_CLASSES;
constexpr int ORDER_SCAN_WG = 256;  // workgroups of the work order's bucket scan

// Per-axis offsets of node i within a slice of a block.
template <int LAYOUT>
__device__ __forceinline__ int ax_off(const BlockDev& B, int i) {
  constexpr int S = brick_shift(LAYOUT), M = (1 << S) - 1;
  if (S) return ((i >> S) << (3 * S)) + (i & M);
  return i;
}
template <int LAYOUT>
__device__ __forceinline__ int ay_off(const BlockDev& B, int j) {
  constexpr int S = brick_shift(LAYOUT), M = (1 << S) - 1;
  if (S) return (j >> S) * (B.nb[0] << (3 * S)) + ((j & M) << S);
  return j * B.nst[0];
}
template <int LAYOUT>
__device__ __forceinline__ int az_off(const BlockDev& B, int k) {
  constexpr int S = brick_shift(LAYOUT), M = (1 << S) - 1;
  if (S) return (k >> S) * ((B.nb[0] * B.nb[1]) << (3 * S)) + ((k & M) << (2 * S));
  return k * (B.nst[0] * B.nst[1]);
}

}  // namespace streami
