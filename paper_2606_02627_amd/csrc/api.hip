// Host side of the C-ABI declared in include/streami.h: argument validation,
// handle state, device buffer management, kernel launches, fetches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/streami.h"
#include "device.h"
#include "seed.h"
#include "forward.h"

namespace streami {
int launch_advect_f32(const AdvectArgs& a, int layout, bool periodic, int mode, bool batched, int grid,
                      hipStream_t st);
int launch_advect_f16(const AdvectArgs& a, int layout, bool periodic, int mode, bool batched, int grid,
                      hipStream_t st);
int launch_advect_bf16(const AdvectArgs& a, int layout, bool periodic, int mode, bool batched, int grid,
                       hipStream_t st);
int launch_surrogate_f32(const SurrogateArgs& s, int layout, bool periodic, bool pre, int grid, hipStream_t st);
int launch_surrogate_f16(const SurrogateArgs& s, int layout, bool periodic, bool pre, int grid, hipStream_t st);
int launch_surrogate_bf16(const SurrogateArgs& s, int layout, bool periodic, bool pre, int grid, hipStream_t st);
int mlp_forward_rows(streami_mlp m, const float* xyz, int xstride, long long n, float* out, hipStream_t st);
int launch_ingest(const void* src, void* pool, const BlockDev& B, int fmt, int layout, int nx, int ny, int nz,
                  int n_slices, hipStream_t st);
int launch_seed(const SeedJobs& J, unsigned n_wg, const BlockDev* blocks, float4* pos, int4* meta, int4* meta2,
                unsigned long long* pid, const VertexLog& log, OutRec* outbox, int* outbox_src,
                unsigned long long* outbox_count, hipStream_t st);
int assemble_lines(const VertexLog& log, long long n_rec, long long n_particles, const int* row_of, long long rows,
                   long long n_vertices, float* out, hipStream_t st, void* (*alloc)(size_t, void*),
                   void (*release)(void*, void*), void* ctx);
int launch_mark_rows(const long long* idx, long long count, int* row_of, hipStream_t st);
int launch_fill_u32(unsigned* p, long long n, unsigned v, hipStream_t st);
int launch_max_abs(const void* src, int fmt, long long n, unsigned* out, hipStream_t st);
int launch_work_order(const float4* pos, const int4* meta, const int4* meta2, const BlockDev* blocks, long long n,
                      int bits, unsigned n_buckets, int n_classes, int span, float h, float t_end, unsigned* key,
                      unsigned* hist, unsigned* cursor, int* order, unsigned* qtab, hipStream_t st);
int launch_fill_u64(unsigned long long* p, long long n, unsigned long long v, hipStream_t st);
int launch_seed_bound(const SeedJobs& J, long long total, unsigned long long* out, hipStream_t st);
std::string build_hex_blob(const float* V, long long nv, const float* val, const int* cells,
                           const unsigned char* types, long long nc, float tol, std::vector<float>& blob,
                           unsigned& n_nodes);
int launch_seed_shape(const double o[3], const double u[3], const double v[3], long long nu, long long nv, float* out,
                      hipStream_t st);
int launch_gather_meta(const long long* idx, long long count, const int4* meta, const int4* meta2,
                       const unsigned long long* pid, long long* nverts, int* steps, int* codes,
                       unsigned long long* ids, hipStream_t st);
int launch_count_codes(const int4* meta, long long n, unsigned long long* counts, hipStream_t st);
int launch_ob_concat(OutRec* outbox, int* outbox_src, long long seg_base, long long seg_cap,
                     const unsigned long long* seg_ctr, unsigned long long* outbox_count, hipStream_t st);
}  // namespace streami

using namespace streami;

// the batched kernel stages the block table in LDS: at most 64 KiB of it
constexpr int MAX_BLOCKS = 65536 / (int)sizeof(BlockDev);
static_assert(MAX_BLOCKS >= 256, "block table too large for LDS");

namespace {

thread_local std::string g_err;

}  // namespace

namespace streami {
int set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace streami

namespace {

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(STREAMI_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// A device buffer that grows by reallocation (contents preserved on `st`).
// A device allocation owned by one object: freed when the object goes away
// (hipFree waits for the device, so no launch still reads it), moved, never
// copied.  Temporaries of a call free themselves on every return path.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  int reserve(size_t need, size_t keep, hipStream_t st) {
    if (need <= bytes) return STREAMI_OK;
    if (!keep) release();  // nothing to preserve: never hold both buffers
    void* q = nullptr;
    if (hipMalloc(&q, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(STREAMI_E_NOMEM, "device allocation of %zu bytes failed", need);
    }
    if (p && keep) {
      HIP_TRY(hipMemcpyAsync(q, p, std::min(keep, bytes), hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipStreamSynchronize(st));
    }
    if (p) (void)hipFree(p);
    p = q;
    bytes = need;
    return STREAMI_OK;
  }
};

struct HostBlock {
  streami_block_desc desc;
  BlockDev dev;
  int nx, ny, nz;  // stored nodes per axis
  std::vector<std::pair<long long, long long>> ranges;  // (first particle, count) in seed order
  long long n_particles = 0;
};

}  // namespace

struct streami_field_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int fmt = 0, layout = LAYOUT_LINEAR;
  long long ob_settled = 0;  // outbox records before this one stayed in an exchange (not read again)
  bool unsteady = false;
  bool periodic = false;
  int n_cu = 256;
  std::vector<HostBlock> blocks;
  DevBuf d_blocks, d_nodes;
  // particles (SoA)
  long long n_particles = 0, cap_particles = 0;
  DevBuf d_pos, d_meta, d_meta2, d_ids, d_outbox;
  DevBuf d_obsrc;  // particle index of each outbox record
  // loopback forwarding: macrocell id -> block of this handle (-1: elsewhere);
  // n_ranks = 0 when the blocks do not share one rank grid with distinct cells
  std::vector<int> rank_map;
  int n_ranks = 0;
  DevBuf d_rankmap, d_fwd, d_outbox2, d_obsrc2;
  // vertex log (see VertexLog): capacity in records, and the sum over all
  // particles of the vertices each may still record at most
  DevBuf d_logv;
  long long log_cap = 0;
  long long vert_bound = 0;
  // host upper bound of the log records still needed (reserved + to come, with
  // the chunk-tail allowance); valid while no advect ran since it was set
  bool log_need_known = false;
  long long log_need_hi = 0;
  DevBuf d_seedred;                         // k_seed_bound output
  unsigned long long* h_seedred = nullptr;  // pinned copy of it
  DevBuf d_ctr;        // CTR_N per-call counters, PER_N persistent counters, 6 code counts
  DevBuf d_qctr;       // per-queue work counters, then the per-XCD outbox segment counters
  DevBuf d_key, d_order, d_hist, d_cursor, d_nwork;  // spatial work order
  DevBuf d_dhat, d_dhat2, d_xh;                      // surrogate jumps
  bool strides_mult16 = true;                        // every seed batch's record stride % 16 == 0
  int max_m = 0;                                     // largest per-particle step limit seeded
  int min_m = INT_MAX;                               // smallest (equal to max_m: one class of work)
  long long active_hint = -1;  // particles known ACTIVE (after an exchange), -1: not known
  unsigned long long next_auto_id = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipGraphExec_t graph = nullptr;
  AdvectArgs graph_args;
  int graph_key[6] = {0, 0, 0, 0, 0, 0};

  unsigned long long* ctr() { return reinterpret_cast<unsigned long long*>(d_ctr.p); }
  unsigned long long* persist() { return ctr() + CTR_N; }
  unsigned long long* outbox_count() { return persist() + PER_OUTBOX; }
  unsigned long long* code_counts() { return persist() + PER_N; }
  VertexLog log() {
    VertexLog l;
    l.v = (float4*)d_logv.p;
    l.count = persist() + PER_LOG;
    l.real = persist() + PER_LOG_REAL;
    l.cap = log_cap;
    return l;
  }
};
constexpr int N_COUNTERS = CTR_N + PER_N + 6;

namespace {

int element_bytes(int fmt) { return fmt == STREAMI_F32 ? 12 : 6; }
int pool_node_bytes(int fmt) { return fmt == STREAMI_F32 ? 12 : 8; }

int validate_desc(const streami_block_desc& d, int i) {
  for (int a = 0; a < 3; ++a) {
    if (d.dims[a] < 1) return fail(STREAMI_E_ARG, "blocks[%d].dims[%d] must be >= 1", i, a);
    if (!(d.spacing[a] > 0) || !std::isfinite(d.spacing[a]))
      return fail(STREAMI_E_ARG, "blocks[%d].spacing[%d] must be finite and > 0", i, a);
    if (!std::isfinite(d.origin[a])) return fail(STREAMI_E_ARG, "blocks[%d].origin[%d] not finite", i, a);
    if (!(d.bounds_lo[a] < d.bounds_hi[a]) || !std::isfinite(d.bounds_lo[a]) || !std::isfinite(d.bounds_hi[a]))
      return fail(STREAMI_E_ARG, "blocks[%d].bounds_lo[%d] must be < bounds_hi[%d]", i, a, a);
    if (d.rank_grid[a] < 1) return fail(STREAMI_E_ARG, "blocks[%d].rank_grid[%d] must be >= 1", i, a);
    if (d.rank_coord[a] < 0 || d.rank_coord[a] >= d.rank_grid[a])
      return fail(STREAMI_E_ARG, "blocks[%d].rank_coord[%d] outside rank_grid", i, a);
  }
  if (d.boundary != STREAMI_BOUNDARY_BLOCK && d.boundary != STREAMI_BOUNDARY_PERIODIC)
    return fail(STREAMI_E_ARG, "blocks[%d].boundary invalid", i);
  if (d.ghost < 0 || d.ghost > 1) return fail(STREAMI_E_ARG, "blocks[%d].ghost must be 0 or 1", i);
  if (d.boundary == STREAMI_BOUNDARY_PERIODIC && d.ghost != 0)
    return fail(STREAMI_E_ARG, "blocks[%d]: a periodic block has no ghost layer", i);
  for (int a = 0; a < 3; ++a) {
    int ns = d.boundary == STREAMI_BOUNDARY_PERIODIC ? d.dims[a] : d.dims[a] + 2 * d.ghost;
    if (ns < 2) return fail(STREAMI_E_ARG, "blocks[%d]: axis %d needs >= 2 stored nodes", i, a);
  }
  if (d.n_slices < 1) return fail(STREAMI_E_ARG, "blocks[%d].n_slices must be >= 1", i);
  if (d.n_slices > 1 && !(d.slice_dt > 0)) return fail(STREAMI_E_ARG, "blocks[%d].slice_dt must be > 0", i);
  if (!d.nodes) return fail(STREAMI_E_ARG, "blocks[%d].nodes is NULL", i);
  long long nodes = (long long)(d.dims[0] + 2 * d.ghost) * (d.dims[1] + 2 * d.ghost) * (d.dims[2] + 2 * d.ghost);
  if (nodes >= (1LL << 31)) return fail(STREAMI_E_ARG, "blocks[%d]: more than 2^31 nodes per slice", i);
  return STREAMI_OK;
}

BlockDev make_dev(const streami_block_desc& d, int layout, int fmt, long long base) {
  BlockDev B;
  std::memset(&B, 0, sizeof B);
  const bool per = d.boundary == STREAMI_BOUNDARY_PERIODIC;
  long long slice = 1;
  for (int a = 0; a < 3; ++a) {
    B.nst[a] = per ? d.dims[a] : d.dims[a] + 2 * d.ghost;
    B.scale[a] = (float)(1.0 / d.spacing[a]);
    B.offs[a] = per ? 0.0f : (float)(d.ghost - d.origin[a] / d.spacing[a]);
    B.lo[a] = (float)d.bounds_lo[a];
    B.hi[a] = (float)d.bounds_hi[a];
    B.inv_ext[a] = (float)(1.0 / (d.bounds_hi[a] - d.bounds_lo[a]));
    B.rgrid[a] = d.rank_grid[a];
    B.rcoord[a] = d.rank_coord[a];
    const int be = 1 << brick_shift(layout);  // brick edge (1: no bricks)
    B.nb[a] = (B.nst[a] + be - 1) / be;
    slice *= brick_shift(layout) ? (long long)B.nb[a] * be : B.nst[a];
  }
  // cell layout: one record per cell (a periodic axis wraps, so it has as many
  // cells as nodes), counted as 8 pool units of 12 bytes
  long long cells[3];
  for (int a = 0; a < 3; ++a) cells[a] = per ? B.nst[a] : B.nst[a] - 1;
  if (layout == LAYOUT_CELL) slice = cells[0] * cells[1] * cells[2] * 8;
  // periodic blocks: origin shift folded into the position before sampling is
  // not needed when origin = 0; otherwise keep s = (x - origin)/spacing exact
  if (per)
    for (int a = 0; a < 3; ++a) B.offs[a] = (float)(-d.origin[a] / d.spacing[a]);
  B.periodic = per ? 1 : 0;
  B.n_slices = d.n_slices;
  B.t0 = (float)d.t0;
  B.inv_sdt = d.n_slices > 1 ? (float)(1.0 / d.slice_dt) : 0.0f;
  B.base = base;
  B.slice_nodes = slice;
  const long long nb = pool_node_bytes(fmt);
  long long ys, zs;
  if (brick_shift(layout)) {
    const long long brick = 1LL << (3 * brick_shift(layout));  // nodes per brick
    ys = (long long)B.nb[0] * brick * nb;
    zs = (long long)B.nb[0] * B.nb[1] * brick * nb;
  } else if (layout == LAYOUT_CELL) {
    ys = cells[0] * 96;
    zs = cells[0] * cells[1] * 96;
  } else {
    ys = (long long)B.nst[0] * nb;
    zs = (long long)B.nst[0] * B.nst[1] * nb;
  }
  B.ys = (unsigned)ys;
  B.zs = (unsigned)zs;
  B.slice_bytes = (unsigned)std::min<long long>(slice * nb, 0xffffffffLL);
  for (int a = 0; a < 3; ++a) {
    B.fn[a] = (float)B.nst[a];
    B.inv_fn[a] = (float)(1.0 / B.nst[a]);
  }
  return B;
}

// The kernels address a slice with 32-bit byte offsets and 24-bit row/plane
// multiplies: a slice must stay below 2 GiB and a z plane below 16 MiB.
bool check_geometry_quiet(const BlockDev& B) {
  return B.ys < (1u << 24) && B.zs < (1u << 24) && (long long)B.slice_bytes < (1LL << 31);
}
int check_geometry(const BlockDev& B, int i) {
  if (B.ys >= (1u << 24) || B.zs >= (1u << 24))
    return fail(STREAMI_E_UNSUPPORTED, "blocks[%d]: a z plane of nodes exceeds 16 MiB", i);
  if ((long long)B.slice_bytes >= (1LL << 31))
    return fail(STREAMI_E_UNSUPPORTED, "blocks[%d]: one time slice exceeds 2 GiB; split the block", i);
  return STREAMI_OK;
}

int ensure_particles(streami_field_s* f, long long need) {
  if (need <= f->cap_particles) return STREAMI_OK;
  long long cap = std::max(need, f->cap_particles + f->cap_particles / 2);
  cap = std::max(cap, 1024LL);
  const long long n = f->n_particles;
  int rc;
  if ((rc = f->d_pos.reserve(cap * sizeof(float4), n * sizeof(float4), f->stream))) return rc;
  if ((rc = f->d_meta.reserve(cap * sizeof(int4), n * sizeof(int4), f->stream))) return rc;
  if ((rc = f->d_meta2.reserve(cap * sizeof(int4), n * sizeof(int4), f->stream))) return rc;
  if ((rc = f->d_ids.reserve(cap * 8, n * 8, f->stream))) return rc;
  unsigned long long ob = 0;
  HIP_TRY(hipMemcpyAsync(&ob, f->outbox_count(), 8, hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(hipStreamSynchronize(f->stream));
  if ((rc = f->d_outbox.reserve(cap * sizeof(OutRec), ob * sizeof(OutRec), f->stream))) return rc;
  if ((rc = f->d_obsrc.reserve(cap * sizeof(int), ob * sizeof(int), f->stream))) return rc;
  f->cap_particles = cap;
  return STREAMI_OK;
}

// Make the vertex log hold every record still to come: the records reserved so
// far, the vertices particles may still record, and `slack` more (unused chunk
// tails of one launch).  Grows by reallocation, keeping the reserved records.
int ensure_log(streami_field_s* f, long long slack, long long chunk = LOG_CHUNK) {
  unsigned long long c[PER_N];
  HIP_TRY(hipMemcpyAsync(c, f->persist(), sizeof c, hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(hipStreamSynchronize(f->stream));
  const long long count = (long long)std::min<unsigned long long>(c[PER_LOG], (unsigned long long)f->log_cap);
  // a wave abandons < 64 records of a chunk when it switches chunks: reserve
  // the remaining bound plus 64/chunk of it (at least 1/8) for those tails,
  // plus `slack` for last chunks
  const long long remaining = std::max<long long>(f->vert_bound - (long long)c[PER_LOG_REAL], 0);
  const long long den = std::max<long long>(1, std::min<long long>(8, chunk / 64));
  const long long need = (long long)c[PER_LOG] + remaining + remaining / den + slack;
  f->log_need_known = true;
  f->log_need_hi = need - slack;
  if (need <= f->log_cap) return STREAMI_OK;
  const long long cap = std::max(need, f->log_cap + f->log_cap / 4);
  int rc;
  if ((rc = f->d_logv.reserve(cap * 16, count * 16, f->stream))) return rc;
  f->log_cap = cap;
  return STREAMI_OK;
}

void drop_graph(streami_field_s* f) {
  if (f->graph) (void)hipGraphExecDestroy(f->graph);
  f->graph = nullptr;
}


int collect_stats(streami_field_s* f, streami_stats* stats) {
  launch_fill_u64(f->code_counts(), 6, 0, f->stream);
  launch_count_codes((const int4*)f->d_meta.p, f->n_particles, f->code_counts(), f->stream);
  unsigned long long h[N_COUNTERS];
  HIP_TRY(hipMemcpyAsync(h, f->ctr(), sizeof h, hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(hipStreamSynchronize(f->stream));
  std::memset(stats, 0, sizeof *stats);
  stats->steps = (int64_t)h[CTR_STEPS];
  stats->vertices = (int64_t)h[CTR_VERTS];
  stats->surrogate_accepted = (int64_t)h[CTR_ACCEPT];
  stats->surrogate_fallback = (int64_t)h[CTR_FALLBACK];
  stats->outbox = (int64_t)h[CTR_N + PER_OUTBOX];
  for (int k = 0; k < 6; ++k) stats->terminated[k] = (int64_t)h[CTR_N + PER_N + k];
  stats->active = stats->terminated[0];
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, f->ev0, f->ev1));
  stats->device_ms = ms;
  stats->gathers = (int64_t)h[CTR_GATHERS];
  if (h[CTR_OVERFLOW]) return fail(STREAMI_E_DEVICE, "vertex log overflow (internal sizing error)");
  return STREAMI_OK;
}

// SURROGATE mode: repeated jumps of 16 steps; the network displacement is
// accepted where its residual is within tolerance, else plain RK4 is used.
int advect_surrogate(streami_field_s* f, const streami_advect_params* p, streami_stats* stats) {
  const int J = 16;
  if (!p->mlp) return fail(STREAMI_E_STATE, "surrogate mode needs a network (params.mlp)");
  if (f->blocks.size() != 1 || f->unsteady || f->layout == LAYOUT_HEX)
    return fail(STREAMI_E_UNSUPPORTED, "surrogate mode supports one steady structured block");
  if (!f->strides_mult16) return fail(STREAMI_E_ARG, "surrogate mode needs record strides that are multiples of 16");
  if (p->step_budget % J != 0) return fail(STREAMI_E_ARG, "surrogate step_budget must be a multiple of 16");
  if (p->residual_kind != 0 && p->residual_kind != 1) return fail(STREAMI_E_ARG, "residual_kind must be 0 or 1");
  if (!(p->residual_tol_cells >= 0)) return fail(STREAMI_E_ARG, "residual_tol_cells must be >= 0");
  const long long n = f->n_particles;
  int rc;
  if ((rc = f->d_dhat.reserve(n * 12, 0, f->stream)) || (rc = f->d_dhat2.reserve(n * 12, 0, f->stream)) ||
      (rc = f->d_xh.reserve(n * 12, 0, f->stream)))
    return rc;
  if ((rc = ensure_log(f, 0))) return rc;  // one record per particle per jump, exactly reserved
  const HostBlock& hb = f->blocks[0];
  const double cell = std::min(hb.desc.spacing[0], std::min(hb.desc.spacing[1], hb.desc.spacing[2]));
  SurrogateArgs s;
  std::memset(&s, 0, sizeof s);
  AdvectArgs& a = s.a;
  a.blocks = (const BlockDev*)f->d_blocks.p;
  a.n_blocks = 1;
  a.nodes = f->d_nodes.p;
  a.pos = (float4*)f->d_pos.p;
  a.meta = (int4*)f->d_meta.p;
  a.meta2 = (const int4*)f->d_meta2.p;
  a.ids = (const unsigned long long*)f->d_ids.p;
  a.log = f->log();
  a.outbox = (OutRec*)f->d_outbox.p;
  a.outbox_src = (int*)f->d_obsrc.p;
  a.outbox_count = f->outbox_count();
  a.ctr = f->ctr();
  a.n_particles = n;
  a.h = p->h;
  a.eps2 = p->stagnation_eps * p->stagnation_eps;
  a.t_end = INFINITY;
  s.dhat = (const float*)f->d_dhat.p;
  s.dhat2 = (const float*)f->d_dhat2.p;
  s.xh = (float*)f->d_xh.p;
  s.tol = (float)(p->residual_tol_cells * cell);
  s.kind = p->residual_kind;
  s.jump = J;
  long long jumps = (f->max_m + J - 1) / J + 1;
  if (p->step_budget > 0) jumps = std::min<long long>(jumps, p->step_budget / J);
  const int grid = (int)std::min<long long>((n + 255) / 256, 8192);
  auto launch = [&](bool pre) {
    if (f->fmt == STREAMI_F32) return launch_surrogate_f32(s, f->layout, f->periodic, pre, grid, f->stream);
    if (f->fmt == STREAMI_F16) return launch_surrogate_f16(s, f->layout, f->periodic, pre, grid, f->stream);
    return launch_surrogate_bf16(s, f->layout, f->periodic, pre, grid, f->stream);
  };
  HIP_TRY(hipEventRecord(f->ev0, f->stream));
  f->log_need_known = false;  // the launch appends records the host does not count
  launch_fill_u64(a.ctr, CTR_N, 0, f->stream);
  for (long long j = 0; j < jumps; ++j) {
    if (s.kind == 0) {
      launch(true);
      if ((rc = mlp_forward_rows(p->mlp, s.xh, 3, n, (float*)f->d_dhat2.p, f->stream))) return rc;
    }
    if ((rc = mlp_forward_rows(p->mlp, (const float*)f->d_pos.p, 4, n, (float*)f->d_dhat.p, f->stream))) return rc;
    launch(false);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipEventRecord(f->ev1, f->stream));
  if (stats) return collect_stats(f, stats);
  return STREAMI_OK;
}

}  // namespace

namespace streami {
int block_count(streami_field f) { return (int)f->blocks.size(); }
}  // namespace streami

namespace {
// Loopback forwarding needs every block on one rank grid, one block per cell:
// then the rank -> block map goes to the device; otherwise forwarding is off.
int setup_rank_map(streami_field_s* f) {
  const int n_blocks = (int)f->blocks.size();
  const int* g0 = f->blocks[0].desc.rank_grid;
  long long nr = (long long)g0[0] * g0[1] * g0[2];
  bool ok = nr <= (1LL << 24) && n_blocks <= FWD_MAX_BLOCKS;
  for (int i = 1; i < n_blocks && ok; ++i)
    for (int a = 0; a < 3; ++a) ok = ok && f->blocks[i].desc.rank_grid[a] == g0[a];
  if (ok) {
    f->rank_map.assign((size_t)nr, -1);
    for (int i = 0; i < n_blocks && ok; ++i) {
      const int* c = f->blocks[i].desc.rank_coord;
      const long long id = c[0] + (long long)g0[0] * (c[1] + (long long)g0[1] * c[2]);
      if (f->rank_map[id] >= 0) ok = false;
      else f->rank_map[id] = i;
    }
  }
  if (!ok) {
    f->rank_map.clear();
    return STREAMI_OK;
  }
  f->n_ranks = (int)nr;
  int rc;
  if ((rc = f->d_rankmap.reserve(sizeof(int) * nr, 0, f->stream))) return rc;
  if (hipMemcpyAsync(f->d_rankmap.p, f->rank_map.data(), sizeof(int) * nr, hipMemcpyHostToDevice, f->stream) !=
      hipSuccess)
    return fail(STREAMI_E_DEVICE, "rank map copy failed");
  return STREAMI_OK;
}

}  // namespace

extern "C" {

const char* streami_last_error(void) { return g_err.c_str(); }

int streami_field_create(const streami_block_desc* blocks, int32_t n_blocks, int32_t dtype,
                         const streami_field_opts* opts, void* hip_stream, streami_field* out) {
  if (!out) return fail(STREAMI_E_ARG, "out is NULL");
  if (!blocks || n_blocks < 1) return fail(STREAMI_E_ARG, "need at least one block");
  // the batched kernel stages the block table in LDS (at most 64 KiB of it)
  if (n_blocks > MAX_BLOCKS) return fail(STREAMI_E_UNSUPPORTED, "at most %d blocks per handle", MAX_BLOCKS);
  if (dtype != STREAMI_F32 && dtype != STREAMI_F16 && dtype != STREAMI_BF16)
    return fail(STREAMI_E_ARG, "dtype must be STREAMI_F32, STREAMI_F16 or STREAMI_BF16");
  int layout = opts ? opts->layout : STREAMI_LAYOUT_AUTO;
  if (layout != STREAMI_LAYOUT_AUTO && layout != STREAMI_LAYOUT_LINEAR && layout != STREAMI_LAYOUT_BRICK4 &&
      layout != STREAMI_LAYOUT_CELL && layout != STREAMI_LAYOUT_BRICK8)
    return fail(STREAMI_E_ARG, "unknown layout %d", layout);
  if (layout == STREAMI_LAYOUT_CELL && dtype != STREAMI_F32)
    return fail(STREAMI_E_UNSUPPORTED, "the cell layout stores FP32 coefficients: dtype must be STREAMI_F32");
  for (int i = 0; i < n_blocks; ++i) {
    int rc = validate_desc(blocks[i], i);
    if (rc) return rc;
  }
  if (layout == STREAMI_LAYOUT_AUTO) {
    // steady FP32 blocks whose cell records fit the kernels' 32-bit addressing
    // take the cell layout (fewer instructions per cell-cache miss, 8x the
    // bytes); everything else x-fastest rows
    bool cell = dtype == STREAMI_F32;
    for (int i = 0; i < n_blocks && cell; ++i)
      cell = blocks[i].n_slices == 1 && check_geometry_quiet(make_dev(blocks[i], LAYOUT_CELL, dtype, 0));
    layout = cell ? STREAMI_LAYOUT_CELL : STREAMI_LAYOUT_LINEAR;
  }
  for (int i = 0; i < n_blocks; ++i) {
    int rc;
    // the addressing limits depend only on the shapes: refuse before any device work
    if ((rc = check_geometry(make_dev(blocks[i], layout, dtype, 0), i))) return rc;
  }
  streami_field_s* f = new (std::nothrow) streami_field_s();
  if (!f) return fail(STREAMI_E_NOMEM, "host allocation failed");
  f->fmt = dtype;
  f->layout = layout;
  f->stream = (hipStream_t)hip_stream;
  auto cleanup = [&](int rc) {
    streami_field_destroy(f);
    return rc;
  };
  if (hipGetDevice(&f->device) != hipSuccess) return cleanup(fail(STREAMI_E_DEVICE, "no HIP device"));
  (void)hipDeviceGetAttribute(&f->n_cu, hipDeviceAttributeMultiprocessorCount, f->device);
  long long base = 0;
  f->blocks.resize(n_blocks);
  for (int i = 0; i < n_blocks; ++i) {
    HostBlock& hb = f->blocks[i];
    hb.desc = blocks[i];
    hb.dev = make_dev(blocks[i], layout, dtype, base);
    hb.nx = hb.dev.nst[0];
    hb.ny = hb.dev.nst[1];
    hb.nz = hb.dev.nst[2];
    base += hb.dev.slice_nodes * blocks[i].n_slices;
    if (blocks[i].n_slices > 1) f->unsteady = true;
    if (blocks[i].boundary == STREAMI_BOUNDARY_PERIODIC) f->periodic = true;
  }
  if (f->periodic && (n_blocks > 1 || f->unsteady))
    return cleanup(fail(STREAMI_E_UNSUPPORTED, "periodic boundaries are supported for one steady block"));
  int rc;
  if ((rc = f->d_nodes.reserve((size_t)base * pool_node_bytes(dtype), 0, f->stream))) return cleanup(rc);
  if (brick_shift(layout) || dtype != STREAMI_F32)  // padding stays zero
    if (hipMemsetAsync(f->d_nodes.p, 0, f->d_nodes.bytes, f->stream) != hipSuccess)
      return cleanup(fail(STREAMI_E_DEVICE, "hipMemsetAsync failed"));
  std::vector<BlockDev> devs(n_blocks);
  DevBuf staging, vmax;
  if ((rc = vmax.reserve(sizeof(unsigned) * 3 * n_blocks, 0, f->stream))) return cleanup(rc);
  launch_fill_u32((unsigned*)vmax.p, 3LL * n_blocks, 0u, f->stream);
  for (int i = 0; i < n_blocks; ++i) {
    HostBlock& hb = f->blocks[i];
    devs[i] = hb.dev;
    const size_t bytes = (size_t)hb.nx * hb.ny * hb.nz * hb.desc.n_slices * element_bytes(dtype);
    const void* src = hb.desc.nodes;
    if (!hb.desc.nodes_on_device) {
      if ((rc = staging.reserve(bytes, 0, f->stream))) return cleanup(rc);
      if (hipMemcpyAsync(staging.p, hb.desc.nodes, bytes, hipMemcpyHostToDevice, f->stream) != hipSuccess)
        return cleanup(fail(STREAMI_E_DEVICE, "copy of blocks[%d].nodes to the device failed", i));
      src = staging.p;
    }
    launch_ingest(src, f->d_nodes.p, hb.dev, dtype, layout, hb.nx, hb.ny, hb.nz, hb.desc.n_slices, f->stream);
    launch_max_abs(src, dtype, (long long)hb.nx * hb.ny * hb.nz * hb.desc.n_slices, (unsigned*)vmax.p + 3 * i,
                   f->stream);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(STREAMI_E_DEVICE, "ingest launch failed"));
    if (!hb.desc.nodes_on_device && hipStreamSynchronize(f->stream) != hipSuccess)
      return cleanup(fail(STREAMI_E_DEVICE, "ingest failed"));
    hb.desc.nodes = nullptr;  // the caller keeps ownership; never read again
  }
  // interior-test bounds per block: the largest |v_a| over the stored nodes
  // bounds every interpolated value (a convex combination), with 2^-10
  // relative slack for the FP32 interpolation; the rounding slack covers a
  // few ulps of the largest world coordinate and of the storage coordinate
  {
    std::vector<unsigned> mx(3 * (size_t)n_blocks);
    if (hipMemcpyAsync(mx.data(), vmax.p, mx.size() * sizeof(unsigned), hipMemcpyDeviceToHost, f->stream) !=
            hipSuccess ||
        hipStreamSynchronize(f->stream) != hipSuccess)
      return cleanup(fail(STREAMI_E_DEVICE, "field maximum readback failed"));
    for (int i = 0; i < n_blocks; ++i) {
      const streami_block_desc& d = blocks[i];
      const int g = d.boundary == STREAMI_BOUNDARY_PERIODIC ? 0 : d.ghost;
      for (int a = 0; a < 3; ++a) {
        float m;
        std::memcpy(&m, &mx[3 * i + a], 4);
        const double sc = 1.0 / d.spacing[a];
        const double w = std::max(std::fabs(d.origin[a] - g * d.spacing[a]),
                                  std::fabs(d.origin[a] + (devs[i].nst[a] - 1 - g) * d.spacing[a]));
        devs[i].vs[a] = (float)((double)m * sc * (1.0 + 0x1p-10));
        devs[i].sl[a] = (float)(w * 0x1p-22 * sc + devs[i].nst[a] * 0x1p-20 + 0x1p-6);
        f->blocks[i].dev.vs[a] = devs[i].vs[a];
        f->blocks[i].dev.sl[a] = devs[i].sl[a];
      }
    }
  }
  if ((rc = f->d_blocks.reserve(sizeof(BlockDev) * n_blocks, 0, f->stream))) return cleanup(rc);
  if (hipMemcpyAsync(f->d_blocks.p, devs.data(), sizeof(BlockDev) * n_blocks, hipMemcpyHostToDevice, f->stream) !=
      hipSuccess)
    return cleanup(fail(STREAMI_E_DEVICE, "block table copy failed"));
  if ((rc = f->d_ctr.reserve(sizeof(unsigned long long) * N_COUNTERS, 0, f->stream))) return cleanup(rc);
  launch_fill_u64(f->ctr(), N_COUNTERS, 0, f->stream);
  if ((rc = setup_rank_map(f))) return cleanup(rc);
  if (hipEventCreate(&f->ev0) != hipSuccess || hipEventCreate(&f->ev1) != hipSuccess)
    return cleanup(fail(STREAMI_E_DEVICE, "event creation failed"));
  if (hipStreamSynchronize(f->stream) != hipSuccess) return cleanup(fail(STREAMI_E_DEVICE, "field upload failed"));
  staging.release();
  *out = f;
  return STREAMI_OK;
}

int streami_field_create_hex(const streami_hex_desc* d, void* hip_stream, streami_field* out) {
  if (!out) return fail(STREAMI_E_ARG, "out is NULL");
  if (!d) return fail(STREAMI_E_ARG, "desc is NULL");
  if (d->n_vertices < 1 || d->n_vertices >= (1LL << 31)) return fail(STREAMI_E_ARG, "n_vertices must be in [1, 2^31)");
  if (d->n_cells < 1 || d->n_cells >= (1LL << 28)) return fail(STREAMI_E_ARG, "n_cells must be in [1, 2^28)");
  if (!d->vertices || !d->values || !d->cells) return fail(STREAMI_E_ARG, "vertices, values and cells must not be NULL");
  for (int a = 0; a < 3; ++a) {
    if (!(std::isfinite(d->bounds_lo[a]) && std::isfinite(d->bounds_hi[a]) && d->bounds_lo[a] < d->bounds_hi[a]))
      return fail(STREAMI_E_ARG, "bounds must be finite with lo < hi");
    if (d->rank_grid[a] < 1 || d->rank_coord[a] < 0 || d->rank_coord[a] >= d->rank_grid[a])
      return fail(STREAMI_E_ARG, "rank_grid must be >= 1 and rank_coord inside it");
  }
  // the builder reads host copies of the mesh
  const long long nv = d->n_vertices, nc = d->n_cells;
  std::vector<float> hv, hval;
  std::vector<int> hc;
  std::vector<unsigned char> ht;
  const float *V = d->vertices, *val = d->values;
  const int* C = d->cells;
  const unsigned char* T = d->cell_types;
  try {
    if (d->inputs_on_device) {
      hv.resize(3 * (size_t)nv);
      hval.resize(3 * (size_t)nv);
      hc.resize(8 * (size_t)nc);
      if (hipMemcpy(hv.data(), d->vertices, hv.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hval.data(), d->values, hval.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hc.data(), d->cells, hc.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(STREAMI_E_DEVICE, "copy of the mesh to the host failed");
      if (T) {
        ht.resize((size_t)nc);
        if (hipMemcpy(ht.data(), d->cell_types, ht.size(), hipMemcpyDeviceToHost) != hipSuccess)
          return fail(STREAMI_E_DEVICE, "copy of the cell types to the host failed");
        T = ht.data();
      }
      V = hv.data();
      val = hval.data();
      C = hc.data();
    }
    std::vector<float> blob;
    unsigned n_nodes = 0;
    const std::string err = build_hex_blob(V, nv, val, C, T, nc, 1e-4f, blob, n_nodes);
    if (!err.empty()) return fail(STREAMI_E_ARG, "%s", err.c_str());
    streami_field_s* f = new (std::nothrow) streami_field_s();
    if (!f) return fail(STREAMI_E_NOMEM, "host allocation failed");
    auto cleanup = [&](int rc) {
      streami_field_destroy(f);
      return rc;
    };
    f->fmt = STREAMI_F32;
    f->layout = LAYOUT_HEX;
    f->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&f->device) != hipSuccess) return cleanup(fail(STREAMI_E_DEVICE, "no HIP device"));
    (void)hipDeviceGetAttribute(&f->n_cu, hipDeviceAttributeMultiprocessorCount, f->device);
    // one block: its owned bounds and rank grid; the storage-coordinate fields map the
    // bounds onto a 64^3 grid, used only to order the work spatially
    f->blocks.resize(1);
    HostBlock& hb = f->blocks[0];
    std::memset(&hb.desc, 0, sizeof hb.desc);
    BlockDev& B = hb.dev;
    std::memset(&B, 0, sizeof B);
    for (int a = 0; a < 3; ++a) {
      const double lo = d->bounds_lo[a], hi = d->bounds_hi[a];
      hb.desc.dims[a] = 64;
      hb.desc.origin[a] = lo;
      hb.desc.spacing[a] = (hi - lo) / 64.0;
      hb.desc.bounds_lo[a] = lo;
      hb.desc.bounds_hi[a] = hi;
      hb.desc.rank_grid[a] = d->rank_grid[a];
      hb.desc.rank_coord[a] = d->rank_coord[a];
      B.scale[a] = (float)(64.0 / (hi - lo));
      B.offs[a] = (float)(-lo * 64.0 / (hi - lo));
      B.nst[a] = 64;
      B.fn[a] = 64.0f;
      B.inv_fn[a] = 1.0f / 64.0f;
      B.lo[a] = (float)lo;
      B.hi[a] = (float)hi;
      B.inv_ext[a] = (float)(1.0 / (hi - lo));
      B.rgrid[a] = d->rank_grid[a];
      B.rcoord[a] = d->rank_coord[a];
      B.nb[a] = 16;
      B.vs[a] = NAN;  // no interior shortcut
    }
    hb.desc.boundary = STREAMI_BOUNDARY_BLOCK;
    hb.desc.n_slices = 1;
    hb.desc.slice_dt = 1.0;
    B.n_slices = 1;
    hb.nx = hb.ny = hb.nz = 64;
    int rc;
    if ((rc = f->d_nodes.reserve(blob.size() * 4, 0, f->stream))) return cleanup(rc);
    if (hipMemcpyAsync(f->d_nodes.p, blob.data(), blob.size() * 4, hipMemcpyHostToDevice, f->stream) != hipSuccess)
      return cleanup(fail(STREAMI_E_DEVICE, "copy of the field to the device failed"));
    if ((rc = f->d_blocks.reserve(sizeof(BlockDev), 0, f->stream))) return cleanup(rc);
    if (hipMemcpyAsync(f->d_blocks.p, &B, sizeof(BlockDev), hipMemcpyHostToDevice, f->stream) != hipSuccess)
      return cleanup(fail(STREAMI_E_DEVICE, "block table copy failed"));
    if ((rc = f->d_ctr.reserve(sizeof(unsigned long long) * N_COUNTERS, 0, f->stream))) return cleanup(rc);
    launch_fill_u64(f->ctr(), N_COUNTERS, 0, f->stream);
    if ((rc = setup_rank_map(f))) return cleanup(rc);
    if (hipEventCreate(&f->ev0) != hipSuccess || hipEventCreate(&f->ev1) != hipSuccess)
      return cleanup(fail(STREAMI_E_DEVICE, "event creation failed"));
    // the host copies are read by the asynchronous upload: wait before they go
    if (hipStreamSynchronize(f->stream) != hipSuccess) return cleanup(fail(STREAMI_E_DEVICE, "field upload failed"));
    *out = f;
    return STREAMI_OK;
  } catch (const std::bad_alloc&) {
    return fail(STREAMI_E_NOMEM, "host allocation for the mesh failed");
  }
}

int streami_field_destroy(streami_field f) {
  if (!f) return STREAMI_OK;
  (void)hipStreamSynchronize(f->stream);
  drop_graph(f);
  for (DevBuf* b : {&f->d_blocks, &f->d_nodes, &f->d_pos, &f->d_meta, &f->d_meta2, &f->d_ids, &f->d_outbox,
                    &f->d_obsrc, &f->d_rankmap, &f->d_fwd, &f->d_outbox2, &f->d_obsrc2,
                    &f->d_logv, &f->d_ctr, &f->d_qctr, &f->d_key,
                    &f->d_order, &f->d_hist, &f->d_cursor, &f->d_nwork, &f->d_dhat, &f->d_dhat2, &f->d_xh,
                    &f->d_seedred})
    b->release();
  if (f->h_seedred) (void)hipHostFree(f->h_seedred);
  if (f->ev0) (void)hipEventDestroy(f->ev0);
  if (f->ev1) (void)hipEventDestroy(f->ev1);
  delete f;
  return STREAMI_OK;
}

}  // extern "C"

namespace {

// Seeding of one or several batches, as consecutive streami_seed() calls
// would do them, with one reduction and at most one wait for all batches.
int seed_batches(streami_field_s* f, const streami_seed_batch* bt, int nb, const streami_seed_opts* opts) {
  if (!opts) return fail(STREAMI_E_ARG, "opts is NULL");
  if (opts->record_stride < 1) return fail(STREAMI_E_ARG, "record_stride must be >= 1");
  const bool dev_in = opts->inputs_on_device != 0;
  long long total = 0;
  bool any_dev_ms = false;
  for (int k = 0; k < nb; ++k) {
    const streami_seed_batch& b = bt[k];
    if (b.block < 0 || b.block >= (int)f->blocks.size())
      return fail(STREAMI_E_ARG, "batch %d: block %d out of range", k, b.block);
    if (b.n < 0) return fail(STREAMI_E_ARG, "batch %d: n must be >= 0", k);
    if (b.n == 0) continue;
    if (!b.xyz) return fail(STREAMI_E_ARG, "batch %d: xyz is NULL", k);
    if (!b.max_steps && opts->default_max_steps < 0) return fail(STREAMI_E_ARG, "default_max_steps must be >= 0");
    total += b.n;
    any_dev_ms = any_dev_ms || (b.max_steps && dev_in);
  }
  if (total == 0) return STREAMI_OK;
  if (f->n_particles + total >= (1LL << 31)) return fail(STREAMI_E_ARG, "more than 2^31 particles per handle");
  // every particle may record at most max_steps/stride + 2 vertices: reserve
  // that in the log; limits on the device are reduced on the device, all
  // batches into one accumulator (32 bytes come back, one wait)
  long long bound = 0;
  int batch_max = 0, batch_min = INT_MAX;
  int rc;
  if (any_dev_ms) {
    if ((rc = f->d_seedred.reserve(32, 0, f->stream))) return rc;
    if (!f->h_seedred && hipHostMalloc((void**)&f->h_seedred, 32, hipHostMallocDefault) != hipSuccess) {
      f->h_seedred = nullptr;
      return fail(STREAMI_E_NOMEM, "pinned host allocation failed");
    }
    launch_fill_u64((unsigned long long*)f->d_seedred.p, 3, 0, f->stream);
    launch_fill_u64((unsigned long long*)f->d_seedred.p + 3, 1, ~0ull, f->stream);
    SeedJobs J;
    std::memset(&J, 0, sizeof J);
    J.stride = opts->record_stride;
    long long part = 0;
    for (int k = 0; k <= nb; ++k) {
      if (k < nb && bt[k].n > 0 && bt[k].max_steps) {
        J.j[J.n_jobs].max_steps = bt[k].max_steps;
        J.j[J.n_jobs].n = bt[k].n;
        ++J.n_jobs;
        part += bt[k].n;
      }
      if (J.n_jobs == SEED_JOBS || (k == nb && J.n_jobs > 0)) {
        launch_seed_bound(J, part, (unsigned long long*)f->d_seedred.p, f->stream);
        J.n_jobs = 0;
        part = 0;
      }
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(f->h_seedred, f->d_seedred.p, 32, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
    if (f->h_seedred[2]) return fail(STREAMI_E_ARG, "max_steps has a negative entry");
    bound = (long long)f->h_seedred[0];
    batch_max = (int)f->h_seedred[1];
    if (f->h_seedred[3] <= (unsigned long long)INT_MAX) batch_min = (int)f->h_seedred[3];
  }
  for (int k = 0; k < nb; ++k) {
    const streami_seed_batch& b = bt[k];
    if (b.n == 0 || (b.max_steps && dev_in)) continue;
    for (long long i = 0; i < b.n; ++i) {
      const int m = b.max_steps ? b.max_steps[i] : opts->default_max_steps;
      if (m < 0) return fail(STREAMI_E_ARG, "batch %d: max_steps[%lld] < 0", k, i);
      bound += m / opts->record_stride + 2;
      batch_max = std::max(batch_max, m);
      batch_min = std::min(batch_min, m);
    }
  }
  drop_graph(f);
  if ((rc = ensure_particles(f, f->n_particles + total))) return rc;
  // Seeding k particles inside a block adds k records and k real vertices
  // and raises vert_bound by `bound` >= k, so the need grows by at most
  // bound + bound/8 + 1: while the host bound covers that, no read-back.
  const long long grow = bound + bound / 8 + 1;
  f->vert_bound += bound;
  if (f->log_need_known && f->log_need_hi + grow <= f->log_cap) {
    f->log_need_hi += grow;
  } else if ((rc = ensure_log(f, 0))) {
    f->vert_bound -= bound;
    return rc;
  }
  // stage host inputs on the device (kept until the one wait below), then
  // seed up to SEED_JOBS batches per launch
  std::vector<DevBuf> stage(dev_in ? 0 : 4 * (size_t)nb);
  SeedJobs J;
  std::memset(&J, 0, sizeof J);
  J.default_max = opts->default_max_steps;
  J.stride = opts->record_stride;
  J.t_birth = opts->t_birth;
  unsigned n_wg = 0;
  for (int k = 0; k <= nb; ++k) {
    if (k < nb && bt[k].n > 0) {
      const streami_seed_batch& b = bt[k];
      SeedJob& jb = J.j[J.n_jobs];
      jb.xyz = b.xyz;
      jb.ids = reinterpret_cast<const unsigned long long*>(b.ids);
      jb.max_steps = b.max_steps;
      jb.t_births = b.t_births;
      if (!dev_in) {
        DevBuf* sb = &stage[4 * (size_t)k];
        if ((rc = sb[0].reserve(b.n * 12, 0, f->stream))) return rc;
        HIP_TRY(hipMemcpyAsync(sb[0].p, b.xyz, b.n * 12, hipMemcpyHostToDevice, f->stream));
        jb.xyz = (const float*)sb[0].p;
        if (b.ids) {
          if ((rc = sb[1].reserve(b.n * 8, 0, f->stream))) return rc;
          HIP_TRY(hipMemcpyAsync(sb[1].p, b.ids, b.n * 8, hipMemcpyHostToDevice, f->stream));
          jb.ids = (const unsigned long long*)sb[1].p;
        }
        if (b.max_steps) {
          if ((rc = sb[2].reserve(b.n * 4, 0, f->stream))) return rc;
          HIP_TRY(hipMemcpyAsync(sb[2].p, b.max_steps, b.n * 4, hipMemcpyHostToDevice, f->stream));
          jb.max_steps = (const int*)sb[2].p;
        }
        if (b.t_births) {
          if ((rc = sb[3].reserve(b.n * 4, 0, f->stream))) return rc;
          HIP_TRY(hipMemcpyAsync(sb[3].p, b.t_births, b.n * 4, hipMemcpyHostToDevice, f->stream));
          jb.t_births = (const float*)sb[3].p;
        }
      }
      jb.first = f->n_particles;
      jb.n = b.n;
      jb.auto_id0 = f->next_auto_id;
      jb.blk = b.block;
      jb.wg0 = n_wg;
      n_wg += (unsigned)((b.n + 1023) / 1024);
      ++J.n_jobs;
      HostBlock& hb = f->blocks[b.block];
      if (!b.ids) f->next_auto_id += (unsigned long long)b.n;
      f->n_particles += b.n;
      hb.ranges.push_back({jb.first, b.n});
      hb.n_particles += b.n;
    }
    if (J.n_jobs == SEED_JOBS || (k == nb && J.n_jobs > 0)) {
      launch_seed(J, n_wg, (const BlockDev*)f->d_blocks.p, (float4*)f->d_pos.p, (int4*)f->d_meta.p,
                  (int4*)f->d_meta2.p, (unsigned long long*)f->d_ids.p, f->log(), (OutRec*)f->d_outbox.p,
                  (int*)f->d_obsrc.p, f->outbox_count(), f->stream);
      HIP_TRY(hipGetLastError());
      J.n_jobs = 0;
      n_wg = 0;
    }
  }
  if (!dev_in) HIP_TRY(hipStreamSynchronize(f->stream));  // staging buffers are freed on return
  f->max_m = std::max(f->max_m, batch_max);
  f->min_m = std::min(f->min_m, batch_min);
  f->active_hint = -1;  // new particles: the active count is no longer known
  if (opts->record_stride % 16 != 0) f->strides_mult16 = false;
  return STREAMI_OK;
}

}  // namespace

extern "C" {

int streami_seed(streami_field f, int32_t block, const float* xyz, const uint64_t* ids, const int32_t* max_steps,
                 int64_t n, const streami_seed_opts* opts) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (n == 0 && block >= 0 && block < (int)f->blocks.size()) return STREAMI_OK;
  streami_seed_batch b;
  b.block = block;
  b.xyz = xyz;
  b.ids = ids;
  b.max_steps = max_steps;
  b.t_births = opts ? opts->t_births : nullptr;
  b.n = n;
  return seed_batches(f, &b, 1, opts);
}

int streami_seed_shape(streami_field f, int32_t block, const streami_shape* shape, const int32_t* max_steps,
                       const streami_seed_opts* opts) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (!shape || !opts) return fail(STREAMI_E_ARG, "shape and opts must not be NULL");
  if (block < 0 || block >= (int)f->blocks.size()) return fail(STREAMI_E_ARG, "block %d out of range", block);
  if (shape->kind != STREAMI_SHAPE_LINE && shape->kind != STREAMI_SHAPE_PLANE)
    return fail(STREAMI_E_ARG, "shape kind must be STREAMI_SHAPE_LINE or STREAMI_SHAPE_PLANE");
  const bool plane = shape->kind == STREAMI_SHAPE_PLANE;
  const long long nu = shape->nu, nv = plane ? shape->nv : 1;
  if (nu < 0 || nv < 1) return fail(STREAMI_E_ARG, "need nu >= 0 and nv >= 1");
  if (nu > 0 && nv > ((1LL << 31) - 1) / nu) return fail(STREAMI_E_ARG, "more than 2^31 seed points");
  double v[3] = {0, 0, 0};
  for (int c = 0; c < 3; ++c) {
    if (plane) v[c] = shape->v[c];
    if (!std::isfinite(shape->origin[c]) || !std::isfinite(shape->u[c]) || !std::isfinite(v[c]))
      return fail(STREAMI_E_ARG, "the shape must be finite");
  }
  const long long n = nu * nv;
  if (n == 0) return STREAMI_OK;
  // the points, and any host limits and birth times, staged on the device for the call
  DevBuf xyz, lim, tb;
  int rc;
  if ((rc = xyz.reserve(n * 12, 0, f->stream))) return rc;
  launch_seed_shape(shape->origin, shape->u, v, nu, nv, (float*)xyz.p, f->stream);
  HIP_TRY(hipGetLastError());
  const int32_t* d_lim = max_steps;
  const float* d_tb = opts->t_births;
  if (!opts->inputs_on_device) {
    if (max_steps) {
      if ((rc = lim.reserve(n * 4, 0, f->stream))) return rc;
      HIP_TRY(hipMemcpyAsync(lim.p, max_steps, n * 4, hipMemcpyHostToDevice, f->stream));
      d_lim = (const int32_t*)lim.p;
    }
    if (opts->t_births) {
      if ((rc = tb.reserve(n * 4, 0, f->stream))) return rc;
      HIP_TRY(hipMemcpyAsync(tb.p, opts->t_births, n * 4, hipMemcpyHostToDevice, f->stream));
      d_tb = (const float*)tb.p;
    }
  }
  streami_seed_opts o = *opts;
  o.inputs_on_device = 1;
  o.t_births = nullptr;
  streami_seed_batch b;
  b.block = block;
  b.xyz = (const float*)xyz.p;
  b.ids = nullptr;
  b.max_steps = d_lim;
  b.t_births = d_tb;
  b.n = n;
  rc = seed_batches(f, &b, 1, &o);
  (void)hipStreamSynchronize(f->stream);  // the staged arrays are freed on return
  return rc;
}

int streami_seed_batches(streami_field f, const streami_seed_batch* batches, int32_t n_batches,
                         const streami_seed_opts* opts) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (n_batches < 0 || (n_batches > 0 && !batches)) return fail(STREAMI_E_ARG, "batches is NULL or n_batches < 0");
  if (n_batches == 0) return STREAMI_OK;
  if (opts && opts->t_births) return fail(STREAMI_E_ARG, "opts->t_births: give birth times per batch");
  return seed_batches(f, batches, n_batches, opts);
}

int streami_advect(streami_field f, const streami_advect_params* p, streami_stats* stats) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (!p) return fail(STREAMI_E_ARG, "params is NULL");
  if (!(p->h > 0) || !std::isfinite(p->h)) return fail(STREAMI_E_ARG, "h must be finite and > 0");
  if (p->step_budget < 0) return fail(STREAMI_E_ARG, "step_budget must be >= 0");
  if (!(p->stagnation_eps >= 0)) return fail(STREAMI_E_ARG, "stagnation_eps must be >= 0");
  if (p->mode != STREAMI_MODE_PLAIN && p->mode != STREAMI_MODE_SURROGATE)
    return fail(STREAMI_E_ARG, "unknown mode %d", p->mode);
  if (p->waves_per_cu < 0 || p->waves_per_cu > 64) return fail(STREAMI_E_ARG, "waves_per_cu must be in [0,64]");
  if (p->refill_threshold < 0 || p->refill_threshold > 64)
    return fail(STREAMI_E_ARG, "refill_threshold must be in [0,64]");
  if (p->work_order != 0 && p->work_order != 1) return fail(STREAMI_E_ARG, "work_order must be 0 or 1");
  if (f->n_particles == 0) return fail(STREAMI_E_STATE, "no particles seeded");
  if (p->use_t_end != 0 && p->use_t_end != 1) return fail(STREAMI_E_ARG, "use_t_end must be 0 or 1");
  if (p->checked_samples != 0 && p->checked_samples != 1)
    return fail(STREAMI_E_ARG, "checked_samples must be 0 or 1");
  if (p->lds_cell_cache != 0 && p->lds_cell_cache != 1) return fail(STREAMI_E_ARG, "lds_cell_cache must be 0 or 1");
  if (p->use_t_end && std::isnan(p->t_end)) return fail(STREAMI_E_ARG, "t_end is NaN");
  if (p->mode == STREAMI_MODE_SURROGATE) {
    if (p->use_t_end) return fail(STREAMI_E_UNSUPPORTED, "surrogate mode takes no time window");
    return advect_surrogate(f, p, stats);
  }
  AdvectArgs a;
  std::memset(&a, 0, sizeof a);  // padding too: the graph cache compares the bytes
  a.blocks = (const BlockDev*)f->d_blocks.p;
  a.n_blocks = (int)f->blocks.size();
  a.nodes = f->d_nodes.p;
  a.pos = (float4*)f->d_pos.p;
  a.meta = (int4*)f->d_meta.p;
  a.meta2 = (const int4*)f->d_meta2.p;
  a.ids = (const unsigned long long*)f->d_ids.p;
  a.outbox = (OutRec*)f->d_outbox.p;
  a.outbox_src = (int*)f->d_obsrc.p;
  a.outbox_count = f->outbox_count();
  a.ctr = f->ctr();
  a.n_particles = f->n_particles;
  a.h = p->h;
  a.eps2 = p->stagnation_eps * p->stagnation_eps;
  a.budget = p->step_budget;
  // defaults measured on MI355X: refilling at the first free lane is 3-6%
  // faster than at 16; with node rows 16 waves/CU suit ~4 particles per lane
  // (1M seeds) and 32 suit larger sets (4M seeds: 16 waves/CU is 9% slower);
  // cell records (wider loads per miss) want 32 already at 1M seeds (5% faster)
  a.refill = p->refill_threshold > 0 ? p->refill_threshold : 1;
  a.windowed = p->use_t_end;
  a.checked = p->checked_samples;
  a.t_end = p->use_t_end ? p->t_end : INFINITY;
  const int wpc = p->waves_per_cu > 0 ? p->waves_per_cu
                                      : (f->layout != LAYOUT_CELL && f->n_particles <= (1LL << 21) ? 16 : 32);
  long long grid = (long long)f->n_cu * wpc / 4;
  grid = std::min(grid, (f->n_particles + 255) / 256);
  grid = std::max(grid, 1LL);
  {
    // chunk size: a quarter of the records a wave may write in this call (every active particle
    // steps at most the budget or its largest limit), as a power of two in [LOG_CHUNK_MIN,
    // LOG_CHUNK], so the tails abandoned at chunk switches and at the end stay near a quarter of
    // what is written even when calls are short (exchange rounds of a few steps)
    const long long steps_bound = p->step_budget > 0 ? std::min<long long>(p->step_budget, f->max_m) : f->max_m;
    const long long n_est = f->active_hint >= 0 ? std::min(f->active_hint, f->n_particles) : f->n_particles;
    const long long per_wave = (n_est * (steps_bound + 1) + grid * 4 - 1) / (grid * 4);
    long long chunk = LOG_CHUNK_MIN;
    while (4 * chunk < per_wave && chunk < LOG_CHUNK) chunk <<= 1;
    a.log_chunk = (unsigned)chunk;
    int rc = ensure_log(f, grid * 4 * chunk, chunk);
    if (rc) return rc;
  }
  a.log = f->log();
  // spatial work order (bucket sort by block and Morton brick) over per-XCD queues; not for
  // one-step calls (the paper's per-step exchange rounds): there the sort of every particle
  // record (~0.2 ms at 1.5M records) costs more than the order saves (with 8 steps per round it
  // still saves more than it costs); the order changes no result
  const bool spatial = p->work_order == 0 && p->step_budget != 1;
  // spatial work order: classes of remaining steps (longest first), then block and Morton brick
  const int bits = f->blocks.size() == 1 ? 5 : 3;
  // one class when every seeded limit is the same (the spatial order alone, fewer buckets), or
  // when the launch has many particles per lane: its end is then a small part of it, and the
  // classes would only cost the queues spatial locality
  const long long n_work_est = f->active_hint >= 0 ? std::min(f->active_hint, f->n_particles) : f->n_particles;
  const int n_classes = f->min_m < f->max_m && n_work_est <= 64 * grid * 256 ? ORDER_CLASSES : 1;
  const int span = (int)std::max<long long>(1, p->step_budget > 0 ? std::min<long long>(p->step_budget, f->max_m) : f->max_m);
  const unsigned n_buckets = (unsigned)n_classes * (unsigned)f->blocks.size() * (1u << (3 * bits)) + 1;
  {
    int rc;
    if ((rc = f->d_qctr.reserve(sizeof(unsigned long long) * 2 * MAX_QUEUES * QCTR_STRIDE, 0, f->stream))) return rc;
    // per-XCD outbox segments behind the outbox proper: n/8 + 64 records each (a launch ends
    // each particle at most once, and the waves of each XCD take an even share of the work);
    // a wave whose records do not fit its segment writes them straight to the outbox
    if (f->n_particles > 0) {
      const long long seg_cap = f->n_particles / OB_SEGS + 64;
      const size_t recs = (size_t)f->cap_particles + (size_t)OB_SEGS * (size_t)seg_cap;
      if ((rc = f->d_outbox.reserve(recs * sizeof(OutRec), (size_t)f->cap_particles * sizeof(OutRec), f->stream)) ||
          (rc = f->d_obsrc.reserve(recs * sizeof(int), (size_t)f->cap_particles * sizeof(int), f->stream)))
        return rc;
      a.outbox = (OutRec*)f->d_outbox.p;
      a.outbox_src = (int*)f->d_obsrc.p;
      a.ob_seg_base = f->cap_particles;
      a.ob_seg_cap = seg_cap;
    }
    if (spatial) {
      if ((rc = f->d_key.reserve(f->n_particles * 4, 0, f->stream)) ||
          (rc = f->d_order.reserve(f->n_particles * 4, 0, f->stream)) ||
          (rc = f->d_hist.reserve(n_buckets * 4, 0, f->stream)) ||
          (rc = f->d_cursor.reserve(n_buckets * 4, 0, f->stream)) || (rc = f->d_nwork.reserve(4 * (MAX_QUEUES * QTAB_STRIDE + ORDER_CLASSES + 1 + ORDER_SCAN_WG), 0, f->stream)))
        return rc;
    }
  }
  a.order = spatial ? (const int*)f->d_order.p : nullptr;
  a.qtab = spatial ? (const unsigned*)f->d_nwork.p : nullptr;
  a.n_classes = spatial ? n_classes : 1;
  a.qctr = (unsigned long long*)f->d_qctr.p;
  a.n_queues = spatial ? MAX_QUEUES : 1;
  const bool batched = f->blocks.size() > 1;
  int mode = f->unsteady ? (p->no_cell_cache ? 3 : 2) : (p->no_cell_cache ? 1 : 0);
  if (mode == 0 && p->lds_cell_cache && f->layout == LAYOUT_CELL && !batched) mode = 4;  // SM_LDS
  auto launch = [&](hipStream_t st) {
    if (f->fmt == STREAMI_F32) return launch_advect_f32(a, f->layout, f->periodic, mode, batched, (int)grid, st);
    if (f->fmt == STREAMI_F16) return launch_advect_f16(a, f->layout, f->periodic, mode, batched, (int)grid, st);
    return launch_advect_bf16(a, f->layout, f->periodic, mode, batched, (int)grid, st);
  };
  // the segments' records to the end of the outbox
  auto append_segments = [&](hipStream_t st) {
    launch_ob_concat(a.outbox, a.outbox_src, a.ob_seg_base, a.ob_seg_cap, a.qctr + (size_t)MAX_QUEUES * QCTR_STRIDE,
                     f->outbox_count(), st);
  };
  HIP_TRY(hipEventRecord(f->ev0, f->stream));
  f->log_need_known = false;  // the launch appends records the host does not count
  if (p->use_graph) {
    const int key[6] = {(int)grid, a.refill, a.budget, mode, (int)(p->h * 1e6f), spatial ? 1 : 0};
    bool same = f->graph && std::memcmp(key, f->graph_key, sizeof key) == 0 &&
                std::memcmp(&a, &f->graph_args, sizeof a) == 0;
    if (!same) {
      drop_graph(f);
      hipStream_t cs;
      HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      struct StreamGuard {  // the capture stream goes away on every return path
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
      } guard{cs};
      hipGraph_t g;
      HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      launch_fill_u64(a.ctr, CTR_N, 0, cs);
      launch_fill_u64(a.qctr, 2 * MAX_QUEUES * QCTR_STRIDE, 0, cs);
      if (spatial)
        launch_work_order((const float4*)f->d_pos.p, (const int4*)f->d_meta.p, (const int4*)f->d_meta2.p,
                          (const BlockDev*)f->d_blocks.p, f->n_particles, bits, n_buckets, n_classes, span, a.h, a.t_end, (unsigned*)f->d_key.p,
                          (unsigned*)f->d_hist.p, (unsigned*)f->d_cursor.p, (int*)f->d_order.p,
                          (unsigned*)f->d_nwork.p, cs);
      launch(cs);
      if (a.ob_seg_cap) append_segments(cs);
      HIP_TRY(hipStreamEndCapture(cs, &g));
      HIP_TRY(hipGraphInstantiate(&f->graph, g, nullptr, nullptr, 0));
      (void)hipGraphDestroy(g);
      std::memcpy(f->graph_key, key, sizeof key);
      f->graph_args = a;
    }
    HIP_TRY(hipGraphLaunch(f->graph, f->stream));
  } else {
    launch_fill_u64(a.ctr, CTR_N, 0, f->stream);
    launch_fill_u64(a.qctr, 2 * MAX_QUEUES * QCTR_STRIDE, 0, f->stream);
    if (spatial)
      launch_work_order((const float4*)f->d_pos.p, (const int4*)f->d_meta.p, (const int4*)f->d_meta2.p,
                        (const BlockDev*)f->d_blocks.p, f->n_particles, bits, n_buckets, n_classes, span, a.h, a.t_end, (unsigned*)f->d_key.p,
                        (unsigned*)f->d_hist.p, (unsigned*)f->d_cursor.p, (int*)f->d_order.p,
                        (unsigned*)f->d_nwork.p, f->stream);
    launch(f->stream);
    if (a.ob_seg_cap) append_segments(f->stream);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(f->ev1, f->stream));
  if (stats) return collect_stats(f, stats);
  return STREAMI_OK;
}

int streami_clear(streami_field f) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  drop_graph(f);
  f->n_particles = 0;
  f->active_hint = -1;
  f->vert_bound = 0;
  f->max_m = 0;
  f->min_m = INT_MAX;
  f->strides_mult16 = true;
  f->next_auto_id = 0;
  f->log_need_known = true;  // the counters below restart at zero
  f->log_need_hi = 0;
  f->ob_settled = 0;
  for (auto& hb : f->blocks) {
    hb.ranges.clear();
    hb.n_particles = 0;
  }
  launch_fill_u64(f->persist(), PER_N, 0, f->stream);
  HIP_TRY(hipGetLastError());
  return STREAMI_OK;
}

int streami_field_info(streami_field f, int32_t* layout, int64_t* field_bytes) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (layout) *layout = f->layout;
  if (field_bytes) *field_bytes = (int64_t)f->d_nodes.bytes;
  return STREAMI_OK;
}

int streami_block_info(streami_field f, int32_t block, int64_t* n_particles, int64_t* n_vertices) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (block < 0 || block >= (int)f->blocks.size()) return fail(STREAMI_E_ARG, "block %d out of range", block);
  if (n_particles) *n_particles = f->blocks[block].n_particles;
  if (n_vertices) {
    int64_t needed = 0;
    int rc = streami_fetch_lines(f, block, 0, f->blocks[block].n_particles, nullptr, nullptr, -1, nullptr, nullptr,
                                 nullptr, &needed);
    if (rc != STREAMI_OK && rc != STREAMI_E_CAPACITY) return rc;
    *n_vertices = needed;
  }
  return STREAMI_OK;
}

int streami_fetch_lines(streami_field f, int32_t block, int64_t first, int64_t count, int64_t* offsets, float* xyz,
                        int64_t cap_vertices, int32_t* steps, int32_t* codes, uint64_t* ids,
                        int64_t* needed_vertices) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (block < 0 || block >= (int)f->blocks.size()) return fail(STREAMI_E_ARG, "block %d out of range", block);
  HostBlock& hb = f->blocks[block];
  if (first < 0 || count < 0 || first + count > hb.n_particles)
    return fail(STREAMI_E_ARG, "range [%lld, %lld) outside the block's %lld particles", (long long)first,
                (long long)(first + count), (long long)hb.n_particles);
  // seed-order index list of the range
  std::vector<long long> idx;
  idx.reserve(count);
  long long skip = first;
  for (auto& r : hb.ranges) {
    if ((long long)idx.size() >= count) break;
    if (skip >= r.second) {
      skip -= r.second;
      continue;
    }
    for (long long k = skip; k < r.second && (long long)idx.size() < count; ++k) idx.push_back(r.first + k);
    skip = 0;
  }
  int rc;
  DevBuf d_idx, d_nv, d_steps, d_codes, d_ids;
  const long long c = std::max<long long>(count, 1);
  if ((rc = d_idx.reserve(c * 8, 0, f->stream)) || (rc = d_nv.reserve(c * 8, 0, f->stream)) ||
      (rc = d_steps.reserve(c * 4, 0, f->stream)) || (rc = d_codes.reserve(c * 4, 0, f->stream)) ||
      (rc = d_ids.reserve(c * 8, 0, f->stream)))
    return rc;
  std::vector<long long> nv(count);
  std::vector<int32_t> h_steps(count), h_codes(count);
  std::vector<unsigned long long> h_ids(count);
  if (count > 0) {
    HIP_TRY(hipMemcpyAsync(d_idx.p, idx.data(), count * 8, hipMemcpyHostToDevice, f->stream));
    launch_gather_meta((const long long*)d_idx.p, count, (const int4*)f->d_meta.p, (const int4*)f->d_meta2.p,
                       (const unsigned long long*)f->d_ids.p, (long long*)d_nv.p, (int*)d_steps.p,
                       (int*)d_codes.p, (unsigned long long*)d_ids.p, f->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(nv.data(), d_nv.p, count * 8, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipMemcpyAsync(h_steps.data(), d_steps.p, count * 4, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipMemcpyAsync(h_codes.data(), d_codes.p, count * 4, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipMemcpyAsync(h_ids.data(), d_ids.p, count * 8, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
  }
  std::vector<long long> off(count + 1);
  off[0] = 0;
  for (long long i = 0; i < count; ++i) off[i + 1] = off[i] + nv[i];
  if (needed_vertices) *needed_vertices = off[count];
  if (cap_vertices < off[count])
    return fail(STREAMI_E_CAPACITY, "need %lld vertices, capacity %lld", (long long)off[count], (long long)cap_vertices);
  if (!offsets || (!xyz && off[count] > 0)) return fail(STREAMI_E_ARG, "offsets/xyz is NULL");
  auto put = [&](void* dst, const void* src, size_t bytes) -> int {
    if (!dst || bytes == 0) return STREAMI_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, is_device_ptr(dst) ? hipMemcpyHostToDevice : hipMemcpyHostToHost,
                           f->stream));
    return STREAMI_OK;
  };
  if ((rc = put(offsets, off.data(), (count + 1) * 8))) return rc;
  if ((rc = put(steps, h_steps.data(), count * 4))) return rc;
  if ((rc = put(codes, h_codes.data(), count * 4))) return rc;
  if ((rc = put(ids, h_ids.data(), count * 8))) return rc;
  if (off[count] > 0) {
    // scatter the log records of the requested particles into CSR rows
    DevBuf d_row;
    unsigned long long cnt[PER_N];
    HIP_TRY(hipMemcpyAsync(cnt, f->persist(), sizeof cnt, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
    const long long n_rec = (long long)std::min<unsigned long long>(cnt[PER_LOG], (unsigned long long)f->log_cap);
    if ((rc = d_row.reserve(std::max<long long>(f->n_particles, 1) * 4, 0, f->stream))) return rc;
    launch_fill_u32((unsigned*)d_row.p, f->n_particles, 0xffffffffu, f->stream);
    launch_mark_rows((const long long*)d_idx.p, count, (int*)d_row.p, f->stream);
    const bool dev_out = is_device_ptr(xyz);
    DevBuf tmp;
    float* dst = xyz;
    if (!dev_out) {
      if ((rc = tmp.reserve(off[count] * 12, 0, f->stream))) return rc;
      dst = (float*)tmp.p;
    }
    // the requested particles' records, stably sorted by row, are the CSR lines
    auto alloc = [](size_t bytes, void*) -> void* {
      void* q = nullptr;
      if (hipMalloc(&q, std::max<size_t>(bytes, 16)) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      return q;
    };
    auto release = [](void* q, void*) { (void)hipFree(q); };
    const int arc = assemble_lines(f->log(), n_rec, f->n_particles, (const int*)d_row.p, count, off[count], dst,
                                   f->stream, alloc, release, nullptr);
    if (arc == 2) return fail(STREAMI_E_NOMEM, "scratch for assembling %lld vertices", (long long)off[count]);
    if (arc == 4) return fail(STREAMI_E_DEVICE, "vertex log inconsistent with the particles' vertex counts");
    if (arc) return fail(STREAMI_E_DEVICE, "line assembly failed");
    if (!dev_out) HIP_TRY(hipMemcpyAsync(xyz, tmp.p, off[count] * 12, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
  }
  HIP_TRY(hipStreamSynchronize(f->stream));
  return STREAMI_OK;
}

int streami_fetch_outbox(streami_field f, streami_outbox_rec* out, int64_t cap, int64_t* n_out) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (!n_out) return fail(STREAMI_E_ARG, "n_out is NULL");
  if (cap < 0) return fail(STREAMI_E_ARG, "cap must be >= 0");
  unsigned long long cnt = 0;
  HIP_TRY(hipMemcpyAsync(&cnt, f->outbox_count(), 8, hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(hipStreamSynchronize(f->stream));
  long long take = std::min<long long>((long long)cnt, cap);
  *n_out = take;
  if (take > 0) {
    if (!out) return fail(STREAMI_E_ARG, "out is NULL");
    // hand out the tail so that the remaining records stay contiguous at the front
    const OutRec* src = reinterpret_cast<const OutRec*>(f->d_outbox.p) + (cnt - take);
    HIP_TRY(hipMemcpyAsync(out, src, take * sizeof(OutRec),
                           is_device_ptr(out) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, f->stream));
    unsigned long long rest = cnt - take;
    f->ob_settled = std::min<long long>(f->ob_settled, (long long)rest);
    HIP_TRY(hipMemcpyAsync(f->outbox_count(), &rest, 8, hipMemcpyHostToDevice, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
  }
  if ((long long)cnt > take) return fail(STREAMI_E_CAPACITY, "%lld records remain in the outbox", (long long)(cnt - take));
  return STREAMI_OK;
}

int streami_forward(streami_field f, int64_t* n_forwarded, int64_t* n_active) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (f->n_ranks == 0)
    return fail(STREAMI_E_UNSUPPORTED, "forwarding needs every block on one rank grid, at most one block per cell "
                                       "(and at most %d blocks)", FWD_MAX_BLOCKS);
  const int nb = (int)f->blocks.size();
  int rc;
  unsigned long long ob = 0;
  HIP_TRY(hipMemcpyAsync(&ob, f->outbox_count(), 8, hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(hipStreamSynchronize(f->stream));
  // layout of d_fwd (u64 units): counts[nb], vertex bound, cursor[nb], kept, base[nb]
  if ((rc = f->d_fwd.reserve(sizeof(unsigned long long) * (3 * (size_t)nb + 2), 0, f->stream))) return rc;
  unsigned long long* counts = (unsigned long long*)f->d_fwd.p;
  unsigned long long* cursor = counts + nb + 1;
  unsigned long long* kept = cursor + nb;
  long long* base = (long long*)(kept + 1);
  long long total = 0;
  std::vector<unsigned long long> h(nb + 1, 0);
  // the records before `first` stayed in an earlier exchange (final exits): only the new ones are read
  const long long first = std::min<long long>(f->ob_settled, (long long)ob);
  if ((long long)ob > first) {
    FwdArgs a;
    a.outbox = (const OutRec*)f->d_outbox.p;
    a.outbox_src = (const int*)f->d_obsrc.p;
    a.outbox_count = f->outbox_count();
    a.first = first;
    a.rank_map = (const int*)f->d_rankmap.p;
    a.n_ranks = f->n_ranks;
    a.n_blocks = nb;
    a.pos = (const float4*)f->d_pos.p;
    a.meta = (const int4*)f->d_meta.p;
    a.meta2 = (const int4*)f->d_meta2.p;
    launch_fill_u64(counts, 2LL * nb + 2, 0, f->stream);
    launch_fwd_count(a, counts, (long long)ob - first, f->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h.data(), counts, sizeof(unsigned long long) * (nb + 1), hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
    for (int b = 0; b < nb; ++b) total += (long long)h[b];
    if (total > 0) {
      if (f->n_particles + total >= (1LL << 31))
        return fail(STREAMI_E_UNSUPPORTED, "forwarding would exceed 2^31 particles in one handle");
      // each block's new particles take one contiguous range after the existing ones
      std::vector<long long> hb(nb);
      long long next = f->n_particles;
      for (int b = 0; b < nb; ++b) {
        hb[b] = next;
        next += (long long)h[b];
      }
      if ((rc = ensure_particles(f, next))) return rc;
      f->vert_bound += (long long)h[nb];
      if ((rc = ensure_log(f, 0))) return rc;
      if ((rc = f->d_outbox2.reserve(f->cap_particles * sizeof(OutRec), 0, f->stream)) ||
          (rc = f->d_obsrc2.reserve(f->cap_particles * sizeof(int), 0, f->stream)))
        return rc;
      HIP_TRY(hipMemcpyAsync(base, hb.data(), sizeof(long long) * nb, hipMemcpyHostToDevice, f->stream));
      // the particle arrays may have moved
      a.pos = (const float4*)f->d_pos.p;
      a.meta = (const int4*)f->d_meta.p;
      a.meta2 = (const int4*)f->d_meta2.p;
      a.outbox = (const OutRec*)f->d_outbox.p;
      a.outbox_src = (const int*)f->d_obsrc.p;
      FwdOut o;
      o.base = base;
      o.cursor = cursor;
      o.pos = (float4*)f->d_pos.p;
      o.meta = (int4*)f->d_meta.p;
      o.meta2 = (int4*)f->d_meta2.p;
      o.ids = (unsigned long long*)f->d_ids.p;
      o.log = f->log();
      o.kept = (OutRec*)f->d_outbox2.p;
      o.kept_src = (int*)f->d_obsrc2.p;
      o.n_kept = kept;
      launch_fwd_write(a, o, (long long)ob - first, f->stream);
      launch_fwd_settle(o.kept, o.kept_src, kept, (OutRec*)f->d_outbox.p, (int*)f->d_obsrc.p, first,
                        f->outbox_count(), (long long)ob - first, f->stream);
      HIP_TRY(hipGetLastError());
      for (int b = 0; b < nb; ++b)
        if (h[b] > 0) {
          f->blocks[b].ranges.push_back({hb[b], (long long)h[b]});
          f->blocks[b].n_particles += (long long)h[b];
        }
      f->n_particles = next;
      f->log_need_known = false;
      drop_graph(f);  // the cached launch holds the old buffers
    }
  }
  f->ob_settled = (long long)ob - total;  // every record left in the outbox is final
  if (n_forwarded) *n_forwarded = total;
  if (n_active) {
    launch_fill_u64(f->code_counts(), 6, 0, f->stream);
    launch_count_codes((const int4*)f->d_meta.p, f->n_particles, f->code_counts(), f->stream);
    unsigned long long c = 0;
    HIP_TRY(hipMemcpyAsync(&c, f->code_counts() + ACTIVE, 8, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
    *n_active = (int64_t)c;
    f->active_hint = (long long)c;
  }
  return STREAMI_OK;
}

int streami_trace(streami_field f, const streami_advect_params* p, int32_t max_rounds, int32_t* rounds,
                  streami_stats* stats) {
  if (!f) return fail(STREAMI_E_ARG, "field handle is NULL");
  if (!p) return fail(STREAMI_E_ARG, "params is NULL");
  if (max_rounds < 1) return fail(STREAMI_E_ARG, "max_rounds must be >= 1");
  if (f->n_ranks == 0)
    return fail(STREAMI_E_UNSUPPORTED, "forwarding needs every block on one rank grid, at most one block per cell");
  streami_stats tot, st;
  std::memset(&tot, 0, sizeof tot);
  int r = 0, rc;
  int64_t active = 1;
  for (; r < max_rounds && active > 0; ++r) {
    if ((rc = streami_advect(f, p, stats ? &st : nullptr))) return rc;
    if (stats) {
      tot.steps += st.steps;
      tot.vertices += st.vertices;
      tot.surrogate_accepted += st.surrogate_accepted;
      tot.surrogate_fallback += st.surrogate_fallback;
      tot.device_ms += st.device_ms;
      tot.gathers += st.gathers;
    }
    int64_t fw = 0;
    if ((rc = streami_forward(f, &fw, &active))) return rc;
  }
  if (rounds) *rounds = r;
  if (stats) {
    // particle counts and the outbox after the last exchange
    launch_fill_u64(f->code_counts(), 6, 0, f->stream);
    launch_count_codes((const int4*)f->d_meta.p, f->n_particles, f->code_counts(), f->stream);
    unsigned long long h[PER_N + 6];
    HIP_TRY(hipMemcpyAsync(h, f->persist(), sizeof h, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
    for (int k = 0; k < 6; ++k) tot.terminated[k] = (int64_t)h[PER_N + k];
    tot.active = tot.terminated[ACTIVE];
    tot.outbox = (int64_t)h[PER_OUTBOX];
    *stats = tot;
  }
  return STREAMI_OK;
}

}  // extern "C"
