/*
 * streami.h -- C-ABI of the MI355X (gfx950) field-line advection library.
 *
 * The library advects many particles through the vector-field block(s) that
 * one GPU holds, with the classical fourth-order Runge-Kutta update, and
 * records each particle's polyline.  Particles that leave the owned bounds of
 * their block are written to an outbox together with the flat id of the
 * macrocell (rank) that owns their new position, instead of being sent.
 *
 * Paper: "Streami: An MPI Data-Parallel Library to Compute Field Lines on
 * GPUs".  Where each call comes from:
 *   - a field is set by the application in its own layout, one per time step
 *     (Sec. 3.2, Tracer::setField; Sec. 3.3, structured float3 voxel grid);
 *   - sampling is defined on the block's domain = owned bounds + halo, and is
 *     undefined outside it (Sec. 3.1.1, sample() and the macrocell domain);
 *   - destinationID() maps a position to the flat id of the macrocell grid
 *     cell that holds it (Sec. 3.1.1, uniform grid of macrocells);
 *   - particles are a position and a unique id (Sec. 3.1.2);
 *   - one RK4 update per particle and step, then the destination test and the
 *     buffered emitOutgoing() (Sec. 3.1.2, the update kernel listing);
 *   - Tracer::step()/trace() advance one step / until no particle is active,
 *     streamlines seed once, streaklines re-seed periodically (Sec. 3.2, the
 *     step() listing); getLines() returns the assembled lines (Sec. 3.2).
 *
 * Conventions for every call:
 *   - returns STREAMI_OK (0) or a STREAMI_E_* code; nothing aborts and no C++
 *     exception crosses the ABI; streami_last_error() gives the calling
 *     thread's last message;
 *   - a handle is bound to the device that was current at creation and to one
 *     HIP stream; all device work is enqueued on that stream; a handle is not
 *     thread-safe;
 *   - caller buffers are only read (inputs) or only written (outputs) during
 *     the call and stay owned by the caller; the library owns every device
 *     buffer it allocates until streami_field_destroy().
 */
#ifndef STREAMI_H
#define STREAMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define STREAMI_OK 0
#define STREAMI_E_ARG 1         /* invalid argument; nothing was changed */
#define STREAMI_E_NOMEM 2       /* device or host allocation failed */
#define STREAMI_E_DEVICE 3      /* a HIP call failed */
#define STREAMI_E_STATE 4       /* call not valid in the handle's current state */
#define STREAMI_E_CAPACITY 5    /* output buffer too small; required size reported */
#define STREAMI_E_UNSUPPORTED 6 /* valid request the library does not implement */
#define STREAMI_E_IO 7          /* a file could not be opened or written */

/* ---- node storage formats (the GPU never quantises: nodes arrive in this format) ---- */
#define STREAMI_F32 0
#define STREAMI_F16 1
#define STREAMI_BF16 2

/* ---- block boundary handling ---- */
#define STREAMI_BOUNDARY_BLOCK 0    /* exits go to the outbox */
#define STREAMI_BOUNDARY_PERIODIC 1 /* sampling wraps, positions stay unwrapped, no exits */

/* ---- termination codes of a particle ---- */
#define STREAMI_ACTIVE 0
#define STREAMI_MAX_STEPS 1
#define STREAMI_EXIT 2      /* left the owned bounds; in the outbox */
#define STREAMI_STAGNANT 3  /* |v| < stagnation_eps at the start of a step */
#define STREAMI_HALO_MISS 4 /* a stage sample was undefined; in the outbox at the old position */
#define STREAMI_NONFINITE 5 /* a sampled value or the new position was NaN/Inf */

/* ---- field storage layouts ---- */
#define STREAMI_LAYOUT_AUTO 0
#define STREAMI_LAYOUT_LINEAR 1 /* x-fastest node rows */
#define STREAMI_LAYOUT_BRICK4 2 /* 4x4x4-node bricks, bricks in x-fastest order */
/* FP32 only: one 96-byte record per cell with the monomial coefficients of its
 * trilinear interpolant (the sample arithmetic of Sec. 3.1.1 moved to ingest);
 * 8x the bytes of LINEAR, and results bit-identical to LINEAR for steady
 * fields. */
#define STREAMI_LAYOUT_CELL 3
#define STREAMI_LAYOUT_HEX 4 /* reported by streami_field_info for a hexahedral field (never requested) */
#define STREAMI_LAYOUT_BRICK8 5 /* 8x8x8-node bricks, bricks in x-fastest order (each axis padded to a
                                   multiple of 8; a plane of bricks must stay below 16 MiB) */

/* ---- advection modes ---- */
#define STREAMI_MODE_PLAIN 0
#define STREAMI_MODE_SURROGATE 1

typedef struct streami_field_s* streami_field;
typedef struct streami_mlp_s* streami_mlp;

/*
 * One block = the part of the domain one rank holds (a macrocell and its
 * halo, Sec. 3.1.1).  Node (i,j,k) of slice s is stored at
 *   nodes[(((s*(nz+2g) + k)*(ny+2g) + j)*(nx+2g) + i)*3 + c],  c = x,y,z component,
 * where storage index 0 is the first ghost node, so interior node (0,0,0) sits
 * at world position `origin`.  Storage coordinate of world x along an axis:
 *   s = (x - origin)/spacing + ghost;  sample() is defined for 0 <= s <= n_store-1
 * (closed), and the value is the trilinear interpolant of the 8 surrounding
 * nodes.  With PERIODIC boundary, ghost must be 0 and indices wrap modulo
 * dims.  Owned bounds are half-open [bounds_lo, bounds_hi).
 * Time slices: slice s holds time t0 + s*slice_dt; between slices the value
 * is blended linearly in time, clamped to the first/last slice pair.
 */
typedef struct {
  int32_t dims[3];         /* interior nodes per axis, >= 1 */
  int32_t ghost;           /* ghost layers per face: 0 or 1 (0 when periodic) */
  double origin[3];        /* world position of interior node (0,0,0) */
  double spacing[3];       /* node spacing per axis, > 0 */
  double bounds_lo[3];     /* owned region, half-open */
  double bounds_hi[3];
  int32_t boundary;        /* STREAMI_BOUNDARY_* */
  int32_t rank_grid[3];    /* macrocell grid dims for destinationID, >= 1 */
  int32_t rank_coord[3];   /* this block's cell in that grid */
  int32_t n_slices;        /* >= 1 */
  double t0;               /* time of slice 0 */
  double slice_dt;         /* > 0 when n_slices > 1 */
  const void* nodes;       /* node values in the handle's dtype (see layout above) */
  int32_t nodes_on_device; /* 1: `nodes` is a device pointer, 0: host memory */
} streami_block_desc;

typedef struct {
  int32_t layout; /* STREAMI_LAYOUT_*; AUTO: CELL when dtype is F32, every block
                     has one slice and fits CELL's limits (below), else LINEAR */
} streami_field_opts;

/*
 * Create a handle over n_blocks blocks (1 for a rank's single block; many
 * for a batched launch) that all store nodes in `dtype`.  The node values are
 * copied into the library's own device buffer and re-laid-out there (the
 * caller keeps ownership of `nodes`); the copy is complete when this returns.
 * hip_stream: the hipStream_t all later work of this handle is enqueued on
 * (NULL = the default stream).  opts may be NULL.
 * Errors: E_ARG for an invalid descriptor (the message names the field);
 * E_UNSUPPORTED for more than 315 blocks, a PERIODIC block in a handle with
 * several blocks or time slices, the CELL layout with a 16-bit dtype, or a
 * block whose time slice exceeds 2 GiB or whose z plane of nodes (CELL: of
 * cell records) exceeds 16 MiB in the chosen layout (the kernels use 32-bit
 * offsets; split such a block); E_NOMEM, E_DEVICE.  *out is set only on
 * success.
 */
int streami_field_create(const streami_block_desc* blocks, int32_t n_blocks, int32_t dtype,
                         const streami_field_opts* opts, void* hip_stream, streami_field* out);

int streami_field_destroy(streami_field f);

/* An unstructured field (Sec. 3.3: the paper's second field type, of
 * tetrahedra, pyramids, prisms and hexahedra, located by a bounding volume
 * hierarchy and point containment; Sec. 5 converts every voxel of a structured
 * data set to a hexahedron). */
#define STREAMI_CELL_TETRA 10      /* VTK cell type codes */
#define STREAMI_CELL_HEXAHEDRON 12
#define STREAMI_CELL_WEDGE 13
#define STREAMI_CELL_PYRAMID 14
typedef struct {
  int64_t n_vertices;
  const float* vertices;   /* [n_vertices][3] world positions */
  const float* values;     /* [n_vertices][3] FP32 vector values at the vertices */
  int64_t n_cells;         /* 1 .. 2^28 - 1 */
  const int32_t* cells;    /* [n_cells][8]: each row the cell's vertex indices in VTK order, entries
                              after the cell's vertices ignored.  Hexahedron (0,0,0) (1,0,0) (1,1,0)
                              (0,1,0) (0,0,1) (1,0,1) (1,1,1) (0,1,1); tetra 4 vertices; wedge the
                              bottom triangle then the top one (vertex 3 above 0, 4 above 1, 5 above
                              2); pyramid the base quad in cyclic order then the apex */
  double bounds_lo[3];     /* owned macrocell, half-open [lo, hi) (Sec. 3.1.1) */
  double bounds_hi[3];
  int32_t rank_grid[3];    /* macrocell grid for destinationID() */
  int32_t rank_coord[3];
  int32_t inputs_on_device;/* 1: the arrays are device pointers, 0: host memory */
  const uint8_t* cell_types; /* [n_cells] STREAMI_CELL_* codes, or NULL: every cell a hexahedron */
} streami_hex_desc;

/*
 * Create a handle over one unstructured field.  sample(x) is defined where a
 * cell holds x.  Each cell maps parametric coordinates (r,s,u) to space with
 * its kind's VTK linear shape functions: hexahedron trilinear over [0,1]^3;
 * tetra 1-r-s-u, r, s, u over the simplex r,s,u >= 0, r+s+u <= 1; wedge
 * (1-r-s)(1-u), r(1-u), s(1-u), (1-r-s)u, ru, su over r,s >= 0, r+s <= 1,
 * 0 <= u <= 1; pyramid (1-r)(1-s)(1-u), r(1-s)(1-u), rs(1-u), (1-r)s(1-u), u
 * over [0,1]^3.  The map is inverted by Newton's method in FP32 and x is
 * accepted when (r,s,u) lies in the domain widened by 1e-4 (slack for points on
 * shared faces); the value is the same combination of the vertex values.  A
 * pyramid's map is singular at its apex: points within about 1e-5 of a cell
 * size of it may be found in no cell.  The library builds, on the host, a
 * depth-first BVH over the cells' boxes and one 192-byte record per cell (both
 * maps in monomial form) and keeps them on the device; the caller keeps
 * ownership of the arrays (read during the call only).  The handle takes the
 * same seeding, advection (PLAIN mode, steady), fetch, outbox, forwarding and
 * OBJ calls as a structured one; streami_field_info reports
 * STREAMI_LAYOUT_HEX.  Errors: E_ARG (NULL arrays, counts out of range, an
 * unknown cell type, a cell index outside the vertices, a non-finite vertex,
 * bounds with lo >= hi, a rank grid < 1 or coordinate outside it), E_NOMEM,
 * E_DEVICE.
 */
int streami_field_create_hex(const streami_hex_desc* desc, void* hip_stream, streami_field* out);

/* Seeding options (Sec. 3.2: streamlines seed once at step 0). */
typedef struct {
  int32_t default_max_steps; /* per-particle step limit when max_steps == NULL, >= 0 */
  int32_t record_stride;     /* keep vertex j when j % stride == 0, and the final vertex; >= 1 */
  int32_t inputs_on_device;  /* 1: xyz/ids/max_steps are device pointers */
  float t_birth;             /* time of step 0 of these particles (unsteady fields) */
  const float* t_births;     /* per-particle birth times (host or device like xyz) or NULL:
                                streaklines release particles from the same emitter at
                                different times (Sec. 3.2) */
} streami_seed_opts;

/*
 * Append n particles to block `block`.  xyz: n*3 FP32 positions; ids: n
 * unique ids or NULL (then ids continue a per-handle counter from 0);
 * max_steps: n per-particle limits (>= 0) or NULL.  Each particle reserves
 * room for max_steps/record_stride + 2 vertex records (16 bytes each) in the
 * handle's vertex log.  The seed position is vertex 0; a seed outside the
 * block's owned bounds (BLOCK boundary) terminates at once with code EXIT and
 * 0 steps and goes to the outbox.  Particles of a block keep their seed order
 * for streami_fetch_lines().  Step limits on the device are reduced on the
 * device (24 bytes come back); host limits are read directly.
 * Errors: E_ARG (bad block, opts or a negative limit), E_NOMEM, E_DEVICE.
 */
int streami_seed(streami_field f, int32_t block, const float* xyz, const uint64_t* ids,
                 const int32_t* max_steps, int64_t n, const streami_seed_opts* opts);

/* A control shape for streami_seed_shape(). */
#define STREAMI_SHAPE_LINE 0
#define STREAMI_SHAPE_PLANE 1
typedef struct {
  int32_t kind;     /* STREAMI_SHAPE_LINE or STREAMI_SHAPE_PLANE */
  double origin[3]; /* line: start point; plane: corner */
  double u[3];      /* line: end - start; plane: first edge */
  double v[3];      /* plane: second edge (ignored for a line) */
  int64_t nu;       /* points along u, >= 0 */
  int64_t nv;       /* points along v, >= 1 (ignored for a line: 1) */
} streami_shape;

/*
 * Uniformly distributed seed points on a simple control shape, generated on
 * the device (Sec. 3.1.2: the low-level interface's convenience kernels seed
 * planes and lines).  Point k = i + nu*j (i fastest) is the midpoint-rule
 * sample  origin + ((2i+1)/(2 nu)) u + ((2j+1)/(2 nv)) v  of the segment
 * (nv = 1, v = 0) or parallelogram, evaluated in FP32 from the FP32-rounded
 * shape (correctly rounded parameters, two fused multiply-adds per
 * coordinate: within 3 ulp of |origin|+|u|+|v| of the exact point).  The
 * points are then seeded exactly as streami_seed() seeds an array of them:
 * same ids, limits (max_steps: nu*nv limits or NULL, host or device as
 * opts->inputs_on_device says), birth times, record stride, and the same
 * treatment of points outside the owned bounds.  The point array is a call
 * temporary.  Errors: E_ARG (bad block, kind, counts, a non-finite shape or
 * more than 2^31 points), then those of streami_seed().
 */
int streami_seed_shape(streami_field f, int32_t block, const streami_shape* shape, const int32_t* max_steps,
                       const streami_seed_opts* opts);

/*
 * Path lines (Sec. 3.2 names them as a further line kind the framework makes
 * easy): the trajectory of one particle through a time-varying field.  They
 * need no call of their own: seed the particles of a field with time slices
 * (n_slices > 1) at their release times (opts->t_birth or t_births), with
 * record_stride = 1, and advect; each line fetched by streami_fetch_lines()
 * is then the particle's path line, vertex i at time t_birth + i*h.
 * Streamlines are the same call on a steady field, streaklines the
 * emitters' particles' final positions ordered by release time.
 */

/* One seed batch of streami_seed_batches(): the arguments of one
 * streami_seed() call (birth times per batch instead of in the options). */
typedef struct {
  int32_t block;
  const float* xyz;         /* n*3 positions */
  const uint64_t* ids;      /* n ids or NULL */
  const int32_t* max_steps; /* n limits or NULL */
  const float* t_births;    /* n birth times or NULL (then opts->t_birth) */
  int64_t n;
} streami_seed_batch;

/*
 * Seed several batches (e.g. one per block of a batched launch) with shared
 * options: the same particles, ids and lines as n_batches consecutive
 * streami_seed() calls, but one device reduction of all step limits and at
 * most one wait instead of one per call (and one seeding launch per 48
 * batches).  opts->t_births must be NULL.  Every argument error is found
 * before anything is seeded.  Errors: as streami_seed(), naming the batch.
 */
int streami_seed_batches(streami_field f, const streami_seed_batch* batches, int32_t n_batches,
                         const streami_seed_opts* opts);

typedef struct {
  float h;                  /* step size in world units per unit time, > 0 */
  int32_t step_budget;      /* >0: at most this many steps per particle in this call (step());
                               0: run every particle to termination (trace()) */
  float stagnation_eps;     /* STAGNANT when |v(P0)|_2 < eps at the start of a step */
  int32_t mode;             /* STREAMI_MODE_PLAIN or STREAMI_MODE_SURROGATE */
  streami_mlp mlp;          /* trained network for SURROGATE mode, else NULL */
  float residual_tol_cells; /* SURROGATE: accept a jump when its residual <= tol (cells) */
  int32_t residual_kind;    /* SURROGATE: 0 commutation residual, 1 one big RK4 step */
  int32_t waves_per_cu;     /* launch shape; 0 = library default (32 for the CELL layout or more
                               than 2^21 particles, else 16) */
  int32_t refill_threshold; /* free lanes that trigger a work-queue refill; 0 = default (1) */
  int32_t use_graph;        /* 1: capture the launch sequence in a hipGraph and replay it */
  int32_t no_cell_cache;    /* 1: re-gather a cell's corners at every sample (A/B measurement;
                               results are bit-identical either way) */
  int32_t work_order;       /* 0: spatial order (block, Morton brick) split over per-XCD queues,
                               except for calls with a step_budget of 1 (seed order there);
                               1: seed order, one queue (results are bit-identical either way) */
  int32_t use_t_end;        /* 1: advance in a time window: a particle takes a step only while its
                               time t_birth + steps*h is < t_end, and stays ACTIVE at t_end (PLAIN
                               mode).  Successive calls with growing t_end bring every particle to
                               a common time and give bit-identical results to one call without a
                               window */
  float t_end;              /* end of the window (with use_t_end); must not be NaN */
  int32_t checked_samples;  /* 1: test every sample's domain, also for steps that start deep inside a
                               single block (A/B measurement; results are bit-identical either way) */
  int32_t lds_cell_cache;   /* 1: keep each lane's cached cell record in LDS (24 KB per workgroup)
                               instead of registers, for steady FP32 cell records in a one-block
                               handle (ignored elsewhere; results are bit-identical either way) */
} streami_advect_params;

typedef struct {
  int64_t active;              /* particles still ACTIVE after the call */
  int64_t steps;               /* RK4 steps taken in this call (a surrogate jump counts 16) */
  int64_t vertices;            /* vertices recorded in this call */
  int64_t outbox;              /* records currently in the outbox */
  int64_t surrogate_accepted;  /* jumps accepted */
  int64_t surrogate_fallback;  /* jumps rejected and redone with plain RK4 */
  int64_t terminated[6];       /* particles per termination code after the call */
  double device_ms;            /* device time of the advect kernels of this call */
  int64_t gathers;             /* PLAIN mode: the lanes' cell-cache refills in this call (a
                                  refill of a time-sliced field reads both slices; without the
                                  cache every defined sample is one) */
} streami_stats;

/*
 * Advance every ACTIVE particle of the handle (all blocks), like
 * Tracer::trace() (step_budget == 0) or a step() of step_budget steps.
 * Enqueued on the handle's stream; returns without waiting unless stats !=
 * NULL, in which case it waits and fills *stats.  A call with a budget that
 * is resumed by further calls produces bit-identical lines, step counts and
 * codes to a single unbudgeted call.  Errors: E_ARG (bad params), E_STATE
 * (no particles, or SURROGATE without a network), E_UNSUPPORTED (SURROGATE
 * with a time window, several blocks or time slices), E_NOMEM (vertex log
 * growth), E_DEVICE.
 */
int streami_advect(streami_field f, const streami_advect_params* p, streami_stats* stats);

/*
 * Copy the lines of particles [first, first+count) of `block` in seed order,
 * as CSR: offsets[count+1] (offsets[0] = 0), xyz[offsets[count]*3] FP32.
 * steps, codes (int32) and ids (uint64) per particle may be NULL.
 * If cap_vertices < the number of vertices needed, nothing is copied,
 * *needed_vertices is set and E_CAPACITY returned (two-call pattern).
 * Output pointers may be host or device memory (detected); the call waits for
 * the handle's stream before returning.  Errors: E_ARG, E_CAPACITY, E_DEVICE.
 */
int streami_fetch_lines(streami_field f, int32_t block, int64_t first, int64_t count,
                        int64_t* offsets, float* xyz, int64_t cap_vertices, int32_t* steps,
                        int32_t* codes, uint64_t* ids, int64_t* needed_vertices);

/* Outbox record: a particle that left its block (emitOutgoing, Sec. 3.1.2). */
typedef struct {
  uint64_t id;
  float pos[3];  /* new position for EXIT, old position for HALO_MISS */
  int32_t steps; /* steps taken when it left */
  int32_t dest;  /* destinationID of pos (EXIT) or of the failing stage point (HALO_MISS); -1 outside the rank grid */
  int16_t code;  /* STREAMI_EXIT or STREAMI_HALO_MISS */
  int16_t block; /* block index within the handle */
} streami_outbox_rec;

/*
 * Move up to `cap` outbox records into `out` (host or device memory,
 * detected) and remove them from the outbox; *n_out = records copied.  Record
 * order is unspecified.  If more records remain than cap, cap of them are
 * copied and the call returns E_CAPACITY with *n_out = cap; the rest stay for
 * the next call.  Waits for the handle's stream.  Errors: E_ARG (NULL handle,
 * n_out, or out with records to copy; cap < 0), E_CAPACITY, E_DEVICE.
 */
int streami_fetch_outbox(streami_field f, streami_outbox_rec* out, int64_t cap, int64_t* n_out);

/*
 * Loopback forwarding: the exchange of outgoing particles between the blocks
 * of one handle (the paper's forwarding of outgoing particles to the rank that
 * owns their new position, rafi_forwardParticles in the step() listing of
 * Sec. 3.2, followed by its numActiveAcrossAllRanks count), done on the GPU.
 * Every outbox record whose `dest` (destinationID, Sec. 3.1.1) is the
 * macrocell of a block of this handle becomes a new particle of that block:
 * the same id, step count, step limit, birth time and record stride, at the
 * record's position, which is vertex 0 of the particle's next line segment
 * (an EXIT record: the exit vertex, also the last vertex of the segment it
 * left, so stitched segments share that joint; a HALO_MISS record: the old
 * position, from which the owner of the failing stage point redoes the step;
 * a halo miss is never sent back to the block it came from).  The forwarded
 * records leave the outbox; the others (destinations outside the handle, -1)
 * stay.  A block's forwarded particles follow its earlier ones in
 * streami_fetch_lines() order, in unspecified order among themselves;
 * segments of one id are ordered by their step counts.
 * Needs every block of the handle on the same rank_grid with distinct
 * rank_coord (E_UNSUPPORTED otherwise).  Waits for the handle's stream.
 * *n_forwarded (nullable): records forwarded; *n_active (nullable): particles
 * ACTIVE after the exchange, over all blocks.  Errors: E_ARG, E_UNSUPPORTED
 * (no common rank grid, or more than 2^31 particles), E_NOMEM, E_DEVICE.
 */
int streami_forward(streami_field f, int64_t* n_forwarded, int64_t* n_active);

/*
 * trace() with forwarding (the step() listing of Sec. 3.2 on one GPU): repeat
 * { streami_advect(p); streami_forward() } until no particle is active or
 * max_rounds rounds ran.  With p->step_budget = k each round advances every
 * particle by at most k steps before the exchange (k = 1 is the paper's
 * one-step exchange); with 0 each round runs the local particles to
 * termination or exit first.  Every budget gives the same lines; the time
 * differs: a round ends with its longest trajectory, so a budget of a few
 * hundred steps, which lets long trajectories continue in the next round beside
 * the others, is usually fastest (256 steps: 1.7x the run-to-exit rounds on a
 * 256^3 field split into 2x2x2 blocks), while small budgets pay per round.
 * *rounds (nullable) receives the rounds run.
 * stats (nullable) sums steps, vertices, gathers, surrogate counts and device
 * time over the rounds and reports particle codes and the outbox after the
 * last exchange.  Errors: as streami_advect() and streami_forward(), E_ARG
 * for max_rounds < 1.
 */
int streami_trace(streami_field f, const streami_advect_params* p, int32_t max_rounds, int32_t* rounds,
                  streami_stats* stats);

/*
 * Drop every particle, line and outbox record of the handle (the field data
 * stays), so the same handle can trace a new seed set -- a new Tracer run on
 * the same fields (Sec. 3.2).  Device buffers are kept for reuse.
 */
int streami_clear(streami_field f);

/* Particle counts of a block (for sizing fetch buffers). */
int streami_block_info(streami_field f, int32_t block, int64_t* n_particles, int64_t* n_vertices);

/* The storage the handle chose: *layout (nullable) receives the STREAMI_LAYOUT_*
 * in use (never AUTO) and *field_bytes (nullable) the device bytes of the
 * stored field, all blocks and slices.  E_ARG for a NULL handle. */
int streami_field_info(streami_field f, int32_t* layout, int64_t* field_bytes);

/* ---------------------------------------------------------------------------
 * Learned flow-map surrogate (not part of the paper: one of the forms this
 * library adds).  A multilayer perceptron maps a position to the displacement
 * of 16 plain RK4 steps:
 *   xhat = 2 (x mod L)/L - 1;  h0 = xhat;  h_{l+1} = SiLU(W_l h_l + b_l), l = 0..3,
 *   widths 3 -> 256 -> 256 -> 256 -> 256;  out = sigma * (W_4 h_4 + b_4)   [3].
 * Weights and activations enter the matrix cores as BF16 with FP32
 * accumulation; FP32 master weights are updated by Adam (b1 = 0.9,
 * b2 = 0.999, eps = 1e-8).  Parameter order of every flat array below: for
 * l = 0..4, W_l (row-major [out x in]) then b_l; 199,171 floats in total.
 * All xyz/target/out arrays are device pointers (n x 3 FP32).
 * ------------------------------------------------------------------------- */
int streami_mlp_create(const float* params, const float* sigma, float period, void* hip_stream,
                       streami_mlp* out);
int streami_mlp_destroy(streami_mlp m);
int streami_mlp_set_params(streami_mlp m, const float* params);  /* host array */
int streami_mlp_get_params(streami_mlp m, float* params);        /* host array */
/* Network output for n positions (enqueued on the network's stream). */
int streami_mlp_forward(streami_mlp m, const float* xyz, int64_t n, float* out);
/* One training step on `batch` samples: loss = mean(((out - target)/sigma)^2);
 * backprop; Adam with learning rate lr (lr = 0: gradients only).  loss_out
 * (host, nullable) receives the batch loss; grads_out (host, nullable,
 * 199,171 floats) the gradients of this step.  Waits for the stream when
 * either output is requested. */
int streami_mlp_train_step(streami_mlp m, const float* xyz, const float* target, int64_t batch, float lr,
                           float* loss_out, float* grads_out);

/* Allocation-free variant of streami_mlp_train_step, for callers that cannot
 * allocate device memory during a call (code under HIP graph capture, tight
 * training or serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernels, results and outputs as streami_mlp_train_step, but the
 * per-batch workspace (layer activations, pre-activations and their
 * gradients, 10,432 bytes per row) lives in one library-static device array
 * per GPU, sized for STREAMI_MLP_NOALLOC_MAX_BATCH rows (85.5 MB, held by
 * every GPU the library runs on until the process ends).  The call allocates
 * nothing (no hipMalloc/hipFree, no library allocation) and does not grow the
 * network's own workspace.  batch must be in [1, STREAMI_MLP_NOALLOC_MAX_BATCH],
 * else E_ARG.  All calls on one GPU share that array: calls whose work may
 * overlap on the device (different streams, or different threads without
 * ordering) race and give undefined results; calls ordered on one stream are
 * safe.  Nothing needs clearing between calls (a step writes every workspace
 * element before reading it). */
#define STREAMI_MLP_NOALLOC_MAX_BATCH 8192
int streami_mlp_train_step_noalloc(streami_mlp m, const float* xyz, const float* target, int64_t batch, float lr,
                                   float* loss_out, float* grads_out);

/* ---------------------------------------------------------------------------
 * Wavefront OBJ output of field lines (Sec. 4: the command line app writes the
 * lines of all particles, gathered over every time step and rank, to one joint
 * obj file of line elements).  Host-side; no device work.
 * ------------------------------------------------------------------------- */

/*
 * Write n_lines polylines given as CSR host arrays (offsets[n_lines+1], xyz
 * [offsets[n_lines]*3] FP32) to `path`: one "v x y z" record per vertex (%.9g,
 * which reads back as the same FP32 value), then one "l a b c ..." element
 * per line with at least two vertices (1-based indices); a line with fewer
 * vertices contributes its vertex records but no element.  append = 0 creates
 * or truncates the file, 1 appends to it; *vertex_base (in/out, nullable =
 * 0) is the number of vertex records already in the file and is advanced past
 * this call's, so repeated appends build one joint file.  Errors: E_ARG (NULL
 * arrays with n_lines > 0, decreasing offsets), E_IO (open/write failure).
 */
int streami_write_obj(const char* path, int64_t n_lines, const int64_t* offsets, const float* xyz, int32_t append,
                      int64_t* vertex_base);

/*
 * The lines of every block of a handle, in block then seed order, fetched to
 * the host and written as one OBJ file (created or truncated).  Errors: those
 * of streami_fetch_lines() and streami_write_obj(), E_NOMEM for host buffers.
 */
int streami_write_obj_field(streami_field f, const char* path);

/* Thread-local description of the last error. *//* Thread-local description of the last error. */
const char* streami_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STREAMI_H */
