/*
 * FP64 CPU oracle for rank-local RK4 field-line advection.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load this library.  It shares no code with the GPU
 * library: no headers, no helpers, no tables.
 *
 * What it computes, and where the paper defines it:
 *  - sample(): the field value at a position, or "undefined" when the position
 *    is outside the data this block holds (Sec. 3.1.1, sample() semantics).
 *    Structured field = node values on a uniform grid addressed by offset
 *    computation (Sec. 3.3); the value between nodes is the trilinear
 *    interpolant, written here as its plain 8-term weighted sum.
 *  - destinationID(): flat rank id of the uniform grid of macrocells holding a
 *    position, by offset computation (Sec. 3.1.1, Fig. device-classes).
 *  - one classical RK4 update per particle (Sec. 3.1.2, Listing update), with
 *    the pseudocode's slips read as: the factor is 1.0/6 (not integer 1/6), the
 *    k's are h * v(.), the destination is computed from the new position.
 *  - termination: max steps, stagnation |k1| < eps, exit from the owned bounds
 *    (the particle goes to the outbox with its destination), undefined sample
 *    ("halo miss": the particle goes to the outbox at its old position with its
 *    step count unchanged so the owner of the data can redo the step), and
 *    non-finite values.
 *  - unsteady fields: one field per time slice (Sec. 3.2, one field per time
 *    step), blended linearly in time between the two neighbouring slices.
 *  - periodic blocks: sampling wraps, positions stay unwrapped, no exits.
 *
 * Everything is FP64.  Stored nodes (FP32 / FP16 / BF16 / FP64) are decoded
 * exactly to FP64 here by this file's own decoder.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_F32 = 0, ORC_F16 = 1, ORC_BF16 = 2, ORC_F64 = 3 };
enum { ORC_ACTIVE = 0, ORC_MAX_STEPS = 1, ORC_EXIT = 2, ORC_STAGNANT = 3, ORC_HALO_MISS = 4,
       ORC_NONFINITE = 5 };
enum { ORC_FIELD_GRID = 0, ORC_FIELD_ABC = 1 };

typedef struct {
  int32_t dims[3];       /* interior nodes along x, y, z */
  int32_t ghost;         /* ghost layers on every face (0 for periodic) */
  double origin[3];      /* world position of interior node (0,0,0) */
  double spacing[3];     /* node spacing per axis */
  double lo[3], hi[3];   /* owned bounds, half-open [lo, hi) */
  int32_t periodic;      /* 1: sampling wraps, no exits */
  int32_t rank_grid[3];  /* macrocell grid dimensions */
  int32_t rank_coord[3]; /* this block's cell in the macrocell grid */
  int32_t n_slices;      /* time slices (1 = steady) */
  double t0, slice_dt;   /* time of slice 0 and slice spacing */
  const void* nodes;     /* [S][nz+2g][ny+2g][nx+2g][3], x fastest */
  int32_t fmt;           /* ORC_F32 / ORC_F16 / ORC_BF16 / ORC_F64 */
  int32_t field_kind;    /* ORC_FIELD_GRID, or ORC_FIELD_ABC (analytic, test pin) */
  double abc[3];         /* A, B, C for the analytic ABC field */
} orc_block;

/* ---------------- exact decoding of stored values ---------------- */
static double dec_f16(uint16_t h) {
  int s = h >> 15, e = (h >> 10) & 0x1F, f = h & 0x3FF;
  double v;
  if (e == 0) v = ldexp((double)f, -24);
  else if (e == 31) v = f ? NAN : INFINITY;
  else v = ldexp(1.0 + f / 1024.0, e - 15);
  return s ? -v : v;
}
static double dec_bf16(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double node_value(const orc_block* b, int64_t flat_vec3, int c) {
  int64_t i = flat_vec3 * 3 + c;
  switch (b->fmt) {
    case ORC_F32: return (double)((const float*)b->nodes)[i];
    case ORC_F16: return dec_f16(((const uint16_t*)b->nodes)[i]);
    case ORC_BF16: return dec_bf16(((const uint16_t*)b->nodes)[i]);
    default: return ((const double*)b->nodes)[i];
  }
}

/* ---------------- sample(): trilinear value of one time slice ---------------- */
/* Per-axis cell index pair and fraction.  Returns 0 if the coordinate is
 * outside the stored nodes (closed interval), which makes sample() undefined. */
static int axis_locate(const orc_block* b, int a, double x, int64_t* i0, int64_t* i1, double* f) {
  int64_t n = b->dims[a];
  if (b->periodic) {
    double s = (x - b->origin[a]) / b->spacing[a];
    double fl = floor(s);
    if (!isfinite(s)) return 0;
    int64_t k = (int64_t)fl % n;
    if (k < 0) k += n;
    *i0 = k;
    *i1 = (k + 1) % n;
    *f = s - fl;
    return 1;
  }
  int64_t ns = n + 2 * b->ghost;
  double s = (x - b->origin[a]) / b->spacing[a] + b->ghost;
  if (!(s >= 0.0 && s <= (double)(ns - 1))) return 0;
  int64_t k = (int64_t)floor(s);
  if (k > ns - 2) k = ns - 2;
  *i0 = k;
  *i1 = k + 1;
  *f = s - (double)k;
  return 1;
}

static int sample_slice(const orc_block* b, int slice, const int64_t ix[2], const int64_t iy[2],
                        const int64_t iz[2], const double w[3][2], double v[3]) {
  int64_t sx = b->dims[0] + 2 * (b->periodic ? 0 : b->ghost);
  int64_t sy = b->dims[1] + 2 * (b->periodic ? 0 : b->ghost);
  int64_t sz = b->dims[2] + 2 * (b->periodic ? 0 : b->ghost);
  int64_t slice_base = (int64_t)slice * sx * sy * sz;
  v[0] = v[1] = v[2] = 0.0;
  for (int c3 = 0; c3 < 2; ++c3)
    for (int b3 = 0; b3 < 2; ++b3)
      for (int a3 = 0; a3 < 2; ++a3) {
        double wt = w[0][a3] * w[1][b3] * w[2][c3];
        int64_t flat = slice_base + (iz[c3] * sy + iy[b3]) * sx + ix[a3];
        for (int c = 0; c < 3; ++c) v[c] += wt * node_value(b, flat, c);
      }
  return 1;
}

/* sample(): returns 1 and the field value at (x, t) if defined, else 0. */
int orc_sample(const orc_block* b, const double x[3], double t, double v[3]) {
  if (b->field_kind == ORC_FIELD_ABC) {
    double A = b->abc[0], B = b->abc[1], C = b->abc[2];
    v[0] = A * sin(x[2]) + C * cos(x[1]);
    v[1] = B * sin(x[0]) + A * cos(x[2]);
    v[2] = C * sin(x[1]) + B * cos(x[0]);
    return 1;
  }
  int64_t ix[2], iy[2], iz[2];
  double f[3];
  if (!axis_locate(b, 0, x[0], &ix[0], &ix[1], &f[0])) return 0;
  if (!axis_locate(b, 1, x[1], &iy[0], &iy[1], &f[1])) return 0;
  if (!axis_locate(b, 2, x[2], &iz[0], &iz[1], &f[2])) return 0;
  double w[3][2];
  for (int a = 0; a < 3; ++a) {
    w[a][0] = 1.0 - f[a];
    w[a][1] = f[a];
  }
  if (b->n_slices <= 1) return sample_slice(b, 0, ix, iy, iz, w, v);
  /* linear blend between the two slices that bracket t (clamped at the ends) */
  double u = (t - b->t0) / b->slice_dt;
  double s = floor(u);
  if (s < 0) s = 0;
  if (s > b->n_slices - 2) s = b->n_slices - 2;
  double al = u - s;
  if (al < 0) al = 0;
  if (al > 1) al = 1;
  double v0[3], v1[3];
  sample_slice(b, (int)s, ix, iy, iz, w, v0);
  sample_slice(b, (int)s + 1, ix, iy, iz, w, v1);
  for (int c = 0; c < 3; ++c) v[c] = (1.0 - al) * v0[c] + al * v1[c];
  return 1;
}

/* destinationID(): flat id of the macrocell containing x, -1 outside the grid. */
int32_t orc_dest(const orc_block* b, const double x[3]) {
  int64_t r[3];
  for (int a = 0; a < 3; ++a) {
    double q = floor((x[a] - b->lo[a]) / (b->hi[a] - b->lo[a]));
    if (!isfinite(q)) return -1;
    r[a] = (int64_t)b->rank_coord[a] + (int64_t)q;
    if (r[a] < 0 || r[a] >= b->rank_grid[a]) return -1;
  }
  return (int32_t)(r[0] + (int64_t)b->rank_grid[0] * (r[1] + (int64_t)b->rank_grid[1] * r[2]));
}

static int inside_owned(const orc_block* b, const double x[3]) {
  for (int a = 0; a < 3; ++a)
    if (!(x[a] >= b->lo[a] && x[a] < b->hi[a])) return 0;
  return 1;
}

static int finite3(const double v[3]) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

/* One RK4 update from (p0, t).  Returns ORC_ACTIVE when the step was taken
 * (p1 set), or the termination code; for ORC_HALO_MISS, fail_pt is the stage
 * point whose sample was undefined.  max-steps is the caller's test. */
int orc_rk4_step(const orc_block* b, const double p0[3], double t, double h, double eps,
                 double p1[3], double fail_pt[3]) {
  double k1[3], k2[3], k3[3], k4[3], q[3];
  if (!orc_sample(b, p0, t, k1)) {
    memcpy(fail_pt, p0, sizeof(double) * 3);
    return ORC_HALO_MISS;
  }
  if (!finite3(k1)) return ORC_NONFINITE;
  if (sqrt(k1[0] * k1[0] + k1[1] * k1[1] + k1[2] * k1[2]) < eps) return ORC_STAGNANT;
  for (int c = 0; c < 3; ++c) q[c] = p0[c] + 0.5 * h * k1[c];
  if (!orc_sample(b, q, t + 0.5 * h, k2)) {
    memcpy(fail_pt, q, sizeof(double) * 3);
    return ORC_HALO_MISS;
  }
  if (!finite3(k2)) return ORC_NONFINITE;
  for (int c = 0; c < 3; ++c) q[c] = p0[c] + 0.5 * h * k2[c];
  if (!orc_sample(b, q, t + 0.5 * h, k3)) {
    memcpy(fail_pt, q, sizeof(double) * 3);
    return ORC_HALO_MISS;
  }
  if (!finite3(k3)) return ORC_NONFINITE;
  for (int c = 0; c < 3; ++c) q[c] = p0[c] + h * k3[c];
  if (!orc_sample(b, q, t + h, k4)) {
    memcpy(fail_pt, q, sizeof(double) * 3);
    return ORC_HALO_MISS;
  }
  if (!finite3(k4)) return ORC_NONFINITE;
  for (int c = 0; c < 3; ++c) p1[c] = p0[c] + (h / 6.0) * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
  if (!finite3(p1)) return ORC_NONFINITE;
  return ORC_ACTIVE;
}

/* Batch of independent single steps (used for the per-vertex local check).
 * status[i] = ORC_ACTIVE when p1[i] holds the stepped position. */
void orc_step_batch(const orc_block* b, int64_t n, const double* p0, const double* t, double h,
                    double eps, double* p1, int32_t* status) {
  for (int64_t i = 0; i < n; ++i) {
    double fp[3];
    status[i] = orc_rk4_step(b, p0 + 3 * i, t ? t[i] : 0.0, h, eps, p1 + 3 * i, fp);
  }
}

/* ---------------- whole trajectories ---------------- */
typedef struct {
  /* inputs */
  const double* seeds;     /* [n][3] */
  const int32_t* max_steps;/* [n] */
  const double* t_birth;   /* [n] or NULL (0) */
  /* outputs */
  int32_t* steps;          /* [n] steps taken */
  int32_t* code;           /* [n] termination code (ORC_ACTIVE never: trace runs to the end) */
  double* final_pos;       /* [n][3] last position held by the particle */
  int64_t* n_verts;        /* [n] recorded vertices */
  double* verts;           /* [n][cap][3] or NULL */
  int8_t* in_outbox;       /* [n] 1 if the particle left through the outbox */
  double* out_pos;         /* [n][3] outbox position */
  int32_t* out_dest;       /* [n] outbox destination */
} orc_trace_io;

typedef struct {
  const orc_block* b;
  const orc_trace_io* io;
  double h, eps;
  int64_t cap, stride, begin, end;
} trace_job;

static void record(const trace_job* J, int64_t p, const double x[3], int64_t* nv) {
  if (J->io->verts && *nv < J->cap) memcpy(J->io->verts + (p * J->cap + *nv) * 3, x, 24);
  ++*nv;
}

static void trace_one(const trace_job* J, int64_t p) {
  const orc_block* b = J->b;
  const orc_trace_io* io = J->io;
  double P[3], P1[3], fp[3];
  memcpy(P, io->seeds + 3 * p, 24);
  double tb = io->t_birth ? io->t_birth[p] : 0.0;
  int32_t m = io->max_steps[p];
  int32_t n = 0;
  int64_t nv = 0;
  int code = ORC_ACTIVE;
  io->in_outbox[p] = 0;
  io->out_dest[p] = -1;
  record(J, p, P, &nv);
  if (!b->periodic && !inside_owned(b, P)) {
    code = ORC_EXIT;
    io->in_outbox[p] = 1;
    memcpy(io->out_pos + 3 * p, P, 24);
    io->out_dest[p] = orc_dest(b, P);
  }
  while (code == ORC_ACTIVE) {
    if (n >= m) {
      code = ORC_MAX_STEPS;
      break;
    }
    int st = orc_rk4_step(b, P, tb + (double)n * J->h, J->h, J->eps, P1, fp);
    if (st == ORC_HALO_MISS) {
      code = st;
      io->in_outbox[p] = 1;
      memcpy(io->out_pos + 3 * p, P, 24);
      io->out_dest[p] = orc_dest(b, fp);
      break;
    }
    if (st != ORC_ACTIVE) {
      code = st;
      break;
    }
    memcpy(P, P1, 24);
    ++n;
    int final = (!b->periodic && !inside_owned(b, P));
    if (final || n == m || (n % J->stride) == 0) record(J, p, P, &nv);
    if (final) {
      code = ORC_EXIT;
      io->in_outbox[p] = 1;
      memcpy(io->out_pos + 3 * p, P, 24);
      io->out_dest[p] = orc_dest(b, P);
    }
  }
  /* the final vertex is always recorded; stagnation, non-finite values and a
   * halo miss stop at a vertex that the stride rule may have skipped */
  if ((code == ORC_STAGNANT || code == ORC_NONFINITE || code == ORC_HALO_MISS) && n % J->stride != 0)
    record(J, p, P, &nv);
  io->steps[p] = n;
  io->code[p] = code;
  memcpy(io->final_pos + 3 * p, P, 24);
  io->n_verts[p] = nv;
}

static void* trace_worker(void* arg) {
  trace_job* J = (trace_job*)arg;
  for (int64_t p = J->begin; p < J->end; ++p) trace_one(J, p);
  return NULL;
}

/* Trace n particles to termination.  Vertex j (seed = 0) of a particle is
 * recorded when j is a multiple of `stride`, and the final vertex always;
 * at most `cap` vertices are stored per particle (n_verts reports all). */
void orc_trace(const orc_block* b, int64_t n, const orc_trace_io* io, double h, double eps,
               int64_t cap, int64_t stride, int n_threads) {
  if (stride < 1) stride = 1;
  if (n_threads < 1) n_threads = 1;
  if (n_threads > n) n_threads = n > 0 ? (int)n : 1;
  trace_job* jobs = (trace_job*)calloc((size_t)n_threads, sizeof(trace_job));
  pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
  for (int t = 0; t < n_threads; ++t) {
    jobs[t].b = b; jobs[t].io = io; jobs[t].h = h; jobs[t].eps = eps;
    jobs[t].cap = cap; jobs[t].stride = stride;
    jobs[t].begin = n * t / n_threads;
    jobs[t].end = n * (t + 1) / n_threads;
    if (n_threads == 1) trace_worker(&jobs[t]);
    else pthread_create(&th[t], NULL, trace_worker, &jobs[t]);
  }
  if (n_threads > 1)
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  free(jobs);
  free(th);
}

/* Batched sample() for tests: defined[i] = 1 when v[i] is set. */
void orc_sample_batch(const orc_block* b, int64_t n, const double* x, const double* t, double* v,
                      int32_t* defined) {
  for (int64_t i = 0; i < n; ++i) defined[i] = orc_sample(b, x + 3 * i, t ? t[i] : 0.0, v + 3 * i);
}

void orc_dest_batch(const orc_block* b, int64_t n, const double* x, int32_t* dest) {
  for (int64_t i = 0; i < n; ++i) dest[i] = orc_dest(b, x + 3 * i);
}

int32_t orc_sizeof_block(void) { return (int32_t)sizeof(orc_block); }
int32_t orc_sizeof_io(void) { return (int32_t)sizeof(orc_trace_io); }
