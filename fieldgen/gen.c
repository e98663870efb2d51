/*
 * Seeded synthetic inputs for the field-line workloads: vector fields sampled
 * at grid nodes, seed point sets, and round-to-nearest-even quantisation of
 * FP64 node values to the storage formats (FP32, FP16, BF16).
 *
 * This module produces INPUTS only.  It contains no part of the advection
 * method (no interpolation, no integration, no termination logic): both the
 * FP64 oracle and the GPU library read the bytes it writes.
 *
 * Random numbers come from a counter-based SplitMix64 (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014): value i of
 * stream s is the SplitMix64 finaliser applied to s + (i+1)*0x9E3779B97F4A7C15.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Stream key from (config, purpose, sub-index). */
uint64_t fg_stream(uint64_t config, uint64_t purpose, uint64_t sub) {
  return mix64(mix64(mix64(config * GOLDEN + 1) ^ (purpose * GOLDEN + 2)) ^ (sub * GOLDEN + 3));
}

uint64_t fg_u64(uint64_t stream, uint64_t i) { return mix64(stream + (i + 1) * GOLDEN); }

/* Uniform double in [0,1) with 53 random bits. */
double fg_unif(uint64_t stream, uint64_t i) { return (double)(fg_u64(stream, i) >> 11) * 0x1.0p-53; }

/* Fill out[n] with uniform doubles in [0,1). */
void fg_unif_fill(uint64_t stream, uint64_t first, int64_t n, double* out) {
  for (int64_t k = 0; k < n; ++k) out[k] = fg_unif(stream, first + (uint64_t)k);
}

/* Uniform FP32-exact values in [0,1): 24 random bits scaled by 2^-24. */
void fg_unif24_fill(uint64_t stream, uint64_t first, int64_t n, double* out) {
  for (int64_t k = 0; k < n; ++k) out[k] = (double)(fg_u64(stream, first + (uint64_t)k) >> 40) * 0x1.0p-24;
}

/* Standard normal pair by Box-Muller from counters 2i, 2i+1. */
void fg_normal_fill(uint64_t stream, uint64_t first, int64_t n, double* out) {
  for (int64_t k = 0; k < n; ++k) {
    uint64_t i = first + (uint64_t)k;
    double u1 = ((double)(fg_u64(stream, 2 * i) >> 11) + 1.0) * 0x1.0p-53; /* (0,1] */
    double u2 = fg_unif(stream, 2 * i + 1);
    out[k] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  }
}

/* ---------------------------------------------------------------------------
 * Round-to-nearest-even of a double into a binary format with `mant` stored
 * fraction bits, minimum normal exponent `emin` and maximum exponent `emax`.
 * Subnormals keep the spacing 2^(emin-mant); overflow gives +-inf.
 * ------------------------------------------------------------------------- */
static double rne_format(double d, int mant, int emin, int emax) {
  if (!isfinite(d) || d == 0.0) return d;
  int e;
  frexp(fabs(d), &e); /* |d| in [2^(e-1), 2^e) */
  int ex = e - 1;
  if (ex < emin) ex = emin;
  double ulp = ldexp(1.0, ex - mant);
  double q = nearbyint(d / ulp) * ulp; /* d/ulp and the product are exact */
  double maxv = ldexp(2.0 - ldexp(1.0, -mant), emax);
  if (fabs(q) > maxv) return d > 0 ? INFINITY : -INFINITY;
  return q;
}

double fg_round_f32(double d) { return (double)(float)d; }
double fg_round_f16(double d) { return rne_format(d, 10, -14, 15); }
double fg_round_bf16(double d) { return rne_format(d, 7, -126, 127); }

static uint16_t f16_bits(double q) { /* q already representable in binary16 */
  uint16_t s = signbit(q) ? 0x8000 : 0;
  double a = fabs(q);
  if (isinf(a)) return s | 0x7C00;
  if (isnan(a)) return 0x7E00;
  if (a == 0.0) return s;
  int e;
  double m = frexp(a, &e); /* a = m 2^e, m in [0.5,1) */
  int ex = e - 1;
  if (ex < -14) return s | (uint16_t)(a * 0x1.0p24); /* subnormal: a / 2^-24 */
  uint16_t frac = (uint16_t)((m * 2.0 - 1.0) * 1024.0);
  return s | (uint16_t)((ex + 15) << 10) | frac;
}

/* Quantise n doubles. fmt: 0 = FP32 (out is float*), 1 = FP16 bits, 2 = BF16 bits. */
void fg_quantize(const double* in, int64_t n, int fmt, void* out) {
  if (fmt == 0) {
    float* o = (float*)out;
    for (int64_t i = 0; i < n; ++i) o[i] = (float)in[i];
  } else if (fmt == 1) {
    uint16_t* o = (uint16_t*)out;
    for (int64_t i = 0; i < n; ++i) o[i] = f16_bits(fg_round_f16(in[i]));
  } else {
    uint16_t* o = (uint16_t*)out;
    for (int64_t i = 0; i < n; ++i) {
      double q = fg_round_bf16(in[i]);
      float f = (float)q; /* exact */
      uint32_t b;
      memcpy(&b, &f, 4);
      if (isnan(q)) b = 0x7FC00000u;
      o[i] = (uint16_t)(b >> 16);
    }
  }
}

/* ---------------------------------------------------------------------------
 * Random Fourier-mode turbulence:  v(x) = sum_m a_m e_m cos(kappa_m (u_m . x) + phi_m)
 * with |k_m| ~ U[kmin,kmax], u_m uniform on the sphere, e_m a unit vector
 * perpendicular to u_m (so div v = 0 exactly), a_m = |k_m|^(-5/6) (energy per
 * mode ~ k^(-5/3)), phi_m ~ U[0,2pi), kappa_m = 2 pi |k_m| / L.
 * Optional linear phase drift per time slice: phi_m(s) = phi_m + 2 pi r_m s / (S-1).
 * ------------------------------------------------------------------------- */
void fg_turb_modes(uint64_t stream, int n_modes, double kmin, double kmax, double L,
                   double* kappa, double* u /*3n*/, double* e /*3n*/, double* amp, double* phi,
                   double* drift) {
  for (int m = 0; m < n_modes; ++m) {
    uint64_t b = (uint64_t)m * 8;
    double kk = kmin + (kmax - kmin) * fg_unif(stream, b + 0);
    double cz = 2.0 * fg_unif(stream, b + 1) - 1.0;
    double az = 2.0 * M_PI * fg_unif(stream, b + 2);
    double sz = sqrt(fmax(0.0, 1.0 - cz * cz));
    double ux = sz * cos(az), uy = sz * sin(az), uz = cz;
    /* orthonormal e1, e2 perpendicular to u */
    double ax = fabs(ux) < 0.9 ? 1.0 : 0.0, ay = ax == 1.0 ? 0.0 : 1.0, a3 = 0.0;
    double e1x = ay * uz - a3 * uy, e1y = a3 * ux - ax * uz, e1z = ax * uy - ay * ux;
    double n1 = sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
    e1x /= n1; e1y /= n1; e1z /= n1;
    double e2x = uy * e1z - uz * e1y, e2y = uz * e1x - ux * e1z, e2z = ux * e1y - uy * e1x;
    double psi = 2.0 * M_PI * fg_unif(stream, b + 3);
    kappa[m] = 2.0 * M_PI * kk / L;
    u[3 * m + 0] = ux; u[3 * m + 1] = uy; u[3 * m + 2] = uz;
    e[3 * m + 0] = cos(psi) * e1x + sin(psi) * e2x;
    e[3 * m + 1] = cos(psi) * e1y + sin(psi) * e2y;
    e[3 * m + 2] = cos(psi) * e1z + sin(psi) * e2z;
    amp[m] = pow(kk, -5.0 / 6.0);
    phi[m] = 2.0 * M_PI * fg_unif(stream, b + 4);
    drift[m] = fg_unif(stream, b + 5);
  }
}

typedef struct {
  int n_modes;
  const double *kappa, *u, *e, *amp, *phi;
  int nx, ny, nz;            /* stored nodes per axis */
  double x0, y0, z0, dx;     /* world position of stored node 0 and spacing */
  double* out;               /* [nz][ny][nx][3] */
  int z_begin, z_end;
  double max_sq;
} turb_job;

static void* turb_worker(void* arg) {
  turb_job* J = (turb_job*)arg;
  int M = J->n_modes, nx = J->nx, ny = J->ny;
  double* pxr = (double*)malloc(sizeof(double) * (size_t)nx * M);
  double* pxi = (double*)malloc(sizeof(double) * (size_t)nx * M);
  double* pyr = (double*)malloc(sizeof(double) * (size_t)ny * M);
  double* pyi = (double*)malloc(sizeof(double) * (size_t)ny * M);
  double* qr = (double*)malloc(sizeof(double) * M);
  double* qi = (double*)malloc(sizeof(double) * M);
  double* ae = (double*)malloc(sizeof(double) * 3 * M);
  for (int m = 0; m < M; ++m)
    for (int c = 0; c < 3; ++c) ae[3 * m + c] = J->amp[m] * J->e[3 * m + c];
  /* x phasors carry the mode phase: exp(i (kappa ux x + phi)) */
  for (int i = 0; i < nx; ++i)
    for (int m = 0; m < M; ++m) {
      double a = J->kappa[m] * J->u[3 * m] * (J->x0 + i * J->dx) + J->phi[m];
      pxr[(size_t)i * M + m] = cos(a);
      pxi[(size_t)i * M + m] = sin(a);
    }
  for (int j = 0; j < ny; ++j)
    for (int m = 0; m < M; ++m) {
      double a = J->kappa[m] * J->u[3 * m + 1] * (J->y0 + j * J->dx);
      pyr[(size_t)j * M + m] = cos(a);
      pyi[(size_t)j * M + m] = sin(a);
    }
  double mx = 0.0;
  for (int k = J->z_begin; k < J->z_end; ++k) {
    double zr[1024], zi[1024];
    for (int m = 0; m < M; ++m) {
      double a = J->kappa[m] * J->u[3 * m + 2] * (J->z0 + k * J->dx);
      zr[m] = cos(a);
      zi[m] = sin(a);
    }
    for (int j = 0; j < ny; ++j) {
      for (int m = 0; m < M; ++m) {
        double ar = pyr[(size_t)j * M + m], ai = pyi[(size_t)j * M + m];
        qr[m] = ar * zr[m] - ai * zi[m];
        qi[m] = ar * zi[m] + ai * zr[m];
      }
      double* row = J->out + (((size_t)k * ny + j) * nx) * 3;
      for (int i = 0; i < nx; ++i) {
        const double* xr = pxr + (size_t)i * M;
        const double* xi = pxi + (size_t)i * M;
        double vx = 0, vy = 0, vz = 0;
        for (int m = 0; m < M; ++m) {
          double c = xr[m] * qr[m] - xi[m] * qi[m];
          vx += ae[3 * m] * c;
          vy += ae[3 * m + 1] * c;
          vz += ae[3 * m + 2] * c;
        }
        row[3 * i] = vx; row[3 * i + 1] = vy; row[3 * i + 2] = vz;
        double s = vx * vx + vy * vy + vz * vz;
        if (s > mx) mx = s;
      }
    }
  }
  J->max_sq = mx;
  free(pxr); free(pxi); free(pyr); free(pyi); free(qr); free(qi); free(ae);
  return NULL;
}

/* Evaluate the mode sum on a stored grid; phases phi (already drifted by the
 * caller when needed). Returns max |v| over the nodes (before any scaling). */
double fg_turb_eval(int n_modes, const double* kappa, const double* u, const double* e,
                    const double* amp, const double* phi, int nx, int ny, int nz, double x0,
                    double y0, double z0, double dx, double* out, int n_threads) {
  if (n_modes > 1024) return -1.0;
  if (n_threads < 1) n_threads = 1;
  if (n_threads > nz) n_threads = nz;
  turb_job* jobs = (turb_job*)calloc((size_t)n_threads, sizeof(turb_job));
  pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
  for (int t = 0; t < n_threads; ++t) {
    turb_job* J = &jobs[t];
    J->n_modes = n_modes; J->kappa = kappa; J->u = u; J->e = e; J->amp = amp; J->phi = phi;
    J->nx = nx; J->ny = ny; J->nz = nz; J->x0 = x0; J->y0 = y0; J->z0 = z0; J->dx = dx;
    J->out = out;
    J->z_begin = (int)((int64_t)nz * t / n_threads);
    J->z_end = (int)((int64_t)nz * (t + 1) / n_threads);
    pthread_create(&th[t], NULL, turb_worker, J);
  }
  double mx = 0.0;
  for (int t = 0; t < n_threads; ++t) {
    pthread_join(th[t], NULL);
    if (jobs[t].max_sq > mx) mx = jobs[t].max_sq;
  }
  free(jobs); free(th);
  return sqrt(mx);
}
