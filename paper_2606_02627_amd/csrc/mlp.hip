// Learned flow-map surrogate: a 3 -> 256 -> 256 -> 256 -> 256 -> 3 MLP with
// SiLU activations, BF16 weights and activations as MFMA operands and FP32
// accumulation (gfx950 v_mfma_f32_32x32x16_bf16), trained on the GPU with
// its own forward/backward GEMMs and an Adam kernel (FP32 master weights).
//
// Network (FP32 master parameters, l = 0..4):
//   xhat = 2 (x mod L)/L - 1;  h0 = xhat;  z_l = W_l h_l + b_l;
//   h_{l+1} = SiLU(z_l) (l < 4);  out = sigma * z_4.
// Loss: mean of ((out - target)/sigma)^2 over samples and components.
//
// Layouts (row-major, padded with zeros so every GEMM dimension is a multiple
// of 16 along K and 32 along M/N): layer l has in_pad = 16 (l = 0) or 256 and
// out_pad = 256 or 32 (l = 4).  Activations are kept in BF16 both row-major
// [B x in_pad] (forward A operand) and transposed [in_pad x B] (weight-gradient
// B operand), so that every MFMA fragment is a contiguous 16-byte load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>
#include <utility>

#include "../../include/streami.h"

namespace streami {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int NL = 5;
constexpr int WID[NL + 1] = {3, 256, 256, 256, 256, 3};
constexpr int IN_PAD[NL] = {16, 256, 256, 256, 256};
constexpr int OUT_PAD[NL] = {256, 256, 256, 256, 32};

__host__ __device__ inline int n_params_total() {
  int s = 0;
  for (int l = 0; l < NL; ++l) s += WID[l] * WID[l + 1] + WID[l + 1];
  return s;
}

__device__ __forceinline__ unsigned short f2bf(float f) {  // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C[M x N] (FP32, ldc) = A[M x K] . B[K x N], BF16 operands with K contiguous:
//   A(i, k) = A[i*lda + k],  B(k, j) = B[j*ldb + k].
// One wave per 32x32 tile; rows/cols beyond M/N read as zero and are not
// stored; K is a multiple of 16.  MFMA operand layout (32x32x16): lane l holds
// row/col (l % 32) and k = 8*(l/32) .. +7; the accumulator register r of lane l
// holds row 8*(r/4) + 4*(l/32) + r%4 and column l % 32.
__global__ void __launch_bounds__(256) k_gemm_bf16(const unsigned short* __restrict__ A, int lda,
                                                   const unsigned short* __restrict__ B, int ldb, float* C, int ldc,
                                                   int M, int N, int K, int accumulate) {
  const int lane = __lane_id();
  const int wave = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int tiles_n = (N + 31) / 32;
  const int tm = wave / tiles_n, tn = wave % tiles_n;
  if (tm * 32 >= M) return;
  const int i = tm * 32 + (lane & 31), j = tn * 32 + (lane & 31);
  const int kh = 8 * (lane >> 5);
  const bool ai = i < M, bj = j < N;
  f32x16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  const bf16x8 zero = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x8 a = ai ? *reinterpret_cast<const bf16x8*>(A + (size_t)i * lda + k0 + kh) : zero;
    const bf16x8 b = bj ? *reinterpret_cast<const bf16x8*>(B + (size_t)j * ldb + k0 + kh) : zero;
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const int col = tn * 32 + (lane & 31);
  if (col >= N) return;
  for (int r = 0; r < 16; ++r) {
    const int row = tm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row < M) {
      float* c = C + (size_t)row * ldc + col;
      *c = accumulate ? *c + acc[r] : acc[r];
    }
  }
}

static void gemm(const unsigned short* A, int lda, const unsigned short* B, int ldb, float* C, int ldc, int M, int N,
                 int K, bool accumulate, hipStream_t st) {
  const long long tiles = (long long)((M + 31) / 32) * ((N + 31) / 32);
  const int grid = (int)((tiles + 3) / 4);
  hipLaunchKernelGGL(k_gemm_bf16, dim3(grid), dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, accumulate ? 1 : 0);
}

// xhat = 2 (x mod L)/L - 1 in columns 0..2 of a [B x 16] BF16 row (zeros
// elsewhere; rows >= n are zero) and its transpose [16 x Bp].
__global__ void k_mlp_input(const float* xyz, int xstride, long long n, long long Bp, float period,
                            unsigned short* H, unsigned short* HT) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < Bp; r += (long long)gridDim.x * blockDim.x) {
    for (int c = 0; c < 16; ++c) {
      float v = 0.0f;
      if (r < n && c < 3) {
        const float x = xyz[r * xstride + c];
        const float w = x - period * floorf(x / period);
        v = 2.0f * (w / period) - 1.0f;
      }
      const unsigned short b = f2bf(v);
      H[r * 16 + c] = b;
      HT[(long long)c * Bp + r] = b;
    }
  }
}

// z += b (FP32, in place); h = BF16(SiLU(z)) row-major and transposed.
__global__ void k_bias_silu(float* Z, const float* bias, long long Bp, int width, unsigned short* H,
                            unsigned short* HT) {
  const long long total = Bp * width;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / width;
    const int c = (int)(e - r * width);
    const float z = Z[e] + bias[c];
    Z[e] = z;
    const unsigned short b = f2bf(silu(z));
    H[e] = b;
    HT[(long long)c * Bp + r] = b;
  }
}

// Output layer: out = sigma * (z + b) for the first n rows; loss terms and
// dL/dz (BF16, row-major [Bp x 32] and transposed [32 x Bp]).
__global__ void k_out_loss(const float* Z, const float* bias, long long n, long long Bp, float sx, float sy, float sz,
                           const float* target, float* out, unsigned short* dZ, unsigned short* dZT, float* loss_acc,
                           float inv_count) {
  const float sig[3] = {sx, sy, sz};
  float part = 0.0f;
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < Bp; r += (long long)gridDim.x * blockDim.x) {
    for (int c = 0; c < 32; ++c) {
      float g = 0.0f;
      if (r < n && c < 3) {
        const float o = sig[c] * (Z[r * 32 + c] + bias[c]);
        if (out) out[r * 3 + c] = o;
        if (target) {
          const float d = (o - target[r * 3 + c]) / sig[c];
          part += d * d;
          g = 2.0f * d * inv_count;  // dL/dz = dL/dout * sigma = 2 d / count
        }
      }
      if (dZ) {
        const unsigned short b = f2bf(g);
        dZ[r * 32 + c] = b;
        dZT[(long long)c * Bp + r] = b;
      }
    }
  }
  if (loss_acc) {
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if (__lane_id() == 0) atomicAdd(loss_acc, part);
  }
}

// dZ = dH * SiLU'(Z) -> BF16 row-major and transposed.
__global__ void k_silu_grad(const float* dH, const float* Z, long long Bp, int width, unsigned short* dZ,
                            unsigned short* dZT) {
  const long long total = Bp * width;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / width;
    const int c = (int)(e - r * width);
    const unsigned short b = f2bf(dH[e] * dsilu(Z[e]));
    dZ[e] = b;
    dZT[(long long)c * Bp + r] = b;
  }
}

// db[c] = sum over rows of dZ[r][c] (dZ^T rows are contiguous).
__global__ void k_rowsum_bf16(const unsigned short* dZT, long long Bp, int width, float* db) {
  const int c = blockIdx.x;
  if (c >= width) return;
  float s = 0.0f;
  for (long long r = threadIdx.x; r < Bp; r += blockDim.x) s += bf2f(dZT[(long long)c * Bp + r]);
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] = red[0];
}

// Adam on FP32 master parameters; gradients of W come padded [out_pad x in_pad].
__global__ void k_adam(float* p, float* m, float* v, const float* g, int rows, int cols, int g_ld, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const long long total = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / cols;
    const int c = (int)(e - r * cols);
    const float gr = g[r * g_ld + c];
    const float mm = b1 * m[e] + (1.0f - b1) * gr;
    const float vv = b2 * v[e] + (1.0f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// BF16 copies of W_l: [out_pad x in_pad] and transposed [in_pad x out_pad].
__global__ void k_refresh_w(const float* W, int out, int in, int out_pad, int in_pad, unsigned short* Wb,
                            unsigned short* WTb) {
  const long long total = (long long)out_pad * in_pad;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / in_pad), c = (int)(e - (long long)r * in_pad);
    const unsigned short b = (r < out && c < in) ? f2bf(W[(long long)r * in + c]) : (unsigned short)0;
    Wb[e] = b;
    WTb[(long long)c * out_pad + r] = b;
  }
}

// ---------------------------------------------------------------- fused inference
// MFMA fragment order of the weights, built from the FP32 masters whenever
// they change: layer l, output tile t (32 rows), k-step s, lane L, slot j
// (8 BF16 = 16 bytes per lane) holds W_l[32 t + L % 32][kmap(l, s, L / 32, j)]:
//   kmap(0, 0, hi, j) = 8 hi + j                    (the padded 3-vector input)
//   kmap(l, s, hi, j) = 32 (s/2) + 16 (s%2) + 8 (j/4) + 4 hi + j%4   (l >= 1).
// The second line is the order in which a layer's accumulators sit in a lane:
// register r = 8q + j of output tile t holds feature 32t + 8(r/4) + 4hi + r%4
// of the lane's particle, which is slot j of k-step 2t + q.  With the input
// dimension of every later layer permuted the same way, a layer's outputs are
// the next layer's B operand in place, with no exchange between lanes.
constexpr int FR_TILES[NL] = {8, 8, 8, 8, 1};
constexpr int FR_KSTEPS[NL] = {1, 16, 16, 16, 16};
constexpr int FR_OFF[NL + 1] = {0, 512, 8704, 16896, 25088, 26112};  // 16-byte units

__host__ __device__ constexpr int frag_k(int l, int s, int hi, int j) {
  return l == 0 ? 8 * hi + j : 32 * (s / 2) + 16 * (s % 2) + 8 * (j / 4) + 4 * hi + j % 4;
}

struct FragArgs {
  const float* W[NL];
};

__global__ void k_frag_w(FragArgs a, unsigned short* frag) {
  const int total = FR_OFF[NL] * 8;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int u = e >> 3, j = e & 7;
    int l = 0;
    while (u >= FR_OFF[l + 1]) ++l;
    const int r = u - FR_OFF[l];
    const int L = r & 63, ts = r >> 6, s = ts % FR_KSTEPS[l], t = ts / FR_KSTEPS[l];
    const int row = 32 * t + (L & 31), k = frag_k(l, s, L >> 5, j);
    frag[e] = (row < WID[l + 1] && k < WID[l]) ? f2bf(a.W[l][row * WID[l] + k]) : (unsigned short)0;
  }
}

typedef __attribute__((__vector_size__(8 * sizeof(float)))) float f32x8;

__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

struct InferArgs {
  const uint4* frag;
  const float* b[NL];
  const float* xyz;
  int xstride;
  long long n;
  float period;
  float sigma[3];
  float* out;
};

// One workgroup = 4 waves = 128 particles; each wave keeps its 32 particles'
// activations in registers as the B operand, and the network runs as a
// software pipeline of 17 compute steps:
//   layer 0 in 4 quarters (output tiles 2q, 2q+1; one k-step each),
//   layers 1..3 in 4 quarters each (2 tiles x 16 k-steps),
//   layer 4 in one step (1 tile x 16 k-steps).
// The weight fragments come through LDS in 14 stages (layer 0 whole, the 12
// hidden quarters, layer 4; at most 32 KB each) and two buffers: a stage is
// copied by direct global-to-LDS loads, which hold no registers, while the
// previous stage computes.  The SiLU epilogue of a step runs between the MFMAs
// of the next one (two accumulator sets), so the matrix cores are not idle
// while the transcendentals execute.  A quarter's outputs are the next layer's
// k-steps 4q..4q+3; quarters 0..2 wait in registers until the layer's last
// quarter has read its input, quarter 3 is produced while the next layer's
// first step consumes k-steps 0..11.  Two workgroups share a CU (69 KB of LDS
// each).
constexpr int INFER_WAVES = 4;
constexpr int N_STEPS = 17, N_STAGES = 14, STAGE_UNITS = 2048;  // 16-byte units
__host__ __device__ constexpr int step_layer(int c) { return c < 4 ? 0 : c < 16 ? 1 + (c - 4) / 4 : 4; }
__host__ __device__ constexpr int step_quarter(int c) { return c < 4 ? c : c < 16 ? (c - 4) % 4 : 0; }
__host__ __device__ constexpr int step_tiles(int c) { return c < 16 ? 2 : 1; }
__host__ __device__ constexpr int step_stage(int c) { return c < 4 ? 0 : c - 3; }
__host__ __device__ constexpr bool step_opens(int c) { return c == 0 || c >= 4; }
// first fragment of step c within its stage (layer 0's quarters share one stage)
__host__ __device__ constexpr int step_base(int c) { return c < 4 ? 2 * c * 64 : 0; }
__host__ __device__ constexpr int stage_off(int d) {
  return d == 0 ? FR_OFF[0] : d < 13 ? FR_OFF[1 + (d - 1) / 4] + ((d - 1) % 4) * STAGE_UNITS : FR_OFF[4];
}
__host__ __device__ constexpr int stage_units(int d) {
  return d == 0 ? FR_OFF[1] - FR_OFF[0] : d < 13 ? STAGE_UNITS : FR_OFF[5] - FR_OFF[4];
}
static_assert(FR_OFF[1] - FR_OFF[0] <= STAGE_UNITS && FR_OFF[5] - FR_OFF[4] <= STAGE_UNITS, "stage size");
static_assert((FR_OFF[1] - FR_OFF[0]) % 256 == 0 && (FR_OFF[5] - FR_OFF[4]) % 256 == 0, "whole copies");
static_assert(FR_OFF[2] - FR_OFF[1] == 4 * STAGE_UNITS, "a hidden layer is four stages");
// the stages tile the fragment array in order, and every step reads only
// within its own stage: its tiles x k-steps x 64 lanes from its first fragment
__host__ __device__ constexpr bool stage_table_ok() {
  int end = 0;
  for (int d = 0; d < N_STAGES; ++d) {
    if (stage_off(d) != end || stage_units(d) > STAGE_UNITS) return false;
    end += stage_units(d);
  }
  if (end != FR_OFF[NL]) return false;
  for (int c = 0; c < N_STEPS; ++c) {
    const int l = step_layer(c), d = step_stage(c);
    const int first = FR_OFF[l] + 2 * step_quarter(c) * FR_KSTEPS[l] * 64;  // tile 2q of layer l
    if (first != stage_off(d) + step_base(c)) return false;
    if (step_base(c) + step_tiles(c) * FR_KSTEPS[l] * 64 > stage_units(d)) return false;
    if (c > 0 && step_stage(c) != step_stage(c - 1) + (step_opens(c) ? 1 : 0)) return false;
  }
  return true;
}
static_assert(stage_table_ok(), "stage table");

typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;

// Stage d into an LDS buffer: each lane copies 16 bytes per instruction, a
// wave 1 KB to consecutive LDS addresses (the LDS base is wave-uniform).
template <int D>
__device__ __forceinline__ void stage_copy(const uint4* frag, uint4* buf, int tid) {
  constexpr int off = stage_off(D), units = stage_units(D);
#pragma unroll
  for (int i = 0; i < units / 256; ++i)
    __builtin_amdgcn_global_load_lds(static_cast<const void*>(frag + off + i * 256 + tid),
                                     (__attribute__((address_space(3))) void*)(buf + i * 256 + (tid & ~63)),
                                     16, 0, 0);
}

template <int... I, class F>
__device__ __forceinline__ void for_steps(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}

__global__ void __launch_bounds__(64 * INFER_WAVES, 2) k_mlp_infer(InferArgs a) {
  // two distinct arrays, so that the compiler sees that a copy in flight writes
  // the other buffer and waits for it only at the barrier
  __shared__ uint4 w0[STAGE_UNITS];
  __shared__ uint4 w1[STAGE_UNITS];
  __shared__ float bl[NL][256];
  const int tid = threadIdx.x, lane = tid & 63, hi = lane >> 5;
  const long long p = (long long)blockIdx.x * (32 * INFER_WAVES) + (tid >> 6) * 32 + (lane & 31);
  const bool live = p < a.n;
  stage_copy<0>(a.frag, w0, tid);
  for (int i = tid; i < NL * 256; i += 64 * INFER_WAVES) {
    const int l = i >> 8, f = i & 255;
    bl[l][f] = f < WID[l + 1] ? a.b[l][f] : 0.0f;
  }
  bf16x8 B[16];
  {
    f32x8 x = {0, 0, 0, 0, 0, 0, 0, 0};
    if (live && hi == 0)
      for (int c = 0; c < 3; ++c) {
        const float v = a.xyz[p * a.xstride + c];
        const float w = v - a.period * floorf(v / a.period);
        x[c] = 2.0f * (w / a.period) - 1.0f;
      }
    B[0] = __builtin_convertvector(x, bf16x8);
    const bf16x8 zero = {};
#pragma unroll
    for (int s = 1; s < 16; ++s) B[s] = zero;  // layer 0 reads B[0] only
  }
  f32x16 acc[2][2];
  unsigned H[48];  // next layer's k-steps 0..11 (quarters 0..2), 4 words each
  unsigned Q[16];  // next layer's k-steps 12..15 (quarter 3)

  // SiLU of value pair e (0..15) of step C's accumulators into the words of
  // the next layer's input: pair e = 8 tt + j of tile tt is word j % 4 of
  // k-step 4 q + 2 tt + j / 4.
  auto epilogue_pair = [&](auto Cc, int e) {
    constexpr int C = decltype(Cc)::value;
    constexpr int q = step_quarter(C);
    const int tt = e >> 3, j = e & 7;
    f32x2 z = {silu_fast(acc[C % 2][tt][2 * j]), silu_fast(acc[C % 2][tt][2 * j + 1])};
    const unsigned w = __builtin_bit_cast(unsigned, __builtin_convertvector(z, bf16x2));
    const int ks = 2 * tt + (j >> 2), wd = j & 3;
    if (q < 3) H[(4 * q + ks) * 4 + wd] = w;
    else Q[ks * 4 + wd] = w;
  };

  for_steps(std::make_integer_sequence<int, N_STEPS>{}, [&](auto Cc) {
    constexpr int C = decltype(Cc)::value;
    constexpr int l = step_layer(C), q = step_quarter(C), tiles = step_tiles(C), ks = FR_KSTEPS[l];
    constexpr int d = step_stage(C);
    uint4* const buf = d % 2 ? w1 : w0;
    if constexpr (step_opens(C)) {
      __syncthreads();  // stage d has landed; every wave is done with the other buffer
      if constexpr (d + 1 < N_STAGES) stage_copy<(d + 1 < N_STAGES ? d + 1 : 0)>(a.frag, (d + 1) % 2 ? w1 : w0, tid);
    }
    if constexpr (C > 0 && step_layer(C - 1) != l) {
      // a new layer: its k-steps 0..11 are the previous layer's quarters 0..2
#pragma unroll
      for (int k = 0; k < 12; ++k)
        B[k] = __builtin_bit_cast(bf16x8, u32x4{H[4 * k], H[4 * k + 1], H[4 * k + 2], H[4 * k + 3]});
    }
    // the accumulators start at the bias of the feature each register holds
#pragma unroll
    for (int tt = 0; tt < tiles; ++tt)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[C % 2][tt][r] = bl[l][32 * (2 * q + tt) + 8 * (r / 4) + 4 * hi + r % 4];
#pragma unroll
    for (int k = 0; k < ks; ++k) {
      if constexpr (C > 0) {
        // the previous step's epilogue, spread over this step's k-steps
        constexpr int per = 16 / ks;
#pragma unroll
        for (int e = k * per; e < (k + 1) * per; ++e) epilogue_pair(std::integral_constant<int, C - 1>{}, e);
        // a new layer's k-step 12 + i is complete once pairs 4i..4i+3 are (at
        // k-step 4i + 3 <= 12 + i of this step)
        if constexpr (step_layer(C - 1) != l) {
          if (k >= 12) {
            const int i = k - 12;
            B[k] = __builtin_bit_cast(bf16x8, u32x4{Q[4 * i], Q[4 * i + 1], Q[4 * i + 2], Q[4 * i + 3]});
          }
        }
      }
#pragma unroll
      for (int tt = 0; tt < tiles; ++tt) {
        const uint4 w = buf[step_base(C) + (tt * ks + k) * 64 + lane];
        acc[C % 2][tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, w), B[k], acc[C % 2][tt], 0, 0, 0);
      }
      if (k % 4 == 3) __builtin_amdgcn_sched_barrier(0);  // bound how far fragment loads run ahead
    }
  });
  // layer 4 (step 16, accumulator set 0): the three outputs are features 0..2 of the hi = 0 lanes
  if (live && hi == 0)
    for (int c = 0; c < 3; ++c) a.out[p * 3 + c] = a.sigma[c] * acc[0][0][c];
}

static int grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace streami

using namespace streami;

namespace streami {
int set_error(int code, const char* msg);  // api.hip: the thread's last-error text
}
namespace {
int mfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return streami::set_error(code, buf);
}
#define MHIP(expr)                                                                                      \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return mfail(STREAMI_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)
}  // namespace

namespace streami {
// The per-batch buffers of one training step, for Bp padded rows.
struct Workspace {
  unsigned short* H[NL] = {};   // BF16 layer inputs [Bp x in_pad]
  unsigned short* HT[NL] = {};  // transposed [in_pad x Bp]
  float* Z[NL] = {};            // FP32 pre-activations [Bp x out_pad]
  unsigned short* dZ = nullptr;  // BF16 [Bp x 256]
  unsigned short* dZT = nullptr;
  float* dH = nullptr;           // FP32 [Bp x 256]
};
}  // namespace streami

struct streami_mlp_s {
  hipStream_t stream = nullptr;
  float sigma[3] = {1, 1, 1};
  float period = 1;
  // FP32 master parameters and Adam moments, per layer: W [out x in], b [out]
  float* W[NL] = {};
  float* b[NL] = {};
  float* mW[NL] = {};
  float* vW[NL] = {};
  float* mb[NL] = {};
  float* vb[NL] = {};
  unsigned short* Wb[NL] = {};   // BF16 [out_pad x in_pad]
  unsigned short* WTb[NL] = {};  // BF16 [in_pad x out_pad]
  float* gW[NL] = {};            // FP32 [out_pad x in_pad]
  float* gb[NL] = {};            // FP32 [out_pad]
  unsigned short* frag = nullptr;  // BF16 weights in MFMA fragment order (fused inference)
  long long t = 0;               // Adam step count
  // batch workspace of streami_mlp_train_step (grown on demand)
  long long cap = 0;
  streami::Workspace ws;
  float* loss = nullptr;
  std::vector<void*> owned;
};

namespace {

int dalloc(streami_mlp_s* m, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return mfail(STREAMI_E_NOMEM, "device allocation of %zu bytes failed", bytes);
  }
  m->owned.push_back(*p);
  return STREAMI_OK;
}

void free_batch(streami_mlp_s* m) {
  auto drop = [&](void* p) {
    if (!p) return;
    for (auto& q : m->owned)
      if (q == p) q = nullptr;
    (void)hipFree(p);
  };
  for (int l = 0; l < NL; ++l) {
    drop(m->ws.H[l]);
    drop(m->ws.HT[l]);
    drop(m->ws.Z[l]);
  }
  drop(m->ws.dZ);
  drop(m->ws.dZT);
  drop(m->ws.dH);
  m->ws = Workspace();
  m->cap = 0;
}

int ensure_batch(streami_mlp_s* m, long long Bp) {
  if (Bp <= m->cap) return STREAMI_OK;
  // the workspace may be in use by kernels on any stream (a field's advection
  // uses this network on its own stream): wait for the device before freeing
  MHIP(hipDeviceSynchronize());
  free_batch(m);
  int rc;
  for (int l = 0; l < NL; ++l) {
    if ((rc = dalloc(m, (void**)&m->ws.H[l], (size_t)Bp * IN_PAD[l] * 2)) ||
        (rc = dalloc(m, (void**)&m->ws.HT[l], (size_t)Bp * IN_PAD[l] * 2)) ||
        (rc = dalloc(m, (void**)&m->ws.Z[l], (size_t)Bp * OUT_PAD[l] * 4)))
      return rc;
  }
  if ((rc = dalloc(m, (void**)&m->ws.dZ, (size_t)Bp * 256 * 2)) ||
      (rc = dalloc(m, (void**)&m->ws.dZT, (size_t)Bp * 256 * 2)) || (rc = dalloc(m, (void**)&m->ws.dH, (size_t)Bp * 256 * 4)))
    return rc;
  m->cap = Bp;
  return STREAMI_OK;
}

void refresh_bf16(streami_mlp_s* m) {
  for (int l = 0; l < NL; ++l)
    hipLaunchKernelGGL(k_refresh_w, dim3(grid_for((long long)OUT_PAD[l] * IN_PAD[l])), dim3(256), 0, m->stream, m->W[l],
                       WID[l + 1], WID[l], OUT_PAD[l], IN_PAD[l], m->Wb[l], m->WTb[l]);
  FragArgs fa;
  for (int l = 0; l < NL; ++l) fa.W[l] = m->W[l];
  hipLaunchKernelGGL(k_frag_w, dim3(grid_for((long long)FR_OFF[NL] * 8)), dim3(256), 0, m->stream, fa, m->frag);
}

// Forward over Bp rows (n real); leaves Z/H for backprop; writes out (n x 3) if given.
void forward(streami_mlp_s* m, const Workspace& w, const float* xyz, int xstride, long long n, long long Bp,
             float* out, const float* target, bool want_grad, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_input, dim3(grid_for(Bp)), dim3(256), 0, st, xyz, xstride, n, Bp, m->period, w.H[0],
                     w.HT[0]);
  for (int l = 0; l < NL; ++l) {
    gemm(w.H[l], IN_PAD[l], m->Wb[l], IN_PAD[l], w.Z[l], OUT_PAD[l], (int)Bp, OUT_PAD[l], IN_PAD[l], false, st);
    if (l < NL - 1)
      hipLaunchKernelGGL(k_bias_silu, dim3(grid_for(Bp * OUT_PAD[l])), dim3(256), 0, st, w.Z[l], m->b[l], Bp,
                         OUT_PAD[l], w.H[l + 1], w.HT[l + 1]);
  }
  const float inv = n > 0 ? 1.0f / (float)(n * 3) : 0.0f;
  hipLaunchKernelGGL(k_out_loss, dim3(grid_for(Bp)), dim3(256), 0, st, w.Z[NL - 1], m->b[NL - 1], n, Bp, m->sigma[0],
                     m->sigma[1], m->sigma[2], target, out, want_grad ? w.dZ : nullptr, want_grad ? w.dZT : nullptr,
                     target ? m->loss : nullptr, inv);
}

// Backward from dZ of the output layer (already in w.dZ/dZT, width 32).
void backward(streami_mlp_s* m, const Workspace& w, long long Bp) {
  hipStream_t st = m->stream;
  for (int l = NL - 1; l >= 0; --l) {
    const int op = OUT_PAD[l], ip = IN_PAD[l];
    // dW_l [op x ip] = dZ^T [op x Bp] . H_l [Bp x ip]  (K = batch, contiguous in dZ^T and H^T)
    gemm(w.dZT, (int)Bp, w.HT[l], (int)Bp, m->gW[l], ip, op, ip, (int)Bp, false, st);
    hipLaunchKernelGGL(k_rowsum_bf16, dim3(op), dim3(256), 0, st, w.dZT, Bp, op, m->gb[l]);
    if (l > 0) {
      // dH_l [Bp x ip] = dZ [Bp x op] . W_l [op x ip]   (B(k=out, j=in) = W^T[in][out])
      gemm(w.dZ, op, m->WTb[l], op, w.dH, ip, (int)Bp, ip, op, false, st);
      hipLaunchKernelGGL(k_silu_grad, dim3(grid_for(Bp * ip)), dim3(256), 0, st, w.dH, w.Z[l - 1], Bp, ip, w.dZ,
                         w.dZT);
    }
  }
}

// Bytes of a workspace for Bp padded rows, each buffer starting on a 256-byte boundary.
constexpr size_t ws_align(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t workspace_bytes(long long Bp) {
  size_t s = 0;
  for (int l = 0; l < NL; ++l)
    s += 2 * ws_align((size_t)Bp * IN_PAD[l] * 2) + ws_align((size_t)Bp * OUT_PAD[l] * 4);
  return s + 2 * ws_align((size_t)Bp * 256 * 2) + ws_align((size_t)Bp * 256 * 4);
}

// A workspace for Bp padded rows carved out of `base` (workspace_bytes(Bp) bytes, 256-aligned).
Workspace carve_workspace(char* base, long long Bp) {
  Workspace w;
  auto take = [&](size_t b) {
    char* p = base;
    base += ws_align(b);
    return p;
  };
  for (int l = 0; l < NL; ++l) {
    w.H[l] = (unsigned short*)take((size_t)Bp * IN_PAD[l] * 2);
    w.HT[l] = (unsigned short*)take((size_t)Bp * IN_PAD[l] * 2);
    w.Z[l] = (float*)take((size_t)Bp * OUT_PAD[l] * 4);
  }
  w.dZ = (unsigned short*)take((size_t)Bp * 256 * 2);
  w.dZT = (unsigned short*)take((size_t)Bp * 256 * 2);
  w.dH = (float*)take((size_t)Bp * 256 * 4);
  return w;
}

// The allocation-free training step's workspace: one copy per device, held until the process
// ends, large enough for STREAMI_MLP_NOALLOC_MAX_BATCH rows.  Host code never passes this
// name to a kernel (on the host it is only a stand-in): it uses the device address
// hipGetSymbolAddress returns for the current device.
constexpr long long NOALLOC_ROWS = (STREAMI_MLP_NOALLOC_MAX_BATCH + 31) / 32 * 32;
static __device__ __align__(256) char scratch[workspace_bytes(NOALLOC_ROWS)];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

// The current device's copy of `scratch`, looked up once per device.
int scratch_for_current_device(char** out) {
  int dev = 0;
  MHIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return mfail(STREAMI_E_UNSUPPORTED, "device %d beyond the %d supported", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    MHIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return mfail(STREAMI_E_DEVICE, "no device address for the training workspace");
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return STREAMI_OK;
}

// One training step on workspace w (forward, backward, Adam, outputs): shared by both entry points.
int train_step_on(streami_mlp_s* m, const Workspace& w, const float* xyz, const float* target, long long batch,
                  long long Bp, float lr, float* loss_out, float* grads_out) {
  MHIP(hipMemsetAsync(m->loss, 0, 4, m->stream));
  forward(m, w, xyz, 3, batch, Bp, nullptr, target, true, m->stream);
  backward(m, w, Bp);
  MHIP(hipGetLastError());
  if (grads_out) {  // gradients of this step, in the parameter order of streami_mlp_set_params
    size_t off = 0;
    for (int l = 0; l < NL; ++l) {
      MHIP(hipMemcpy2DAsync(grads_out + off, (size_t)WID[l] * 4, m->gW[l], (size_t)IN_PAD[l] * 4, (size_t)WID[l] * 4,
                            WID[l + 1], hipMemcpyDeviceToHost, m->stream));
      off += (size_t)WID[l + 1] * WID[l];
      MHIP(hipMemcpyAsync(grads_out + off, m->gb[l], (size_t)WID[l + 1] * 4, hipMemcpyDeviceToHost, m->stream));
      off += WID[l + 1];
    }
  }
  if (lr > 0) {
    ++m->t;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)m->t), c2 = 1.0f - powf(b2, (float)m->t);
    for (int l = 0; l < NL; ++l) {
      hipLaunchKernelGGL(k_adam, dim3(grid_for((long long)WID[l + 1] * WID[l])), dim3(256), 0, m->stream, m->W[l],
                         m->mW[l], m->vW[l], m->gW[l], WID[l + 1], WID[l], IN_PAD[l], lr, b1, b2, eps, c1, c2);
      hipLaunchKernelGGL(k_adam, dim3(grid_for(WID[l + 1])), dim3(256), 0, m->stream, m->b[l], m->mb[l], m->vb[l],
                         m->gb[l], 1, WID[l + 1], WID[l + 1], lr, b1, b2, eps, c1, c2);
    }
    refresh_bf16(m);
  }
  if (loss_out) {
    float s = 0;
    MHIP(hipMemcpyAsync(&s, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
    MHIP(hipStreamSynchronize(m->stream));
    *loss_out = s / (float)(batch * 3);
  } else if (grads_out) {
    MHIP(hipStreamSynchronize(m->stream));
  }
  MHIP(hipGetLastError());
  return STREAMI_OK;
}

}  // namespace

namespace streami {
// Network output for n rows of positions spaced xstride floats apart (3 for
// packed xyz, 4 for the particle float4 array): one fused launch, no workspace.
int mlp_forward_rows(streami_mlp m, const float* xyz, int xstride, long long n, float* out, hipStream_t st) {
  if (n <= 0) return STREAMI_OK;
  if (st != m->stream) MHIP(hipStreamSynchronize(m->stream));
  InferArgs a;
  a.frag = reinterpret_cast<const uint4*>(m->frag);
  for (int l = 0; l < NL; ++l) a.b[l] = m->b[l];
  a.xyz = xyz;
  a.xstride = xstride;
  a.n = n;
  a.period = m->period;
  for (int c = 0; c < 3; ++c) a.sigma[c] = m->sigma[c];
  a.out = out;
  const long long per = 32 * INFER_WAVES;
  const long long grid = (n + per - 1) / per;
  if (grid > 0x7fffffffLL) return mfail(STREAMI_E_ARG, "too many rows for one launch");
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)grid), dim3(64 * INFER_WAVES), 0, st, a);
  MHIP(hipGetLastError());
  return STREAMI_OK;
}
}  // namespace streami

extern "C" {

int streami_mlp_create(const float* params, const float* sigma, float period, void* hip_stream, streami_mlp* out) {
  if (!out || !params || !sigma) return mfail(STREAMI_E_ARG, "NULL argument");
  if (!(period > 0)) return mfail(STREAMI_E_ARG, "period must be > 0");
  for (int c = 0; c < 3; ++c)
    if (!(sigma[c] > 0)) return mfail(STREAMI_E_ARG, "sigma must be > 0");
  streami_mlp_s* m = new (std::nothrow) streami_mlp_s();
  if (!m) return mfail(STREAMI_E_NOMEM, "host allocation failed");
  m->stream = (hipStream_t)hip_stream;
  std::memcpy(m->sigma, sigma, sizeof m->sigma);
  m->period = period;
  int rc = STREAMI_OK;
  for (int l = 0; l < NL && !rc; ++l) {
    const size_t nw = (size_t)WID[l + 1] * WID[l], nb = WID[l + 1];
    const size_t npad = (size_t)OUT_PAD[l] * IN_PAD[l];
    if ((rc = dalloc(m, (void**)&m->W[l], nw * 4)) || (rc = dalloc(m, (void**)&m->b[l], nb * 4)) ||
        (rc = dalloc(m, (void**)&m->mW[l], nw * 4)) || (rc = dalloc(m, (void**)&m->vW[l], nw * 4)) ||
        (rc = dalloc(m, (void**)&m->mb[l], nb * 4)) || (rc = dalloc(m, (void**)&m->vb[l], nb * 4)) ||
        (rc = dalloc(m, (void**)&m->Wb[l], npad * 2)) || (rc = dalloc(m, (void**)&m->WTb[l], npad * 2)) ||
        (rc = dalloc(m, (void**)&m->gW[l], npad * 4)) || (rc = dalloc(m, (void**)&m->gb[l], (size_t)OUT_PAD[l] * 4)))
      break;
    (void)hipMemsetAsync(m->mW[l], 0, nw * 4, m->stream);
    (void)hipMemsetAsync(m->vW[l], 0, nw * 4, m->stream);
    (void)hipMemsetAsync(m->mb[l], 0, nb * 4, m->stream);
    (void)hipMemsetAsync(m->vb[l], 0, nb * 4, m->stream);
  }
  if (!rc) rc = dalloc(m, (void**)&m->loss, 4);
  if (!rc) rc = dalloc(m, (void**)&m->frag, (size_t)FR_OFF[NL] * 16);
  if (rc) {
    streami_mlp_destroy(m);
    return rc;
  }
  rc = streami_mlp_set_params(m, params);
  if (rc) {
    streami_mlp_destroy(m);
    return rc;
  }
  *out = m;
  return STREAMI_OK;
}

int streami_mlp_destroy(streami_mlp m) {
  if (!m) return STREAMI_OK;
  (void)hipDeviceSynchronize();  // kernels on other streams may still read the weights
  for (void* p : m->owned)
    if (p) (void)hipFree(p);
  delete m;
  return STREAMI_OK;
}

int streami_mlp_set_params(streami_mlp m, const float* params) {
  if (!m || !params) return mfail(STREAMI_E_ARG, "NULL argument");
  size_t off = 0;
  for (int l = 0; l < NL; ++l) {
    const size_t nw = (size_t)WID[l + 1] * WID[l], nb = WID[l + 1];
    MHIP(hipMemcpyAsync(m->W[l], params + off, nw * 4, hipMemcpyHostToDevice, m->stream));
    off += nw;
    MHIP(hipMemcpyAsync(m->b[l], params + off, nb * 4, hipMemcpyHostToDevice, m->stream));
    off += nb;
  }
  refresh_bf16(m);
  MHIP(hipStreamSynchronize(m->stream));
  return STREAMI_OK;
}

int streami_mlp_get_params(streami_mlp m, float* params) {
  if (!m || !params) return mfail(STREAMI_E_ARG, "NULL argument");
  size_t off = 0;
  for (int l = 0; l < NL; ++l) {
    const size_t nw = (size_t)WID[l + 1] * WID[l], nb = WID[l + 1];
    MHIP(hipMemcpyAsync(params + off, m->W[l], nw * 4, hipMemcpyDeviceToHost, m->stream));
    off += nw;
    MHIP(hipMemcpyAsync(params + off, m->b[l], nb * 4, hipMemcpyDeviceToHost, m->stream));
    off += nb;
  }
  MHIP(hipStreamSynchronize(m->stream));
  return STREAMI_OK;
}

int streami_mlp_forward(streami_mlp m, const float* xyz, int64_t n, float* out) {
  if (!m || (!xyz && n > 0) || (!out && n > 0)) return mfail(STREAMI_E_ARG, "NULL argument");
  if (n < 0) return mfail(STREAMI_E_ARG, "n must be >= 0");
  return streami::mlp_forward_rows(m, xyz, 3, n, out, m->stream);
}

int streami_mlp_train_step(streami_mlp m, const float* xyz, const float* target, int64_t batch, float lr,
                           float* loss_out, float* grads_out) {
  if (!m || !xyz || !target) return mfail(STREAMI_E_ARG, "NULL argument");
  if (batch < 1 || batch > (1LL << 22)) return mfail(STREAMI_E_ARG, "batch must be in [1, 2^22]");
  if (!(lr >= 0)) return mfail(STREAMI_E_ARG, "lr must be >= 0");
  const long long Bp = (batch + 31) / 32 * 32;
  int rc = ensure_batch(m, Bp);
  if (rc) return rc;
  return train_step_on(m, m->ws, xyz, target, batch, Bp, lr, loss_out, grads_out);
}

int streami_mlp_train_step_noalloc(streami_mlp m, const float* xyz, const float* target, int64_t batch, float lr,
                                   float* loss_out, float* grads_out) {
  if (!m || !xyz || !target) return mfail(STREAMI_E_ARG, "NULL argument");
  if (batch < 1 || batch > STREAMI_MLP_NOALLOC_MAX_BATCH)
    return mfail(STREAMI_E_ARG, "batch must be in [1, %d] for the allocation-free training step",
                 (int)STREAMI_MLP_NOALLOC_MAX_BATCH);
  if (!(lr >= 0)) return mfail(STREAMI_E_ARG, "lr must be >= 0");
  char* ws = nullptr;
  int rc = scratch_for_current_device(&ws);
  if (rc) return rc;
  const long long Bp = (batch + 31) / 32 * 32;
  // every workspace element a step reads is written earlier in the same step (padded rows
  // included), so the previous call's contents need no clearing
  return train_step_on(m, carve_workspace(ws, Bp), xyz, target, batch, Bp, lr, loss_out, grads_out);
}

}  // extern "C"
