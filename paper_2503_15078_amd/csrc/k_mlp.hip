// Learned warm start of the contact impulses (an addition to the paper's method, which
// leaves the initial impulse of a frame open): a 12 -> 128 -> 128 -> 3 network with GELU
// (inputs padded to 16, outputs to 16), bf16 weights and activations on the matrix
// cores with float32 accumulation, float32 master weights and Adam for training.
//
// Every layer is computed transposed, Z^T = W H^T, with the 16 samples of a wavefront
// as the N dimension of the 16x16 matrix-core tiles.  In that form the float32 output
// tile of one layer (lane l: rows 4 (l / 16) + i, column l % 16) is, after bias, GELU
// and bf16 rounding, a B operand of the next layer, so activations stay in registers
// through the forward and backward passes.  Contractions over 128 features use
// v_mfma_f32_16x16x32_bf16, whose B operand is two such output tiles side by side; the
// 16-wide ones (the input layer, the output gradient) use v_mfma_f32_16x16x16_bf16.
// Weight gradients contract over samples; for them the block's 64 samples of each
// activation are written to LDS with samples contiguous and each wavefront accumulates
// 20 of the 80 gradient tiles.
//
// LDS rows are padded by 16 bytes so that the 16 rows one operand load touches start
// on different banks.  The 128-wide weight rows are stored with their columns permuted
// within each block of 32 (kperm), so that one 16-byte load gives a lane the eight
// weights that meet its two output-tile halves.
//
// Features (per contact, frame start), with l the mean rest edge length of the scene:
//   f0 (n . x~ - d_n) / l, f1..3 n, f4..6 h C (v_t - u_obstacle) / l,
//   f7..9 h^2 K_jj lambda_prev / l, f10 log K_jj, f11 mu, f12..15 0;
// the network predicts h^2 K_jj lambda / l.  The prediction replaces the previous-frame
// impulse after projection onto the friction cone (lambda_n >= 0, |lambda_f| <= mu
// lambda_n); a contact whose prediction is not finite keeps the previous-frame value.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace lg {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// bf16 by round to nearest even on the bit pattern (NaN kept quiet)
__device__ inline short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (short)0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ inline float bf2f(short b) { return __uint_as_float(((unsigned)(unsigned short)b) << 16); }
// GELU h = z Phi(z) and its derivative Phi(z) + z phi(z), from one erf
__device__ inline float gelu(float z, float& grad) {
  const float Phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  grad = Phi + z * 0.39894228040143268f * __expf(-0.5f * z * z);
  return z * Phi;
}
__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// K = 32: slot s of lane group g carries one contraction index for both operands alike,
// so the sum is the same for any assignment of the 32 indices to (g, s)
__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}
__device__ inline bf16x4 ld4(const short* p) { return *reinterpret_cast<const bf16x4*>(p); }
__device__ inline bf16x8 ld8(const short* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ inline bf16x8 cat(bf16x4 a, bf16x4 b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7); }

// Row strides in LDS (shorts): 128-wide weight rows and 64-sample activation rows, each
// padded by 8.
constexpr int kW = 136, kS = 72;
// Position of column c of a 128-wide weight row: within each block of 32 columns, lane
// group g reads positions 8 g .. 8 g + 7, which hold columns 4 g .. 4 g + 3 (the first
// output tile's rows for that group) and 16 + 4 g .. 16 + 4 g + 3 (the second tile's).
__host__ __device__ constexpr int kperm(int c) { return (c & ~31) + 8 * ((c & 15) >> 2) + 4 * ((c & 31) >> 4) + (c & 3); }
constexpr bool kperm_valid() {  // a permutation of 0..127 that keeps runs of four whole
  bool seen[128] = {};
  for (int c = 0; c < 128; ++c) {
    const int p = kperm(c);
    if (p < 0 || p >= 128 || seen[p] || ((c & 3) != 0 && p != kperm(c - 1) + 1)) return false;
    seen[p] = true;
  }
  return true;
}
static_assert(kperm_valid(), "kperm");

constexpr int kOW1 = 0, kOB1 = 2048, kOW2 = 2176, kOB2 = 18560, kOW3 = 18688, kOB3 = 20736;
static_assert(kOB3 + 16 == kMlpParams, "parameter layout");
static_assert(kOB1 % 4 == 0 && kOW2 % 4 == 0 && kOB2 % 4 == 0 && kOW3 % 4 == 0 && kOB3 % 4 == 0, "float4 staging");

// weights of the forward pass in LDS (bf16, row-major [out][in], W2 and W3 rows padded
// to kW with columns at kperm) and biases (float32)
struct __attribute__((aligned(16))) MlpSmem {
  short W1[128 * 16], W2[128 * kW], W3[16 * kW];
  float b1[128], b2[128], b3[16];
};

__device__ inline bf16x4 f2bf4(float4 v) {
  bf16x4 b;
  b[0] = f2bf(v.x);
  b[1] = f2bf(v.y);
  b[2] = f2bf(v.z);
  b[3] = f2bf(v.w);
  return b;
}

// Reads N floats at src (16-byte aligned; the block's kBlock threads) as float4, up to
// eight loads in flight per thread, and hands each to put(index of its first float, v).
template <int N, class F>
__device__ inline void stage(const float* src, F put) {
  static_assert(N % 4 == 0, "whole float4");
  constexpr int n4 = N / 4;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  for (int i0 = threadIdx.x; i0 < n4; i0 += 8 * kBlock) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * kBlock < n4) v[u] = s4[i0 + u * kBlock];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * kBlock < n4) put(4 * (i0 + u * kBlock), v[u]);
  }
}

// Transposed bf16 copy of an R x 128 block of float32 parameters at src (row-major,
// 16-byte aligned): entry (o, c) goes to dst[c * ld + col(o)], where col keeps every run
// of four rows o = 4 k .. 4 k + 3 consecutive.  Each thread moves 4 x 4 sub-blocks, so
// its stores are 8 bytes wide and the 32 lanes that share a row of dst fill it.
template <int R, class Col>
__device__ inline void stage_transposed(short* dst, int ld, const float* src, Col col) {
  constexpr int nb = (R / 4) * 32;
  for (int b0 = threadIdx.x; b0 < nb; b0 += 4 * kBlock) {
    f32x4 v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * kBlock, o = 4 * (b % (R / 4)), c = 4 * (b / (R / 4));
      if (b < nb)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[u][q] = *reinterpret_cast<const f32x4*>(src + (o + q) * 128 + c);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * kBlock, o = 4 * (b % (R / 4)), c = 4 * (b / (R / 4));
      if (b < nb)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          bf16x4 t;
#pragma unroll
          for (int q = 0; q < 4; ++q) t[q] = f2bf(v[u][q][k]);
          *reinterpret_cast<bf16x4*>(dst + (c + k) * ld + col(o)) = t;
        }
    }
  }
}

// P: the float32 parameters, 16-byte aligned; the block has kBlock threads
__device__ inline void load_forward_weights(MlpSmem& s, const float* P) {
  stage<128 * 16>(P + kOW1, [&](int e, float4 v) { *reinterpret_cast<bf16x4*>(s.W1 + e) = f2bf4(v); });
  // four consecutive columns of a 128-wide row stay consecutive under kperm
  stage<128 * 128>(P + kOW2, [&](int e, float4 v) {
    *reinterpret_cast<bf16x4*>(s.W2 + (e >> 7) * kW + kperm(e & 127)) = f2bf4(v);
  });
  stage<16 * 128>(P + kOW3, [&](int e, float4 v) {
    *reinterpret_cast<bf16x4*>(s.W3 + (e >> 7) * kW + kperm(e & 127)) = f2bf4(v);
  });
  stage<128>(P + kOB1, [&](int e, float4 v) { *reinterpret_cast<float4*>(s.b1 + e) = v; });
  stage<128>(P + kOB2, [&](int e, float4 v) { *reinterpret_cast<float4*>(s.b2 + e) = v; });
  stage<16>(P + kOB3, [&](int e, float4 v) { *reinterpret_cast<float4*>(s.b3 + e) = v; });
}

// Forward pass of one wavefront's 16 samples.  xb: B operand of the input (lane l:
// sample l % 16, features 4 (l / 16) .. +3).  Returns y (lane l < 16: outputs 0..3 of
// sample l); g1, g2 (GELU derivatives at the pre-activations, for the backward pass)
// and h1b, h2b (bf16 activations) in the output tile layout (lane l: features
// 16 m + 4 (l / 16) + i of sample l % 16).
__device__ inline f32x4 forward_tile(const MlpSmem& s, bf16x4 xb, f32x4 g1[8], bf16x4 h1b[8], f32x4 g2[8],
                                     bf16x4 h2b[8]) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    f32x4 z = mfma(ld4(s.W1 + (16 * m + r) * 16 + 4 * g), xb, zero);
    bf16x4 hb;
    f32x4 gr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float d;
      hb[i] = f2bf(gelu(z[i] + s.b1[16 * m + 4 * g + i], d));
      gr[i] = d;
    }
    g1[m] = gr;
    h1b[m] = hb;
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    f32x4 z = zero;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
      z = mfma32(ld8(s.W2 + (16 * m + r) * kW + 32 * kc + 8 * g), cat(h1b[2 * kc], h1b[2 * kc + 1]), z);
    bf16x4 hb;
    f32x4 gr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float d;
      hb[i] = f2bf(gelu(z[i] + s.b2[16 * m + 4 * g + i], d));
      gr[i] = d;
    }
    g2[m] = gr;
    h2b[m] = hb;
  }
  f32x4 y = zero;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) y = mfma32(ld8(s.W3 + r * kW + 32 * kc + 8 * g), cat(h2b[2 * kc], h2b[2 * kc + 1]), y);
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] += s.b3[4 * g + i];
  return y;
}

// B operand of 16 input rows X[n][16] (float32), rows >= n read as zero
__device__ inline bf16x4 load_x(const float* X, int row, int n) {
  const int g = (threadIdx.x & 63) >> 4;
  bf16x4 xb;
  if (row < n) {
    const float4 v = *reinterpret_cast<const float4*>(X + (int64_t)row * 16 + 4 * g);
    xb[0] = f2bf(v.x);
    xb[1] = f2bf(v.y);
    xb[2] = f2bf(v.z);
    xb[3] = f2bf(v.w);
  } else {
    xb[0] = xb[1] = xb[2] = xb[3] = 0;
  }
  return xb;
}

// ---------------------------------------------------------------- inference
__global__ void __launch_bounds__(kBlock) k_mlp_forward(const float* P, const float* X, float* Y, int n) {
  __shared__ MlpSmem s;
  load_forward_weights(s, P);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  f32x4 g1[8], g2[8];
  bf16x4 h1b[8], h2b[8];
  for (int base = (blockIdx.x * 4 + wave) * 16; base < n; base += gridDim.x * 64) {
    const int row = base + (lane & 15);
    const f32x4 y = forward_tile(s, load_x(X, row, n), g1, h1b, g2, h2b);
    if (lane < 16 && row < n)
      for (int i = 0; i < 3; ++i) Y[(int64_t)row * 3 + i] = y[i];
  }
}

// ---------------------------------------------------------------- training
struct __attribute__((aligned(16))) MlpTrainSmem {
  MlpSmem f;
  short W2T[128 * kW], W3T[128 * 16];  // transposes for the backward products
  // the block's 64 samples of each activation, [feature][sample], rows padded to kS
  short XT[16 * kS], H1T[128 * kS], H2T[128 * kS], D1T[128 * kS], D2T[128 * kS], DYT[16 * kS];
  float red[kBlock / 64];
};

// Forward and backward over the 64 samples [64 blockIdx, +64) of X (n x 16), targets T
// (n x 3); loss = sum (y - t)^2 / (3 n).  Writes the block's gradient partial sums and
// its loss sum to partial[blockIdx][0 .. kMlpParams].  (One sample tile per block keeps
// the 80 weight-gradient accumulators apart from the forward/backward registers.)
__global__ void __launch_bounds__(kBlock) k_mlp_train(const float* P, const float* X, const float* T, int n,
                                                      float* partial) {
  __shared__ MlpTrainSmem s;
  load_forward_weights(s.f, P);
  stage_transposed<128>(s.W2T, kW, P + kOW2, [](int o) { return kperm(o); });
  stage_transposed<16>(s.W3T, 16, P + kOW3, [](int o) { return o; });
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r = lane & 15, g = lane >> 4;
  const float inv3n = 1.0f / (3.0f * (float)n);
  const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  f32x4 acc[20];
  float db = 0.0f, db3 = 0.0f, loss = 0.0f;
  const int s0 = blockIdx.x * 64, s1 = min(n, s0 + 64);
  f32x4 g1[8], g2[8];
  bf16x4 h1b[8], h2b[8];
  {
    const int base = s0;
    const int row = base + 16 * wave + r, col = 16 * wave + r;
    const bool valid = row < s1;
    const bf16x4 xb = load_x(X, valid ? row : n, n);
    const f32x4 y = forward_tile(s.f, xb, g1, h1b, g2, h2b);
    // dL/dy for outputs 0..2 of valid samples (lanes 0..15 hold outputs 0..3)
    bf16x4 dyb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float dy = 0.0f;
      if (g == 0 && i < 3 && valid) {
        const float e = y[i] - T[(int64_t)row * 3 + i];
        loss += e * e;
        dy = 2.0f * e * inv3n;
      }
      dyb[i] = f2bf(dy);
    }
    // dZ2 = (W3^T dY^T) * gelu'(z2)
    bf16x4 d2b[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      f32x4 dh = mfma(ld4(s.W3T + (16 * m + r) * 16 + 4 * g), dyb, zero);
#pragma unroll
      for (int i = 0; i < 4; ++i) d2b[m][i] = f2bf(dh[i] * g2[m][i]);
    }
    // dZ1 = (W2^T dZ2^T) * gelu'(z1); activations to LDS, samples contiguous
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      f32x4 dh = zero;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        dh = mfma32(ld8(s.W2T + (16 * m + r) * kW + 32 * kc + 8 * g), cat(d2b[2 * kc], d2b[2 * kc + 1]), dh);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int f = 16 * m + 4 * g + i;
        s.D1T[f * kS + col] = f2bf(dh[i] * g1[m][i]);
        s.D2T[f * kS + col] = d2b[m][i];
        s.H1T[f * kS + col] = h1b[m][i];
        s.H2T[f * kS + col] = h2b[m][i];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s.XT[(4 * g + i) * kS + col] = xb[i];
      s.DYT[(4 * g + i) * kS + col] = dyb[i];
    }
    __syncthreads();
    // weight gradients of this wavefront's tiles: t < 8 dW1 (row tile t), t < 72 dW2
    // (row tile (t-8)/8, column tile (t-8)%8), else dW3 (column tile t-72); K = 64 samples
#pragma unroll
    for (int k = 0; k < 20; ++k) {
      acc[k] = zero;
      const int t = wave + 4 * k;
      const short *A, *Bm;
      if (t < 8) {
        A = s.D1T + (16 * t + r) * kS;
        Bm = s.XT + r * kS;
      } else if (t < 72) {
        A = s.D2T + (16 * ((t - 8) >> 3) + r) * kS;
        Bm = s.H1T + (16 * ((t - 8) & 7) + r) * kS;
      } else {
        A = s.DYT + r * kS;
        Bm = s.H2T + (16 * (t - 72) + r) * kS;
      }
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) acc[k] = mfma32(ld8(A + 32 * kc + 8 * g), ld8(Bm + 32 * kc + 8 * g), acc[k]);
    }
    // bias gradients: sums over the block's samples
    {
      const short* Dr = tid < 128 ? s.D1T + tid * kS : s.D2T + (tid - 128) * kS;
      float a = 0.0f;
      for (int q = 0; q < 64; ++q) a += bf2f(Dr[q]);
      db += a;
      if (tid < 16) {
        float b = 0.0f;
        for (int q = 0; q < 64; ++q) b += bf2f(s.DYT[tid * kS + q]);
        db3 += b;
      }
    }
    __syncthreads();
  }
  float* out = partial + (int64_t)blockIdx.x * (kMlpParams + 1);
#pragma unroll
  for (int k = 0; k < 20; ++k) {
    const int t = wave + 4 * k;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 4 * g + i;  // row within the tile; r is the column
      int idx;
      if (t < 8) idx = kOW1 + (16 * t + m) * 16 + r;
      else if (t < 72) idx = kOW2 + (16 * ((t - 8) >> 3) + m) * 128 + 16 * ((t - 8) & 7) + r;
      else idx = kOW3 + m * 128 + 16 * (t - 72) + r;
      out[idx] = acc[k][i];
    }
  }
  out[tid < 128 ? kOB1 + tid : kOB2 + tid - 128] = db;
  if (tid < 16) out[kOB3 + tid] = db3;
  // loss: wave sums, then the block's sum in wave order
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
  if (lane == 0) s.red[wave] = loss;
  __syncthreads();
  if (tid == 0) out[kMlpParams] = (s.red[0] + s.red[1]) + (s.red[2] + s.red[3]);
}

// Sum of the block partials (gradient and loss), then optionally one Adam step on the
// float32 master weights: m, v moments; c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t).  A
// block takes 64 consecutive entries, one per lane; each of its four wavefronts sums one
// quarter of the partials (a contiguous range, in block order) and the four sums are
// added in wavefront order, a fixed order for a given batch size.
__global__ void __launch_bounds__(kBlock) k_mlp_adam(float* P, float* Mo, float* Vo, const float* partial, int nblk,
                                                     float lr, float b1, float b2, float eps, float c1, float c2,
                                                     float inv3n, int update, float* grad_out, float* loss_out) {
  __shared__ float part[kBlock / 64][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  const int quarter = (nblk + 3) / 4, r0 = min(nblk, wave * quarter), r1 = min(nblk, r0 + quarter);
  float a = 0.0f;
  if (p <= kMlpParams) {
    const float* src = partial + p;
    constexpr int64_t kRow = kMlpParams + 1;
    int b = r0;
    for (; b + 8 <= r1; b += 8) {
      float v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = src[(int64_t)(b + i) * kRow];
#pragma unroll
      for (int i = 0; i < 8; ++i) a += v[i];
    }
    for (; b < r1; ++b) a += src[(int64_t)b * kRow];
  }
  part[wave][lane] = a;
  __syncthreads();
  if (wave != 0 || p > kMlpParams) return;
  const float gsum = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
  if (p == kMlpParams) {
    loss_out[0] = gsum * inv3n;
    return;
  }
  if (grad_out) grad_out[p] = gsum;
  if (!update) return;
  const float m = b1 * Mo[p] + (1.0f - b1) * gsum;
  const float v = b2 * Vo[p] + (1.0f - b2) * gsum * gsum;
  Mo[p] = m;
  Vo[p] = v;
  P[p] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// ---------------------------------------------------------------- simulator side
// Features of every contact of the frame (after the plain warm start and the Delassus
// diagonal are known).
__global__ void k_mlp_features(Dev d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = min(d.n_contacts[0], d.CMAX);
  if (j >= c || d.k_off[d.NS] > d.KCAP) return;
  const int CM = d.CMAX, v = d.c_node[j], s = d.c_scene[j];
  const int cs = d.cs_off[s], cnt = d.cs_off[s + 1] - cs;
  const float kjj = d.K[d.k_off[s] + (int64_t)(j - cs) * kstride(cnt) + (j - cs)];
  const double ell = d.ell[s];
  const double h = d.h;
  double xp[3], rel[3];
  // self-contact rows (no obstacle) keep the previous-frame start: their features are zero
  if (d.c_obst[j] < 0) {
    float4* out = reinterpret_cast<float4*>(d.c_feat + (int64_t)j * 16);
    for (int q = 0; q < 4; ++q) out[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return;
  }
  const ObstacleDev& ob = d.obst[d.c_obst[j]];
  for (int q = 0; q < 3; ++q) {
    xp[q] = d.qp[q * d.N4 + v];
    rel[q] = (double)d.vt[q * d.N4 + v] - ob.vel[q];
  }
  float f[16];
  double gap = -d.c_dn64[j];
  for (int q = 0; q < 3; ++q) gap += d.cC64[q * CM + j] * xp[q];
  f[0] = (float)(gap / ell);
  for (int q = 0; q < 3; ++q) f[1 + q] = d.cC[q * CM + j];
  for (int a = 0; a < 3; ++a) {
    double w = 0.0;
    for (int q = 0; q < 3; ++q) w += (double)d.cC[(3 * a + q) * CM + j] * rel[q];
    f[4 + a] = (float)(h * w / ell);
  }
  const double sc = h * h * (double)kjj / ell;
  for (int a = 0; a < 3; ++a) f[7 + a] = (float)(sc * d.lam[a * CM + j]);
  f[10] = logf(kjj);
  f[11] = d.c_mu[j];
  for (int q = 12; q < 16; ++q) f[q] = 0.0f;
  float4* out = reinterpret_cast<float4*>(d.c_feat + (int64_t)j * 16);
  for (int q = 0; q < 4; ++q) out[q] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
}

// Network prediction -> candidate start impulse lam_ml (projected onto the friction
// cone); non-finite predictions keep the previous-frame impulse already in lambda, and
// so do bilateral (binding) rows, whose impulse has no sign or cone.  The candidate
// replaces lambda only where the judge that follows finds it better.
__global__ void __launch_bounds__(kBlock) k_mlp_warm(Dev d) {
  __shared__ MlpSmem s;
  const int c = min(d.n_contacts[0], d.CMAX);
  if (c == 0 || d.k_off[d.NS] > d.KCAP) return;
  load_forward_weights(s, d.mlp_P);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, CM = d.CMAX;
  f32x4 g1[8], g2[8];
  bf16x4 h1b[8], h2b[8];
  for (int base = (blockIdx.x * 4 + wave) * 16; base < c; base += gridDim.x * 64) {
    const int j = base + (lane & 15);
    const f32x4 y = forward_tile(s, load_x(d.c_feat, j, c), g1, h1b, g2, h2b);
    if (lane < 16 && j < c) {
      const int sc = d.c_scene[j], cs = d.cs_off[sc], cnt = d.cs_off[sc + 1] - cs;
      const float kjj = d.K[d.k_off[sc] + (int64_t)(j - cs) * kstride(cnt) + (j - cs)];
      const float back = (float)(d.ell[sc] / (d.h * d.h * (double)kjj));
      float l[3] = {y[0] * back, y[1] * back, y[2] * back};
      const bool fresh = d.warm == 3 && d.lam[j] == 0.0f && d.lam[CM + j] == 0.0f && d.lam[2 * CM + j] == 0.0f;
      if (isfinite(l[0]) && isfinite(l[1]) && isfinite(l[2]) && !(d.c_comp[j] >= 0.0f) && !fresh &&
          d.c_obst[j] >= 0) {  // self-contact rows keep the previous-frame start
        const float mu = d.c_mu[j];
        l[0] = fmaxf(l[0], 0.0f);
        const float lf = sqrtf(l[1] * l[1] + l[2] * l[2]), cap = mu * l[0];
        if (lf > cap) {
          const float sh = lf > 0.0f ? cap / lf : 0.0f;
          l[1] *= sh;
          l[2] *= sh;
        }
      } else {
        for (int q = 0; q < 3; ++q) l[q] = d.lam[q * CM + j];
      }
      for (int q = 0; q < 3; ++q) d.lam_ml[q * CM + j] = l[q];
    }
  }
}

// Scaled impulses h^2 K_jj lambda / l of the frame's contacts (training targets).
__global__ void k_mlp_targets(Dev d, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = min(d.n_contacts[0], d.CMAX);
  if (j >= c || d.k_off[d.NS] > d.KCAP) return;
  const int s = d.c_scene[j], cs = d.cs_off[s], cnt = d.cs_off[s + 1] - cs;
  const float kjj = d.K[d.k_off[s] + (int64_t)(j - cs) * kstride(cnt) + (j - cs)];
  const double sc = d.h * d.h * (double)kjj / d.ell[s];
  for (int a = 0; a < 3; ++a) out[(int64_t)j * 3 + a] = (float)(sc * d.lam[a * d.CMAX + j]);
}

// ---------------------------------------------------------------- launchers
void launch_mlp_forward(const float* P, const float* X, float* Y, int n, hipStream_t st) {
  const int blocks = max(1, min(1024, (n + 63) / 64));
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(kBlock), 0, st, P, X, Y, n);
}

int mlp_train_blocks(int n) { return (n + 63) / 64; }

void launch_mlp_train(const float* P, const float* X, const float* T, int n, float* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_train, dim3(mlp_train_blocks(n)), dim3(kBlock), 0, st, P, X, T, n, partial);
}

void launch_mlp_adam(float* P, float* M, float* V, const float* partial, int n, float lr, float b1, float b2,
                     float eps, float c1, float c2, int update, float* grad_out, float* loss_out, hipStream_t st) {
  const int nb = mlp_train_blocks(n);
  static_assert(kBlock == 256, "four wavefronts per block");
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 1 + 63) / 64), dim3(kBlock), 0, st, P, M, V,
                     partial, nb, lr, b1, b2, eps, c1, c2, 1.0f / (3.0f * (float)n), update, grad_out, loss_out);
}

void launch_mlp_features(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_features, dim3((d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

void launch_mlp_warm(const Dev& d, hipStream_t st) {
  const int blocks = max(1, min(256, (d.CMAX + 63) / 64));
  hipLaunchKernelGGL(k_mlp_warm, dim3(blocks), dim3(kBlock), 0, st, d);
}

void launch_mlp_targets(const Dev& d, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_targets, dim3((d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d, out);
}

}  // namespace lg
