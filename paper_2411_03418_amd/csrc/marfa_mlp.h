// marfa_mlp.h -- device primitives of the learned line shape: a 3-64-64-64-64-1
// SiLU network evaluated with BF16-in / FP32-accumulate MFMA on gfx950.
//
// What the network models.  For a Voigt line (Eq.(7)-(8)) with
// x = sqrt(ln2) d / alpha_D and y = sqrt(ln2) gamma_L / alpha_D, the line
// shape times the wing factor chi (Eq.(10)) is written
//     F(d) chi(|d|) = sqrt(ln2 / pi) / alpha_D * Kb(x, y) * exp(t)
// with the analytic base (rho = x^2 + y^2)
//     Kb(x, y) = y (1 + (3x^2 - y^2) / (2 rho^2 + 1)) / (sqrt(pi) (rho + exp(-rho) / 2))
//              + exp(-x^2) / (1 + sqrt(pi) y)^2,
// whose first part is the two leading terms of the large-|z| expansion of
// Re w(z) = K (kept finite at z = 0) and whose second is the Doppler core;
// the network
// predicts the bounded residual t = log(K chi) - log(Kb) from the inputs
//     f1 = asinh(|x|) / 8,  f2 = log10(y) / 2,  f3 = max(|d| - 3, 0) / c
// (|d| and the cut-off c in cm^-1; f3 is |d|/c measured from the first
// Tonkov break, where log chi turns linear in |d|).  Trained domain:
// 1e-4 <= y <= 1e3; other pairs take the plain line shape.
//
// Parameters follow the oracle's packing: W0[64][3], b0[64], W1..W3[64][64]
// with b1..b3[64], W4[1][64], b4[1] (row-major [out][in]); 12801 values.
//
// MFMA layout (v_mfma_f32_16x16x32_bf16, one wavefront).  Activations are
// kept transposed: a 16x16 accumulator tile holds 16 output features (rows)
// of 16 samples (columns); lane l = 16 q + col holds rows 4q .. 4q+3 of
// sample col.  With the weights as the A operand and the activations as the
// B operand, the 32 K slots of lane group q in chunk c are the input
// features 16 (2c + e/4) + 4q + e%4, e = 0..7 -- exactly the values the lane
// already holds from the previous layer's accumulators (row tiles 2c and
// 2c+1), so layers chain without any exchange between lanes.  The weight
// blocks are stored pre-permuted to match.  Activations enter the MFMA as a
// BF16 pair hi + lo (two MFMAs), so only the weights are rounded to BF16.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace marfa {

constexpr int kMlpIn = 3;
constexpr int kMlpHid = 64;
constexpr int kMlpHidLayers = 3;   // 64 -> 64 layers on MFMA
constexpr int kMlpParams = kMlpHid * kMlpIn + kMlpHid + kMlpHidLayers * (kMlpHid * kMlpHid + kMlpHid) + kMlpHid + 1;
// offsets of the packed parameters
constexpr int kMlpOffW0 = 0;
constexpr int kMlpOffB0 = kMlpOffW0 + kMlpHid * kMlpIn;
constexpr int kMlpOffHid = kMlpOffB0 + kMlpHid;                  // W1, b1, W2, b2, W3, b3
constexpr int kMlpHidStride = kMlpHid * kMlpHid + kMlpHid;
constexpr int kMlpOffW4 = kMlpOffHid + kMlpHidLayers * kMlpHidStride;
constexpr int kMlpOffB4 = kMlpOffW4 + kMlpHid;
static_assert(kMlpOffB4 + 1 == kMlpParams, "parameter packing");
// trained domain in y
constexpr float kMlpYMin = 1e-4f, kMlpYMax = 1e3f;
constexpr float kMlpChiBreak = 3.0f;   // cm^-1, first break of the Tonkov chi

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Device copy of a network in evaluation form (all pointers device memory).
struct MlpDev {
  const float4* w0b;      // [64] {W0[o][0], W0[o][1], W0[o][2], b0[o]}, weights BF16-rounded
  const uint4* wp;        // [3][8][64] forward A blocks (8 BF16 per lane), block = 2 r + c
  const uint4* wpt;       // [3][8][64] backward A blocks of W^T
  const float* bh;        // [3][64] hidden biases
  const float* w4;        // [64] output weights, BF16-rounded
  const float* b4;        // [1]
};

// K slot e of lane group q in chunk c -> feature index
__host__ __device__ constexpr int mlp_feat(int c, int q, int e) { return 16 * (2 * c + e / 4) + 4 * q + (e % 4); }

__device__ __forceinline__ float mlp_silu(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float mlp_dsilu(float z) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// round-to-nearest-even FP32 -> BF16 bits
__device__ __forceinline__ uint32_t mlp_bf16_bits(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float mlp_bf16_round(float v) { return __uint_as_float(mlp_bf16_bits(v) << 16); }

// B operand (8 BF16) of chunk c from the lane's 16 activations h[t*4+i],
// split into hi and lo parts, both rounded to nearest even: in integer
// arithmetic (training), or with v_cvt_pk_bf16_f32 (inference; the same
// values in a quarter of the instructions)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <bool HW = false>
__device__ __forceinline__ void mlp_pack_b(const float* h, int c, bf16x8& hi, bf16x8& lo) {
  uint32_t wh[4], wl[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    // elements 2p, 2p+1 -> features (t = 2c + (2p)/4, i = (2p)%4) and next
    const int e0 = 2 * p, e1 = 2 * p + 1;
    const float v0 = h[(2 * c + e0 / 4) * 4 + (e0 % 4)];
    const float v1 = h[(2 * c + e1 / 4) * 4 + (e1 % 4)];
    if constexpr (HW) {
      const bf16x2 hp = __builtin_convertvector((f32x2){v0, v1}, bf16x2);
      uint32_t u;
      __builtin_memcpy(&u, &hp, 4);
      const f32x2 r = {v0 - __uint_as_float(u << 16), v1 - __uint_as_float(u & 0xffff0000u)};
      const bf16x2 lp = __builtin_convertvector(r, bf16x2);
      wh[p] = u;
      __builtin_memcpy(&wl[p], &lp, 4);
    } else {
      const uint32_t h0 = mlp_bf16_bits(v0), h1 = mlp_bf16_bits(v1);
      const float r0 = v0 - __uint_as_float(h0 << 16), r1 = v1 - __uint_as_float(h1 << 16);
      wh[p] = h0 | (h1 << 16);
      wl[p] = mlp_bf16_bits(r0) | (mlp_bf16_bits(r1) << 16);
    }
  }
  __builtin_memcpy(&hi, wh, 16);
  __builtin_memcpy(&lo, wl, 16);
}

__device__ __forceinline__ bf16x8 mlp_as_bf16x8(uint4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

// One hidden layer for one sample tile: z_out[r*4+i] = b[16r+4q+i] + sum_in W[..][in] h_in[in]
template <bool HW = false>
__device__ __forceinline__ void mlp_hidden(const uint4* __restrict__ wp_layer, const float* __restrict__ bias,
                                           const float* h, float* z, int lane) {
  const int q = lane >> 4;
  bf16x8 bh[2], bl[2];
  mlp_pack_b<HW>(h, 0, bh[0], bl[0]);
  mlp_pack_b<HW>(h, 1, bh[1], bl[1]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    f32x4 acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = bias[16 * r + 4 * q + i];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const bf16x8 a = mlp_as_bf16x8(wp_layer[(2 * r + c) * 64 + lane]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh[c], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl[c], acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) z[r * 4 + i] = acc[i];
  }
}

// Input features of one (line, node) pair
__device__ __forceinline__ void mlp_features(float x, float y, float ad_cm, float inv_c_cm, float& f1, float& f2,
                                             float& f3) {
  const float ax = fabsf(x);
  f1 = __logf(ax + sqrtf(ax * ax + 1.0f)) * 0.125f;
  f2 = __log10f(y) * 0.5f;
  f3 = fmaxf(ad_cm - kMlpChiBreak, 0.0f) * inv_c_cm;
}

// the analytic base Kb(x, y)
__device__ __forceinline__ float mlp_base(float x, float y) {
  const float kSqrtPi = 1.7724538509055160f;
  const float x2 = x * x, y2 = y * y;
  const float r = x2 + y2;
  const float u = 1.0f + kSqrtPi * y;
  const float wing = y * (1.0f + (3.0f * x2 - y2) * __builtin_amdgcn_rcpf(2.0f * r * r + 1.0f)) *
                     __builtin_amdgcn_rcpf(kSqrtPi * (r + 0.5f * __expf(-r)));
  return wing + __expf(-x2) * __builtin_amdgcn_rcpf(u * u);
}

// Wave-collective forward pass: every lane brings one sample (f1, f2, f3)
// and receives its network output t.  All 64 lanes must call it together.
// Weights may live in global memory or LDS (generic pointers).  Only the
// first 16 ns lanes' samples are evaluated (ns uniform, 1..4); the other
// lanes receive 0.
//
// SCALED: the weights are in the scaled form of mlp_scaled_* (layer 0 and the
// hidden biases times log2 e, the output weights times ln 2).  Every hidden
// value then carries the factor log2 e, z' = z log2 e, and the activation is
// h' = z' / (1 + 2^-z') = log2 e SiLU(z): one multiply fewer per value than
// z / (1 + e^-z), the same network up to single-precision rounding.
constexpr float kMlpLog2e = 1.44269504088896340736f;
constexpr float kMlpLn2 = 0.693147180559945309417f;
__device__ __forceinline__ float mlp_silu_scaled(float zs) {
  return zs * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-zs));
}
__host__ __device__ __forceinline__ float4 mlp_scaled_w0b(float4 w) {
  return make_float4(w.x * kMlpLog2e, w.y * kMlpLog2e, w.z * kMlpLog2e, w.w * kMlpLog2e);
}
__host__ __device__ __forceinline__ float mlp_scaled_bh(float b) { return b * kMlpLog2e; }
__host__ __device__ __forceinline__ float mlp_scaled_w4(float w) { return w * kMlpLn2; }

template <bool SCALED = false>
__device__ __forceinline__ float mlp_forward_wave(const MlpDev& W, float f1, float f2, float f3, int ns = 4) {
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, col = lane & 15;
  auto act = [](float z) { return SCALED ? mlp_silu_scaled(z) : mlp_silu(z); };
  float result = 0.0f;
#pragma unroll 1
  for (int s = 0; s < ns; ++s) {
    // keeps the weight loads inside the loop: hoisted to the callers' loops
    // they would hold ~100 registers for the whole kernel
    asm volatile("" ::: "memory");
    const int src = 16 * s + col;
    const float g1 = __shfl(f1, src), g2 = __shfl(f2, src), g3 = __shfl(f3, src);
    float h[16], z[16];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float4 w = W.w0b[16 * t + 4 * q + i];
        h[t * 4 + i] = act(fmaf(w.x, g1, fmaf(w.y, g2, fmaf(w.z, g3, w.w))));
      }
#pragma unroll 1
    for (int k = 0; k < kMlpHidLayers; ++k) {
      mlp_hidden<true>(W.wp + k * 8 * 64, W.bh + k * 64, h, z, lane);
#pragma unroll
      for (int v = 0; v < 16; ++v) h[v] = act(z[v]);
    }
    float part = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) part = fmaf(W.w4[16 * t + 4 * q + i], h[t * 4 + i], part);
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    if (q == s) result = part + W.b4[0];
  }
  return result;
}

}  // namespace marfa
