// marfa_surrogate.hip -- the learned line shape: forward, backward and Adam
// kernels of the 3-64-64-64-64-1 SiLU network (BF16-in / FP32-accumulate
// MFMA, v_mfma_f32_16x16x32_bf16) and the host object behind the
// marfa_surrogate_* entry points.  The network, its inputs and its target are
// described in marfa_mlp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "marfa.h"
#include "marfa_internal.h"
#include "marfa_mlp.h"

namespace marfa {

// ------------------------------------------------------------------
// evaluation form of the parameters
// ------------------------------------------------------------------
struct MlpBuffers {
  float4* w0b = nullptr;
  uint4* wp = nullptr;
  uint4* wpt = nullptr;
  float* bh = nullptr;
  float* w4 = nullptr;
  float* b4 = nullptr;
};

// Write parameter p of the packed FP32 vector into the evaluation form:
// BF16-rounded weights, pre-permuted MFMA blocks, FP32 biases.
__device__ __forceinline__ void publish_param(int p, float v, MlpBuffers B) {
  uint16_t* wp16 = reinterpret_cast<uint16_t*>(B.wp);
  uint16_t* wpt16 = reinterpret_cast<uint16_t*>(B.wpt);
  float* w0b = reinterpret_cast<float*>(B.w0b);
  if (p < kMlpOffB0) {
    const int o = p / kMlpIn, i = p % kMlpIn;
    w0b[4 * o + i] = mlp_bf16_round(v);
  } else if (p < kMlpOffHid) {
    w0b[4 * (p - kMlpOffB0) + 3] = v;
  } else if (p < kMlpOffW4) {
    const int k = (p - kMlpOffHid) / kMlpHidStride;
    const int r = (p - kMlpOffHid) % kMlpHidStride;
    if (r >= kMlpHid * kMlpHid) {
      B.bh[k * kMlpHid + (r - kMlpHid * kMlpHid)] = v;
      return;
    }
    const int o = r / kMlpHid, in = r % kMlpHid;
    const uint16_t bits = (uint16_t)mlp_bf16_bits(v);
    {
      // forward block: row o (tile o/16, lane column o%16), K feature in
      const int t = in / 16, rem = in % 16;
      const int c = t / 2, e = 4 * (t % 2) + rem % 4, q = rem / 4;
      const int lane = 16 * q + o % 16;
      wp16[((size_t)(k * 8 + 2 * (o / 16) + c) * 64 + lane) * 8 + e] = bits;
    }
    {
      // backward block of W^T: row in, K feature o
      const int t = o / 16, rem = o % 16;
      const int c = t / 2, e = 4 * (t % 2) + rem % 4, q = rem / 4;
      const int lane = 16 * q + in % 16;
      wpt16[((size_t)(k * 8 + 2 * (in / 16) + c) * 64 + lane) * 8 + e] = bits;
    }
  } else if (p < kMlpOffB4) {
    B.w4[p - kMlpOffW4] = mlp_bf16_round(v);
  } else {
    B.b4[0] = v;
  }
}

__global__ void k_mlp_publish(const float* __restrict__ master, MlpBuffers B) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kMlpParams) publish_param(p, master[p], B);
}

// ------------------------------------------------------------------
// forward pass over a batch (evaluation)
// ------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_forward(MlpDev W, const float* __restrict__ X, int64_t n,
                                                     float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float f1 = 0.f, f2 = 0.f, f3 = 0.f;
  if (i < n) {
    f1 = X[3 * i];
    f2 = X[3 * i + 1];
    f3 = X[3 * i + 2];
  }
  // every lane of the wavefront takes part in the MFMA pass
  const float t = mlp_forward_wave(W, f1, f2, f3);
  if (i < n) out[i] = t;
}

// ------------------------------------------------------------------
// forward + backward of 32 samples per workgroup (one wavefront)
// ------------------------------------------------------------------
// Partial gradient of L = gscale/2 * sum_b (y_b - t_b)^2 (or, with pow4,
// of 1e6 gscale/2 * sum_b (y_b - t_b)^4) over this workgroup's samples, in
// the packed parameter order, followed by the sum of squared errors.
// gscale = 2 / batch gives the gradient of the mean.
constexpr int kGradSamples = 32;

__global__ void __launch_bounds__(64) k_mlp_grad(MlpDev W, const float* __restrict__ X, const float* __restrict__ Tg,
                                                 int64_t n_all, int64_t first, int64_t count, int64_t perm_a,
                                                 int64_t perm_b, float gscale, int pow4, float* __restrict__ partial) {
  // pre-activations z of layers 0..3 for 2 tiles, later their gradients;
  // index [layer][tile][row tile * 4 + i][lane]
  __shared__ float zs[4][2][16][64];
  __shared__ __attribute__((aligned(16))) uint16_t dzs[64][kGradSamples];   // dZ^T [out][sample], BF16
  __shared__ __attribute__((aligned(16))) uint16_t hs[64][kGradSamples];    // H [in][sample], BF16
  __shared__ float fs[3][kGradSamples];
  __shared__ float douts[kGradSamples];
  __shared__ float errs[kGradSamples];
  const int lane = threadIdx.x;
  const int q = lane >> 4, col = lane & 15;
  float* P = partial + (size_t)blockIdx.x * (kMlpParams + 1);
  // my sample (lanes 0..31): position first + 32 b + lane of the affine
  // permutation pos -> (perm_a pos + perm_b) mod n_all of the sample set
  const int64_t local = (int64_t)blockIdx.x * kGradSamples + lane;
  float f1 = 0.f, f2 = 0.f, f3 = 0.f, tg = 0.f;
  bool valid = false;
  if (lane < kGradSamples && local < count) {
    const int64_t idx = (perm_a * ((first + local) % n_all) + perm_b) % n_all;
    f1 = X[3 * idx];
    f2 = X[3 * idx + 1];
    f3 = X[3 * idx + 2];
    tg = Tg[idx];
    valid = true;
  }
  if (lane < kGradSamples) {
    fs[0][lane] = f1;
    fs[1][lane] = f2;
    fs[2][lane] = f3;
  }
  // ---- forward
  for (int s = 0; s < 2; ++s) {
    const int src = 16 * s + col;
    const float g1 = __shfl(f1, src), g2 = __shfl(f2, src), g3 = __shfl(f3, src);
    float h[16], z[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float4 w = W.w0b[16 * (v / 4) + 4 * q + (v % 4)];
      z[v] = fmaf(w.x, g1, fmaf(w.y, g2, fmaf(w.z, g3, w.w)));
      zs[0][s][v][lane] = z[v];
      h[v] = mlp_silu(z[v]);
    }
    for (int k = 0; k < kMlpHidLayers; ++k) {
      mlp_hidden(W.wp + k * 8 * 64, W.bh + k * 64, h, z, lane);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        zs[k + 1][s][v][lane] = z[v];
        h[v] = mlp_silu(z[v]);
      }
    }
    float part = 0.f;
#pragma unroll
    for (int v = 0; v < 16; ++v) part = fmaf(W.w4[16 * (v / 4) + 4 * q + (v % 4)], h[v], part);
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    const float y = part + W.b4[0];
    const float ts = __shfl(tg, src);
    const bool vs = __shfl((int)valid, src) != 0;
    if (q == 0) {
      const float e = vs ? y - ts : 0.f;
      // mean squared error, or a mean fourth power (scaled by 1e6) that
      // weights the largest errors
      douts[src] = pow4 ? gscale * 2e6f * e * e * e : gscale * e;
      errs[src] = e * e;
    }
  }
  __syncthreads();
  if (lane == 0) {
    float sse = 0.f, db = 0.f;
    for (int i = 0; i < kGradSamples; ++i) {
      sse += errs[i];
      db += douts[i];
    }
    P[kMlpParams] = sse;
    P[kMlpOffB4] = db;
  }
  // ---- output layer: dW4[f] = sum_s dout_s h3[f][s]; thread f = lane
  {
    const int f = lane, t = f / 16, qo = (f % 16) / 4, i = f % 4;
    float acc = 0.f;
    for (int s = 0; s < 2; ++s)
      for (int c = 0; c < 16; ++c) acc = fmaf(douts[16 * s + c], mlp_silu(zs[3][s][4 * t + i][16 * qo + c]), acc);
    P[kMlpOffW4 + f] = acc;
  }
  __syncthreads();
  // dz3 = w4 dout silu'(z3), in place
  for (int s = 0; s < 2; ++s) {
    const float d = douts[16 * s + col];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float z = zs[3][s][v][lane];
      zs[3][s][v][lane] = W.w4[16 * (v / 4) + 4 * q + (v % 4)] * d * mlp_dsilu(z);
    }
  }
  // ---- hidden layers k = 3, 2, 1 (weights of hidden layer k-1)
  for (int k = kMlpHidLayers; k >= 1; --k) {
    __syncthreads();
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int f = 16 * (v / 4) + 4 * q + (v % 4);
        dzs[f][16 * s + col] = (uint16_t)mlp_bf16_bits(zs[k][s][v][lane]);
        hs[f][16 * s + col] = (uint16_t)mlp_bf16_bits(mlp_silu(zs[k - 1][s][v][lane]));
      }
    __syncthreads();
    float* gW = P + kMlpOffHid + (k - 1) * kMlpHidStride;
    // dW[o][in] = sum_s dZ[o][s] H[in][s]: K = 32 samples, slots 8q .. 8q+7
    for (int ro = 0; ro < 4; ++ro) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&dzs[16 * ro + col][8 * q]);
      for (int ri = 0; ri < 4; ++ri) {
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&hs[16 * ri + col][8 * q]);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) gW[(16 * ro + 4 * q + i) * kMlpHid + 16 * ri + col] = acc[i];
      }
    }
    // db[o] = sum_s dZ[o][s] (single precision, from zs); thread o = lane
    {
      const int o = lane, t = o / 16, qo = (o % 16) / 4, i = o % 4;
      float acc = 0.f;
      for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 16; ++c) acc += zs[k][s][4 * t + i][16 * qo + c];
      gW[kMlpHid * kMlpHid + o] = acc;
    }
    // dH_(k-1) = W^T dZ, then dz_(k-1) = dH silu'(z_(k-1)) in place
    for (int s = 0; s < 2; ++s) {
      float dz[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) dz[v] = zs[k][s][v][lane];
      bf16x8 bh[2], bl[2];
      mlp_pack_b(dz, 0, bh[0], bl[0]);
      mlp_pack_b(dz, 1, bh[1], bl[1]);
      const uint4* wt = W.wpt + (k - 1) * 8 * 64;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const bf16x8 a = mlp_as_bf16x8(wt[(2 * r + c) * 64 + lane]);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh[c], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl[c], acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int v = 4 * r + i;
          const float z = zs[k - 1][s][v][lane];
          zs[k - 1][s][v][lane] = acc[i] * mlp_dsilu(z);
        }
      }
    }
  }
  __syncthreads();
  // ---- input layer: dW0[o][j] = sum_s dz0[o][s] f_j[s], db0[o]; thread o = lane
  {
    const int o = lane, t = o / 16, qo = (o % 16) / 4, i = o % 4;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, ab = 0.f;
    for (int s = 0; s < 2; ++s)
      for (int c = 0; c < 16; ++c) {
        const float d = zs[0][s][4 * t + i][16 * qo + c];
        const int smp = 16 * s + c;
        a0 = fmaf(d, fs[0][smp], a0);
        a1 = fmaf(d, fs[1][smp], a1);
        a2 = fmaf(d, fs[2][smp], a2);
        ab += d;
      }
    P[kMlpOffW0 + 3 * o + 0] = a0;
    P[kMlpOffW0 + 3 * o + 1] = a1;
    P[kMlpOffW0 + 3 * o + 2] = a2;
    P[kMlpOffB0 + o] = ab;
  }
}

// Sum the partial gradients in a fixed order; optionally apply one Adam step
// to the FP32 master parameters and publish the evaluation form.
struct AdamArgs {
  float lr, beta1, beta2, eps;
  float bc1, bc2;   // 1 - beta^step
  int apply;
};

__global__ void k_mlp_reduce_adam(const float* __restrict__ partial, int n_parts, float* __restrict__ grad,
                                  float* master, float* m, float* v, AdamArgs a, MlpBuffers B, float last_div) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  float g = 0.f;
  for (int w = 0; w < n_parts; ++w) g += partial[(size_t)w * (kMlpParams + 1) + p];
  grad[p] = p == kMlpParams ? g / last_div : g;
  if (!a.apply || p == kMlpParams) return;
  const float mm = a.beta1 * m[p] + (1.f - a.beta1) * g;
  const float vv = a.beta2 * v[p] + (1.f - a.beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float w = master[p] - a.lr * (mm / a.bc1) / (sqrtf(vv / a.bc2) + a.eps);
  master[p] = w;
  publish_param(p, w, B);
}

}  // namespace marfa

using namespace marfa;

// ------------------------------------------------------------------
// host object
// ------------------------------------------------------------------
// Partial gradients of marfa_surrogate_loss_grad_noalloc: a fixed array of
// the library (one copy per device, alive until the process ends), so that
// entry point allocates nothing.  Host code reaches it only through the
// address hipGetSymbolAddress returns on each device.
constexpr int kNoAllocGroups = 128;
constexpr int64_t kNoAllocMaxSamples = (int64_t)kNoAllocGroups * kGradSamples;  // 4096
static __device__ __align__(256) float scratch[kNoAllocGroups * (kMlpParams + 1)];
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[64];

struct marfa_surrogate {
  int device = 0;
  int32_t chi = 0;
  double cutoff = 0.0;
  int trained = 0;
  double x_max = 0.0;       // largest |x| of the training distribution
  float* master = nullptr;  // FP32 parameters
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;    // [kMlpParams + 1] last reduced gradient and SSE
  MlpBuffers eb;
  float* partial = nullptr;
  int64_t partial_cap = 0;  // workgroups
  float* noalloc_partial = nullptr;  // this device's copy of `scratch`
  hipStream_t stream = nullptr;
};

namespace {

thread_local char g_serr[512];

marfa_status sfail(marfa_status s, const char* msg) {
  std::snprintf(g_serr, sizeof g_serr, "%s", msg);
  marfa_set_error(s, g_serr);
  return s;
}

#define SHIP(expr)                                                             \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) return sfail(MARFA_E_DEVICE, hipGetErrorString(e_)); \
  } while (0)

template <typename T>
marfa_status salloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return sfail(MARFA_E_NOMEM, "device allocation failed");
  }
  return MARFA_OK;
}

MlpDev dev_view(const marfa_surrogate* s) {
  MlpDev W;
  W.w0b = s->eb.w0b;
  W.wp = s->eb.wp;
  W.wpt = s->eb.wpt;
  W.bh = s->eb.bh;
  W.w4 = s->eb.w4;
  W.b4 = s->eb.b4;
  return W;
}

void free_surrogate(marfa_surrogate* s) {
  if (!s) return;
  void* bufs[] = {s->master, s->m, s->v, s->grad, s->eb.w0b, s->eb.wp, s->eb.wpt, s->eb.bh, s->eb.w4, s->eb.b4,
                  s->partial};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

marfa_status ensure_partial(marfa_surrogate* s, int64_t groups) {
  if (groups <= s->partial_cap) return MARFA_OK;
  if (s->partial) (void)hipFree(s->partial);
  s->partial = nullptr;
  s->partial_cap = 0;
  marfa_status st = salloc(&s->partial, (size_t)groups * (kMlpParams + 1));
  if (st == MARFA_OK) s->partial_cap = groups;
  return st;
}

uint64_t host_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// gradient over n samples at [first, first + n) of the permutation
// i -> (a i + b) mod n_all of a sample set of n_all entries
marfa_status run_grad(marfa_surrogate* s, const float* X, const float* T, int64_t n_all, int64_t first, int64_t n,
                      int64_t pa, int64_t pb, float gscale, const AdamArgs& ad, int pow4 = 0) {
  const int64_t groups = (n + kGradSamples - 1) / kGradSamples;
  marfa_status st = ensure_partial(s, groups);
  if (st != MARFA_OK) return st;
  k_mlp_grad<<<(unsigned)groups, 64, 0, s->stream>>>(dev_view(s), X, T, n_all, first, n, pa, pb, gscale, pow4,
                                                     s->partial);
  k_mlp_reduce_adam<<<(kMlpParams + 1 + 255) / 256, 256, 0, s->stream>>>(s->partial, (int)groups, s->grad, s->master,
                                                                         s->m, s->v, ad, s->eb, 1.f);
  SHIP(hipGetLastError());
  return MARFA_OK;
}

marfa_status publish(marfa_surrogate* s) {
  k_mlp_publish<<<(kMlpParams + 255) / 256, 256, 0, s->stream>>>(s->master, s->eb);
  SHIP(hipGetLastError());
  return MARFA_OK;
}

// This device's address of `scratch` (the device must be current): looked up
// once per device, at the first surrogate created on it.
marfa_status noalloc_scratch(int device, float** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= 64) return sfail(MARFA_E_INVALID, "device index out of range");
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return sfail(MARFA_E_DEVICE, "hipGetSymbolAddress(scratch) failed");
    g_scratch_ptr[device] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[device];
  return MARFA_OK;
}

}  // namespace

extern "C" marfa_status marfa_surrogate_create(marfa_surrogate** out, int32_t chi, double cutoff, uint64_t seed,
                                               int32_t device) {
  if (!out) return sfail(MARFA_E_INVALID, "null argument");
  *out = nullptr;
  if (chi == MARFA_CHI_USER)
    return sfail(MARFA_E_UNSUPPORTED, "the learned shape's distance feature is built on the Tonkov chi's first break");
  if (chi != MARFA_CHI_NONE && chi != MARFA_CHI_TONKOV) return sfail(MARFA_E_INVALID, "unknown chi");
  if (!(cutoff > 0.0) || !std::isfinite(cutoff)) return sfail(MARFA_E_INVALID, "cutoff must be > 0");
  marfa_status st = marfa_use_device(device);
  if (st != MARFA_OK) return st;
  marfa_surrogate* s = new marfa_surrogate;
  s->device = device;
  s->chi = chi;
  s->cutoff = cutoff;
#define SALLOC(p, n)                            \
  do {                                          \
    st = salloc(&(p), (n));                     \
    if (st != MARFA_OK) { free_surrogate(s); return st; } \
  } while (0)
  SALLOC(s->master, kMlpParams);
  SALLOC(s->m, kMlpParams);
  SALLOC(s->v, kMlpParams);
  SALLOC(s->grad, kMlpParams + 1);
  SALLOC(s->eb.w0b, kMlpHid);
  SALLOC(s->eb.wp, kMlpHidLayers * 8 * 64);
  SALLOC(s->eb.wpt, kMlpHidLayers * 8 * 64);
  SALLOC(s->eb.bh, kMlpHidLayers * kMlpHid);
  SALLOC(s->eb.w4, kMlpHid);
  SALLOC(s->eb.b4, 1);
#undef SALLOC
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    free_surrogate(s);
    return sfail(MARFA_E_DEVICE, "stream create");
  }
  st = noalloc_scratch(device, &s->noalloc_partial);
  if (st != MARFA_OK) {
    free_surrogate(s);
    return st;
  }
  // Glorot-uniform weights from a counter-based generator, zero biases
  std::vector<float> P(kMlpParams, 0.0f);
  auto uni = [&](uint64_t k) { return (double)(host_mix(seed ^ host_mix(k)) >> 11) * 0x1.0p-53 * 2.0 - 1.0; };
  uint64_t k = 0;
  for (int o = 0; o < kMlpHid; ++o)
    for (int i = 0; i < kMlpIn; ++i) P[kMlpOffW0 + o * kMlpIn + i] = (float)(uni(k++) * std::sqrt(6.0 / (3 + 64)));
  for (int l = 0; l < kMlpHidLayers; ++l)
    for (int j = 0; j < kMlpHid * kMlpHid; ++j)
      P[kMlpOffHid + l * kMlpHidStride + j] = (float)(uni(k++) * std::sqrt(6.0 / 128.0));
  for (int i = 0; i < kMlpHid; ++i) P[kMlpOffW4 + i] = (float)(uni(k++) * std::sqrt(6.0 / 65.0));
  st = marfa_surrogate_set_params(s, P.data(), kMlpParams);
  if (st != MARFA_OK) {
    free_surrogate(s);
    return st;
  }
  *out = s;
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_set_params(marfa_surrogate* s, const float* params, int64_t n) {
  if (!s || !params) return sfail(MARFA_E_INVALID, "null argument");
  if (n != kMlpParams) return sfail(MARFA_E_INVALID, "parameter count must be 12801");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return sfail(MARFA_E_INVALID, "non-finite parameter");
  SHIP(hipSetDevice(s->device));
  // plans may have queued work on other streams that reads the evaluation
  // form rewritten below: let every enqueued kernel of the device finish first
  SHIP(hipDeviceSynchronize());
  SHIP(hipMemcpyAsync(s->master, params, n * sizeof(float), hipMemcpyHostToDevice, s->stream));
  SHIP(hipMemsetAsync(s->m, 0, n * sizeof(float), s->stream));
  SHIP(hipMemsetAsync(s->v, 0, n * sizeof(float), s->stream));
  // the evaluation form is rebuilt entirely, so stale bits never survive
  SHIP(hipMemsetAsync(s->eb.wp, 0, kMlpHidLayers * 8 * 64 * sizeof(uint4), s->stream));
  SHIP(hipMemsetAsync(s->eb.wpt, 0, kMlpHidLayers * 8 * 64 * sizeof(uint4), s->stream));
  marfa_status st = publish(s);
  if (st != MARFA_OK) return st;
  SHIP(hipStreamSynchronize(s->stream));
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_get_params(const marfa_surrogate* s, float* params, int64_t n) {
  if (!s || !params) return sfail(MARFA_E_INVALID, "null argument");
  if (n != kMlpParams) return sfail(MARFA_E_INVALID, "parameter count must be 12801");
  SHIP(hipSetDevice(s->device));
  SHIP(hipStreamSynchronize(s->stream));
  SHIP(hipMemcpy(params, s->master, n * sizeof(float), hipMemcpyDeviceToHost));
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_load(marfa_surrogate* s, const float* params, int64_t n, double x_max) {
  if (!s || !params) return sfail(MARFA_E_INVALID, "null argument");
  if (!(std::isfinite(x_max) && x_max > 0.0)) return sfail(MARFA_E_INVALID, "x_max must be finite and > 0");
  const marfa_status st = marfa_surrogate_set_params(s, params, n);
  if (st != MARFA_OK) return st;
  s->x_max = x_max;
  s->trained = 1;
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_save(const marfa_surrogate* s, float* params, int64_t n, double* x_max) {
  if (!s || !params || !x_max) return sfail(MARFA_E_INVALID, "null argument");
  if (!s->trained) return sfail(MARFA_E_UNSUPPORTED, "the surrogate is not trained");
  const marfa_status st = marfa_surrogate_get_params(s, params, n);
  if (st != MARFA_OK) return st;
  *x_max = s->x_max;
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_forward(marfa_surrogate* s, const float* X, int64_t n, float* out,
                                                void* stream) {
  if (!s || (n > 0 && (!X || !out))) return sfail(MARFA_E_INVALID, "null argument");
  if (n < 0) return sfail(MARFA_E_INVALID, "n < 0");
  if (n == 0) return MARFA_OK;
  SHIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  SHIP(hipStreamSynchronize(s->stream));
  k_mlp_forward<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(dev_view(s), X, n, out);
  SHIP(hipGetLastError());
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_loss_grad(marfa_surrogate* s, const float* X, const float* T, int64_t n,
                                                  float* loss, float* grad) {
  if (!s || !X || !T || !loss || !grad) return sfail(MARFA_E_INVALID, "null argument");
  if (n < 1) return sfail(MARFA_E_INVALID, "n < 1");
  SHIP(hipSetDevice(s->device));
  AdamArgs ad{0.f, 0.f, 0.f, 0.f, 1.f, 1.f, 0};
  marfa_status st = run_grad(s, X, T, n, 0, n, 1, 0, 2.0f / (float)n, ad);
  if (st != MARFA_OK) return st;
  std::vector<float> g(kMlpParams + 1);
  SHIP(hipMemcpyAsync(g.data(), s->grad, g.size() * sizeof(float), hipMemcpyDeviceToHost, s->stream));
  SHIP(hipStreamSynchronize(s->stream));
  std::memcpy(grad, g.data(), kMlpParams * sizeof(float));
  *loss = g[kMlpParams] / (float)n;
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_loss_grad_noalloc(marfa_surrogate* s, const float* X, const float* T,
                                                          int64_t n, float* out, void* stream) {
  if (!s || !X || !T || !out) return sfail(MARFA_E_INVALID, "null argument");
  if (n < 1 || n > kNoAllocMaxSamples)
    return sfail(MARFA_E_INVALID, "n must be in [1, 4096]: the fixed partial-gradient array holds 128 workgroups");
  if (!s->noalloc_partial) return sfail(MARFA_E_STATE, "no partial-gradient array on this device");
  SHIP(hipSetDevice(s->device));
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  const int64_t groups = (n + kGradSamples - 1) / kGradSamples;
  // the same kernels and fixed summation order as marfa_surrogate_loss_grad;
  // every read row of the array is written first by this call's k_mlp_grad
  k_mlp_grad<<<(unsigned)groups, 64, 0, hs>>>(dev_view(s), X, T, n, 0, n, 1, 0, 2.0f / (float)n, 0,
                                              s->noalloc_partial);
  AdamArgs ad{0.f, 0.f, 0.f, 0.f, 1.f, 1.f, 0};
  k_mlp_reduce_adam<<<(kMlpParams + 1 + 255) / 256, 256, 0, hs>>>(s->noalloc_partial, (int)groups, out, s->master,
                                                                   s->m, s->v, ad, s->eb, (float)n);
  SHIP(hipGetLastError());
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_make_samples(marfa_surrogate* s, const marfa_sample_cfg* c, uint64_t seed,
                                                     int64_t n, float* X, float* T, void* stream) {
  if (!s || !c || (n > 0 && (!X || !T))) return sfail(MARFA_E_INVALID, "null argument");
  if (n < 0) return sfail(MARFA_E_INVALID, "n < 0");
  if (!(c->nu_lo > 0.0) || !(c->nu_hi >= c->nu_lo) || !(c->T_lo > 0.0) || !(c->T_hi >= c->T_lo) ||
      !(c->molar_mass_g > 0.0))
    return sfail(MARFA_E_INVALID, "sample ranges must be positive and ordered");
  SHIP(hipSetDevice(s->device));
  MlpSampleCfg mc{c->nu_lo, c->nu_hi, c->T_lo, c->T_hi, c->molar_mass_g, (double)kMlpYMin, (double)kMlpYMax,
                  s->cutoff, s->chi, 0};
  launch_mlp_samples(mc, seed, n, X, T, device_tables(s->device), (hipStream_t)stream);
  SHIP(hipGetLastError());
  return MARFA_OK;
}

extern "C" marfa_status marfa_surrogate_train(marfa_surrogate* s, const marfa_sample_cfg* c,
                                              const marfa_train_cfg* cfg, marfa_train_report* rep) {
  if (!s || !c || !cfg || !rep) return sfail(MARFA_E_INVALID, "null argument");
  if (cfg->n_train < kGradSamples || cfg->n_val < 1 || cfg->epochs < 1 || cfg->batch < kGradSamples ||
      cfg->batch % kGradSamples != 0 || !(cfg->lr_max > 0.f) || !(cfg->lr_min >= 0.f) ||
      (cfg->loss_power != 2 && cfg->loss_power != 4))
    return sfail(MARFA_E_INVALID, "training configuration");
  SHIP(hipSetDevice(s->device));
  // training rewrites the weights that queued plan launches may still read
  SHIP(hipDeviceSynchronize());
  const auto t0 = std::chrono::steady_clock::now();
  std::memset(rep, 0, sizeof *rep);
  const int64_t N = cfg->n_train, V = cfg->n_val;
  float *X = nullptr, *T = nullptr, *Xv = nullptr, *Tv = nullptr, *pv = nullptr;
  marfa_status st = salloc(&X, (size_t)N * 3);
  if (st == MARFA_OK) st = salloc(&T, (size_t)N);
  if (st == MARFA_OK) st = salloc(&Xv, (size_t)V * 3);
  if (st == MARFA_OK) st = salloc(&Tv, (size_t)V);
  if (st == MARFA_OK) st = salloc(&pv, (size_t)V);
  auto cleanup = [&]() {
    for (void* b : {(void*)X, (void*)T, (void*)Xv, (void*)Tv, (void*)pv})
      if (b) (void)hipFree(b);
  };
  if (st != MARFA_OK) { cleanup(); return st; }
  st = marfa_surrogate_make_samples(s, c, cfg->seed, N, X, T, s->stream);
  if (st == MARFA_OK) st = marfa_surrogate_make_samples(s, c, cfg->seed ^ 0x5bd1e995ull, V, Xv, Tv, s->stream);
  if (st != MARFA_OK) { cleanup(); return st; }
  // a fresh optimizer state for every run
  if (hipMemsetAsync(s->m, 0, kMlpParams * sizeof(float), s->stream) != hipSuccess ||
      hipMemsetAsync(s->v, 0, kMlpParams * sizeof(float), s->stream) != hipSuccess) {
    cleanup();
    return sfail(MARFA_E_DEVICE, "optimizer reset");
  }
  const int64_t steps_per_epoch = N / cfg->batch;
  const int64_t total = steps_per_epoch * cfg->epochs;
  const int64_t warm = std::max<int64_t>(1, total / 50);
  const float b1 = 0.9f, b2 = 0.999f;
  double pb1 = 1.0, pb2 = 1.0;
  int64_t step = 0;
  for (int ep = 0; ep < cfg->epochs && st == MARFA_OK; ++ep) {
    // a fresh affine permutation of the training set each epoch
    int64_t pa = (int64_t)(host_mix(cfg->seed + 17 * (uint64_t)ep) % (uint64_t)N) | 1;
    while (std::gcd(pa, N) != 1) pa += 2;
    const int64_t pbo = (int64_t)(host_mix(cfg->seed + 31 * (uint64_t)ep) % (uint64_t)N);
    for (int64_t b = 0; b < steps_per_epoch && st == MARFA_OK; ++b, ++step) {
      float lr;
      if (step < warm) lr = cfg->lr_max * (float)(step + 1) / (float)warm;
      else {
        const double u = (double)(step - warm) / (double)std::max<int64_t>(1, total - warm);
        lr = (float)(cfg->lr_min + 0.5 * (cfg->lr_max - cfg->lr_min) * (1.0 + std::cos(M_PI * u)));
      }
      pb1 *= b1;
      pb2 *= b2;
      AdamArgs ad{lr, b1, b2, 1e-8f, (float)(1.0 - pb1), (float)(1.0 - pb2), 1};
      st = run_grad(s, X, T, N, b * cfg->batch, cfg->batch, pa, pbo, 2.0f / (float)cfg->batch, ad,
                    cfg->loss_power == 4 ? 1 : 0);
    }
  }
  if (st == MARFA_OK) {
    float g[1];
    hipError_t e = hipMemcpyAsync(g, s->grad + kMlpParams, sizeof(float), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) st = sfail(MARFA_E_DEVICE, hipGetErrorString(e));
    rep->train_loss = g[0] / (float)cfg->batch;
  }
  if (st == MARFA_OK) {
    k_mlp_forward<<<(unsigned)((V + 255) / 256), 256, 0, s->stream>>>(dev_view(s), Xv, V, pv);
    std::vector<float> a(V), b(V);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(a.data(), pv, V * sizeof(float), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.data(), Tv, V * sizeof(float), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) st = sfail(MARFA_E_DEVICE, hipGetErrorString(e));
    double mx = 0.0, sum = 0.0, sq = 0.0;
    for (int64_t i = 0; i < V && st == MARFA_OK; ++i) {
      const double d = std::fabs((double)a[i] - (double)b[i]);
      mx = std::max(mx, d);
      sum += d;
      sq += d * d;
    }
    rep->val_max_abs = (float)mx;
    rep->val_mean_abs = (float)(sum / (double)V);
    rep->val_loss = (float)(sq / (double)V);
  }
  cleanup();
  if (st != MARFA_OK) return st;
  rep->steps = step;
  rep->ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  // largest x of the training distribution: the full cut-off at the narrowest
  // Doppler width
  const double aD_min = c->nu_lo / 299792458.0 *
                        std::sqrt(2.0 * 0.693147180559945309417 * 1.380649e-23 * 6.02214076e23 * c->T_lo /
                                  (c->molar_mass_g * 1e-3));
  s->x_max = std::sqrt(0.693147180559945309417) * s->cutoff / aD_min;
  rep->x_max = s->x_max;
  s->trained = 1;
  return MARFA_OK;
}

extern "C" void marfa_surrogate_destroy(marfa_surrogate* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  free_surrogate(s);
}

// view for the level kernel
bool marfa_surrogate_view(const marfa_surrogate* s, MlpDev* W, double* x_max, int32_t* chi, double* cutoff,
                          int* device) {
  if (!s || !s->trained) return false;
  *W = dev_view(s);
  *x_max = s->x_max;
  *chi = s->chi;
  *cutoff = s->cutoff;
  *device = s->device;
  return true;
}
