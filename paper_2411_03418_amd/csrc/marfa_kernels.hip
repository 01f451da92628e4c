// marfa_kernels.hip -- gfx950 kernels of the eleven-grid line-by-line library.
//
// Paper: MARFA (arXiv 2411.03418).  What is computed:
//   sigma(nu) = sum_j S_j(T) f_j(nu - nu~0_j) chi(|nu - nu~0_j|), |nu - nu~0_j| <= cutoff
//     (Eq.(3), Section 2.1; chi of Eq.(10), Section 2.3)
// with the eleven-grid scheme of Section 2.4: every line is split into a
// central part on its start level and annular wing parts on coarser levels;
// the eleven level arrays are interpolated coarse to fine with 3-point
// Lagrange stencils.  Jumps of a line's coarse-level part (its inner edge, the
// cut-off, chi breakpoints) are corrected exactly on bands of finer-level
// nodes (our reading; the paper defers the details to Fomin 1995).
//
// Kernels (all launched on the caller's stream, captured into one HIP graph):
//   k_fill_*          clear counters and maxima (graph-safe, no memset nodes)
//   k_layer_const     per-layer factors of the FP64 line preparation
//   k_prep_smax       FP64 S(T) per (line, layer), max per layer
//   k_prep_count      per-block counts of kept lines by start level
//   k_prep_scan       exclusive offsets per (layer, start level)
//   k_prep_scatter    FP64 placement nu~0*2048 -> (int k0, frac) and the
//                     compacted per-layer line records, grouped by start level
//   k_prep_bucket     per-layer index: first kept line at or above each
//                     1/256 cm^-1 bucket (one thread per line fills its gap)
//   k_layer_scale     output scale per layer (max S(T), number density)
//   k_level           persistent work queue over (layer, level, node tile):
//                     each lane owns one level node and sums the contributions
//                     of the lines in its windows (wave-uniform line loads)
//   k_cascade         3-, 4- or 5-point interpolation from level l+1 into level l,
//                     one thread per coarse cell with compile-time weights
//                     (k_cascade_out: level 0 in single precision, four
//                     aligned output nodes per thread);
//                     the level-0 pass applies the layer scale and writes out.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "marfa_device.h"

namespace marfa {

// ------------------------------------------------------------------
// fills
// ------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u32(unsigned int* p, int64_t n, unsigned int v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------
// line preparation (FP64)
// ------------------------------------------------------------------

struct LineState {
  double S, gL, aD, nut;
};

// HITRAN forms: S(T) = S296 Q(296)/Q(T) exp(-c2 E''(1/T - 1/296))
//   (1 - exp(-c2 nu/T))/(1 - exp(-c2 nu/296));
// gamma_L = (296/T)^n (gamma_air (p - p_self) + gamma_self p_self);
// alpha_D = nu/c sqrt(2 ln2 k_B T N_A / M);  nu~0 = nu0 + delta_air p.
// The factors that depend on the layer alone are formed once per layer:
// c = {p, p_self, Q(296)/Q(T), c2 (1/T - 1/296), ln(296/T), c2/T,
//      sqrt(2 ln2 k_B N_A T / M)/c_light, 296/T}.
constexpr int kLayerConst = 8;
__global__ void k_layer_const(const double* __restrict__ layers, int nL, double molar_mass, double* lc) {
  const int L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= nL) return;
  const double p = layers[4 * L], T = layers[4 * L + 1], ps = layers[4 * L + 2], q = layers[4 * L + 3];
  double* c = lc + kLayerConst * L;
  c[0] = p;
  c[1] = ps;
  c[2] = q > 0.0 ? q : kTref / T;
  c[3] = kC2 * (1.0 / T - 1.0 / kTref);
  c[4] = log(kTref / T);
  c[5] = kC2 / T;
  c[6] = sqrt(2.0 * kLn2d * kBoltzmann * kNA * T / (molar_mass * 1e-3)) / kCLight;
  c[7] = kTref / T;
}

__device__ __forceinline__ LineState line_state(const LineIn& in, int64_t j, const double* __restrict__ c) {
  constexpr double kC2Tref = kC2 / kTref;
  const double nu = in.nu0[j];
  const double boltz = exp(-(double)in.El[j] * c[3]);
  const double stim = nu > 0.0 ? expm1(-nu * c[5]) / expm1(-nu * kC2Tref) : c[7];
  LineState s;
  s.S = (double)in.S296[j] * c[2] * boltz * stim;
  s.gL = exp((double)in.nair[j] * c[4]) * ((double)in.gair[j] * (c[0] - c[1]) + (double)in.gself[j] * c[1]);
  s.aD = nu * c[6];
  s.nut = nu + (double)in.dair[j] * c[0];
  return s;
}

// Grid-stride over the layer's lines (a few dozen blocks per layer), so that
// only that many atomics per layer meet on its maximum.
__global__ void k_prep_smax(LineIn in, const double* __restrict__ lc, unsigned long long* smax) {
  __shared__ double wmax[4];
  const int L = blockIdx.y;
  double S = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < in.n; j += (int64_t)gridDim.x * 256)
    S = fmax(S, line_state(in, j, lc + kLayerConst * L).S);
  // wavefront maximum by butterfly shuffles, then the block's four
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) S = fmax(S, __shfl_xor(S, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = S;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    if (m > 0.0) atomicMax(&smax[L], (unsigned long long)__double_as_longlong(m));
  }
}

__device__ __forceinline__ int start_level(double w, double R, const Geometry& G) {
  // largest l with R h_l <= w, 0 if none (w in cm, h_l = r_l / 2048)
  double wf = w * 2048.0;
  int s = 0;
#pragma unroll
  for (int l = 0; l < kLevels; ++l)
    if (R * (double)G.r[l] <= wf) s = l;
  return s;
}

// start level of a kept line, kGroups if pruned
__device__ __forceinline__ int line_key(const LineIn& in, int64_t j, const double* lc, double smax,
                                        double prune, double R, const Geometry& G, LineState& st) {
  st = line_state(in, j, lc);
  bool keep = prune <= 0.0 || st.S >= prune * smax;
  if (!keep) return kGroups;
  return start_level(fmax(st.gL, st.aD), R, G);
}

__global__ void k_prep_count(LineIn in, Geometry G, PrepArgs pa, int nblk) {
  __shared__ int cnt[kGroups + 1];
  if (threadIdx.x <= kGroups) cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int L = blockIdx.y;
  if (i < in.n) {
    const int64_t j = pa.perm[(int64_t)L * in.n + i];
    LineState st;
    int key = line_key(in, j, pa.lc + kLayerConst * L, __longlong_as_double((long long)pa.smax[L]), pa.prune, pa.R, G,
                       st);
    atomicAdd(&cnt[key], 1);
  }
  __syncthreads();
  int64_t blk = (int64_t)L * nblk + blockIdx.x;
  if (threadIdx.x <= kGroups) pa.scount[blk * (kGroups + 1) + threadIdx.x] = cnt[threadIdx.x];
  if (threadIdx.x == 0) {
    int k = 0;
    for (int g = 0; g < kGroups; ++g) k += cnt[g];
    pa.bcount[blk] = k;
  }
}

// exclusive offsets of kept lines over blocks (in place), kept totals, and
// lines per start level of each layer
__global__ void k_prep_scan(PrepArgs pa, int nblk) {
  __shared__ int part[256];
  __shared__ int gpart[kGroups + 1][256];
  int L = blockIdx.x;
  int t = threadIdx.x;
  int chunk = (nblk + 255) / 256;
  int b0 = t * chunk, b1 = min(nblk, b0 + chunk);
  int s = 0;
  int gs[kGroups + 1];
#pragma unroll
  for (int g = 0; g <= kGroups; ++g) gs[g] = 0;
  for (int b = b0; b < b1; ++b) {
    const int64_t k = (int64_t)L * nblk + b;
    s += pa.bcount[k];
#pragma unroll
    for (int g = 0; g <= kGroups; ++g) gs[g] += pa.scount[k * (kGroups + 1) + g];
  }
  part[t] = s;
#pragma unroll
  for (int g = 0; g <= kGroups; ++g) gpart[g][t] = gs[g];
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int v = (t >= o) ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int b = b0; b < b1; ++b) {
    int64_t k = (int64_t)L * nblk + b;
    int v = pa.bcount[k];
    pa.bcount[k] = run;
    run += v;
  }
  if (t == 255) pa.kept[L] = part[255];
  if (t <= kGroups) {
    int c = 0;
    for (int k = 0; k < 256; ++k) c += gpart[t][k];
    pa.gcount[L * (kGroups + 1) + t] = c;
  }
}

template <typename R>
__global__ void k_prep_scatter(LineIn in, Geometry G, PrepArgs pa, int nblk) {
  __shared__ int wcnt[4];
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int L = blockIdx.y;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double sm = __longlong_as_double((long long)pa.smax[L]);
  int key = kGroups;
  LineState st{0, 0, 0, 0};
  int64_t j = 0;
  if (i < in.n) {
    j = pa.perm[(int64_t)L * in.n + i];
    key = line_key(in, j, pa.lc + kLayerConst * L, sm, pa.prune, pa.R, G, st);
  }
  bool keep = key < kGroups;
  unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long m = __ballot(keep);
  int rank = __popcll(m & lt);
  if (lane == 0) wcnt[wv] = __popcll(m);
  __syncthreads();
  if (!keep) return;
  int off = rank;
  for (int w = 0; w < wv; ++w) off += wcnt[w];
  int64_t dest = (int64_t)pa.bcount[(int64_t)L * nblk + blockIdx.x] + off;
  int64_t base = (int64_t)L * in.n;
  // FP64 placement of the shifted centre on the finest lattice
  double t = st.nut * 2048.0;
  double k0 = floor(t);
  typename RecOf<R>::T r;
  R fr = R(t - k0);
  if (fr >= R(1)) { k0 += 1.0; fr = R(0); }
  r.k0 = (int32_t)k0;
  r.frac = fr;
  const double sp = sm > 0.0 ? st.S / sm : 0.0;
  r.A = generic_shape(G) ? R(sp) : R(sp * st.gL * kInvPi);
  r.gam = R(st.gL);
  if constexpr (sizeof(R) == 8) r.gam2 = R(st.gL * st.gL);
  // the Lorentz shape is the Voigt wing with alpha_D = 0
  const bool lor = G.shape == MARFA_SHAPE_LORENTZ;
  r.ae = lor ? R(0) : R(st.aD * st.aD / (2.0 * kLn2d));
  const double xs = (st.aD > 0.0 && !lor) ? sqrt(kLn2d) / st.aD : 0.0;
  r.xs = R(xs);
  r.amp = R(sp * xs * kInvSqrtPi);
  r.s = key;
  reinterpret_cast<typename RecOf<R>::T*>(pa.rec)[base + dest] = r;
  reinterpret_cast<R*>(pa.csp)[base + dest] = R(sp);
  pa.cnu[base + dest] = st.nut;
}

// bucket[b] = first kept line with nu~0 >= v_b = origin + b / kBucketPerCm
// (per layer; bucket[nbucket] = kept): thread i writes the buckets with
// nu~0_(i-1) < v_b <= nu~0_i, found from floor((nu - origin) kBucketPerCm)
// and settled by comparing with v_b itself, so every bucket is written once.
__device__ __forceinline__ double bucket_value(const Geometry& G, int64_t b) {
  return G.bucket_origin + (double)b / kBucketPerCm;
}
__global__ void k_prep_bucket(int64_t n_lines, Geometry G, PrepArgs pa) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int L = blockIdx.y;
  const int64_t kept = pa.kept[L];
  if (i > kept) return;
  const double* cnu = pa.cnu + (int64_t)L * n_lines;
  int32_t* bk = pa.bucket + (int64_t)L * (G.nbucket + 1);
  const int64_t nb = G.nbucket;
  // first bucket with v_b > nu~0_(i-1)
  int64_t b0 = 0;
  if (i > 0) {
    const double lo = cnu[i - 1];
    b0 = (int64_t)floor((lo - G.bucket_origin) * kBucketPerCm) + 1;
    b0 = b0 < 0 ? 0 : (b0 > nb ? nb : b0);
    while (b0 > 0 && bucket_value(G, b0 - 1) > lo) --b0;
    while (b0 < nb && !(bucket_value(G, b0) > lo)) ++b0;
  }
  // last bucket with v_b <= nu~0_i
  int64_t b1 = nb - 1;
  if (i < kept) {
    const double hi = cnu[i];
    b1 = (int64_t)floor((hi - G.bucket_origin) * kBucketPerCm);
    b1 = b1 < -1 ? -1 : (b1 > nb - 1 ? nb - 1 : b1);
    while (b1 + 1 < nb && bucket_value(G, b1 + 1) <= hi) ++b1;
    while (b1 >= 0 && bucket_value(G, b1) > hi) --b1;
  }
  for (int64_t b = b0; b <= b1; ++b) bk[b] = (int32_t)i;
  if (i == kept) bk[nb] = (int32_t)kept;
}

// Position of line i in the order of shifted centres nu~0 = nu0 + delta p
// (ties by index).  Lines are sorted by nu0 and |(delta_i - delta_j) p| <=
// span, so only neighbours within span of nu0 can change places.
__global__ void k_rank(LineIn in, const double* __restrict__ layers, const double* __restrict__ span,
                       int32_t* perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int L = blockIdx.y;
  if (i >= in.n) return;
  const double p = layers[4 * L];
  const double sp = span[L];
  const double ni = in.nu0[i];
  const double ti = ni + (double)in.dair[i] * p;
  int64_t rank = i;
  for (int64_t j = i + 1; j < in.n && in.nu0[j] <= ni + sp; ++j) {
    const double tj = in.nu0[j] + (double)in.dair[j] * p;
    if (tj < ti) ++rank;
  }
  for (int64_t j = i - 1; j >= 0 && in.nu0[j] >= ni - sp; --j) {
    const double tj = in.nu0[j] + (double)in.dair[j] * p;
    if (tj > ti) --rank;
  }
  perm[(int64_t)L * in.n + rank] = (int32_t)i;
}

__global__ void k_layer_scale(const double* __restrict__ layers, const unsigned long long* smax, int nL,
                              int out_kind, double* scale) {
  int L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= nL) return;
  double s = __longlong_as_double((long long)smax[L]);
  if (out_kind == MARFA_OUT_K_PER_KM) {
    double n = layers[4 * L + 2] * kAtmPa / (kBoltzmann * layers[4 * L + 1]) * 1e-6;
    s *= n * 1e5;
  }
  scale[L] = s;
}

// ------------------------------------------------------------------
// cascade: A_l += P(A_(l+1)); level 0 also scales into the output
// ------------------------------------------------------------------
// Interpolation weights of the cascade, fixed at compile time: fine node j
// (0 <= j < RHO) of coarse cell q takes sum_e w(j, e) A[q - kCascL + e] over
// the window e = 0 .. kCascL + kCascR.  Injection at j = 0; the 3- and
// 5-point rules centre on the nearest coarse node (ties to the left), the
// 4-point rule uses q - 1 .. q + 2.
template <int NS>
constexpr int kCascL = NS == 5 ? 2 : 1;
template <int NS>
constexpr int kCascR = NS == 5 ? 3 : 2;
template <int RHO, int NS>
struct CascadeStencil {
  double w[RHO][kCascL<NS> + kCascR<NS> + 1] = {};
  bool used[RHO][kCascL<NS> + kCascR<NS> + 1] = {};
  constexpr CascadeStencil() {
    constexpr int WL = kCascL<NS>;
    w[0][WL] = 1.0;
    used[0][WL] = true;
    for (int j = 1; j < RHO; ++j) {
      const double f = (double)j / (double)RHO;
      if (NS == 4) {
        for (int k = -1; k <= 2; ++k) {
          w[j][WL + k] = lagrange_w4(k, f);
          used[j][WL + k] = true;
        }
      } else {
        const int kc = f <= 0.5 ? 0 : 1;
        const double t = f - kc;
        constexpr int H = NS == 5 ? 2 : 1;
        for (int k = -H; k <= H; ++k) {
          w[j][WL + kc + k] = lagrange_w<H>(k, t);
          used[j][WL + kc + k] = true;
        }
      }
    }
  }
};

// Level l from level l+1 (ratio RHO = 2 or 4, NS-point stencil): one thread
// per coarse cell q holds the coarse window once and writes the RHO fine nodes
// m = RHO q + j that lie in level l's range; level 0 gets the layer's scale.
template <typename R, int RHO, int NS>
__global__ void __launch_bounds__(256) k_cascade(Geometry G, int l, R* A, R* out, int64_t stride,
                                                 const double* scale) {
  constexpr CascadeStencil<RHO, NS> S{};
  constexpr int WL = kCascL<NS>, NW = kCascL<NS> + kCascR<NS> + 1;
  const int layer = blockIdx.y;
  const int64_t lo = G.lo[l], hi = G.lo[l] + G.n[l];
  const int64_t q = floor_div(lo, RHO) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m0 = q * RHO;
  if (m0 >= hi) return;
  const R* Ac = A + (int64_t)layer * G.a_total + G.aoff[l + 1] - G.lo[l + 1];
  const R sc = l == 0 ? R(scale[layer]) : R(1);
  bool in[RHO];
#pragma unroll
  for (int j = 0; j < RHO; ++j) in[j] = m0 + j >= lo && m0 + j < hi;
  // the window entries some in-range node reads (all of them inside the range)
  R c[NW];
#pragma unroll
  for (int e = 0; e < NW; ++e) {
    bool need = false;
#pragma unroll
    for (int j = 0; j < RHO; ++j) need = need || (in[j] && S.used[j][e]);
    c[e] = need ? Ac[q - WL + e] : R(0);
  }
#pragma unroll
  for (int j = 0; j < RHO; ++j) {
    if (!in[j]) continue;
    R v;
    if (j == 0) {
      v = c[WL];
    } else {
      v = R(0);
#pragma unroll
      for (int e = 0; e < NW; ++e)
        if (S.used[j][e]) v += R(S.w[j][e]) * c[e];
    }
    const int64_t i = m0 + j - lo;
    if (l > 0) {
      A[(int64_t)layer * G.a_total + G.aoff[l] + i] += v;
    } else {
      R* o = out + (int64_t)layer * stride + i;
      *o = sc * (*o + v);
    }
  }
}

// Value interpolated at fine node rem (0 .. 3) of a ratio-4 cell whose
// window starts at c (only the entries the node's stencil uses are read).
template <int NS, int REM>
__device__ __forceinline__ float cascade_node4(const float* __restrict__ c) {
  constexpr CascadeStencil<4, NS> S{};
  constexpr int NW = kCascL<NS> + kCascR<NS> + 1;
  if constexpr (REM == 0) {
    return c[kCascL<NS>];
  } else {
    float v = 0.0f;
#pragma unroll
    for (int e = 0; e < NW; ++e)
      if (S.used[REM][e]) v += float(S.w[REM][e]) * c[e];
    return v;
  }
}

// The four nodes of one aligned group: node k sits at REM = (PH + k) mod 4 of
// cell qa + (PH + k) / 4.  Only the window entries some node uses are loaded.
template <int NS, int PH>
__device__ __forceinline__ void cascade_group4(const float* __restrict__ Ac, int64_t qa, float (&v)[4]) {
  constexpr CascadeStencil<4, NS> S{};
  constexpr int WL = kCascL<NS>, NW = kCascL<NS> + kCascR<NS> + 1;
  float c[NW + 1];
#pragma unroll
  for (int e = 0; e <= NW; ++e) {
    bool need = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = (PH + k) & 3, co = (PH + k) >> 2;
      if (e - co >= 0 && e - co < NW) need = need || S.used[r][e - co];
    }
    c[e] = need ? Ac[qa - WL + e] : 0.0f;
  }
  v[0] = cascade_node4<NS, (PH + 0) & 3>(c + ((PH + 0) >> 2));
  v[1] = cascade_node4<NS, (PH + 1) & 3>(c + ((PH + 1) >> 2));
  v[2] = cascade_node4<NS, (PH + 2) & 3>(c + ((PH + 2) >> 2));
  v[3] = cascade_node4<NS, (PH + 3) & 3>(c + ((PH + 3) >> 2));
}

// Level 0 of the single-precision cascade (ratio 4) with 16-byte output
// accesses: thread t owns output nodes i0 + 4t .. i0 + 4t + 3, where i0 puts
// the group on a 16-byte boundary of the layer's output row, so the phase
// PH = (lo + i0) mod 4 of its nodes within their coarse cells is the same for
// the whole layer and every weight is a constant.  Threads past the groups
// take the (at most six) nodes before i0 and after the last group one each.
template <int NS>
__global__ void __launch_bounds__(256) k_cascade_out(Geometry G, const float* A, float* out, int64_t stride,
                                                     const double* scale) {
  const int layer = blockIdx.y;
  const int64_t lo = G.lo[0], n = G.n[0];
  float* row = out + (int64_t)layer * stride;
  const int64_t i0 = (int64_t)((4 - (((uintptr_t)row >> 2) & 3)) & 3);
  const int64_t ngrp = n > i0 ? (n - i0) / 4 : 0;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float* Ac = A + (int64_t)layer * G.a_total + G.aoff[1] - G.lo[1];
  const float sc = float(scale[layer]);
  if (t < ngrp) {
    const int64_t i = i0 + 4 * t;
    const int64_t m = lo + i;   // level-0 nodes are at or above 0
    float v[4];
    switch ((int)(m & 3)) {
      case 0: cascade_group4<NS, 0>(Ac, m >> 2, v); break;
      case 1: cascade_group4<NS, 1>(Ac, m >> 2, v); break;
      case 2: cascade_group4<NS, 2>(Ac, m >> 2, v); break;
      default: cascade_group4<NS, 3>(Ac, m >> 2, v); break;
    }
    float4* o = reinterpret_cast<float4*>(row + i);
    float4 w = *o;
    w.x = sc * (w.x + v[0]);
    w.y = sc * (w.y + v[1]);
    w.z = sc * (w.z + v[2]);
    w.w = sc * (w.w + v[3]);
    *o = w;
    return;
  }
  // single nodes: k = 0 .. 5 -> the head (k < i0) or the tail after the groups
  const int64_t k = t - ngrp;
  if (k >= 6) return;
  const int64_t head = i0 < n ? i0 : n;
  const int64_t i = k < 3 ? k : i0 + 4 * ngrp + (k - 3);
  if (k < 3 ? i >= head : i >= n) return;
  const int64_t m = lo + i;
  constexpr int WL = kCascL<NS>;
  const float* c = Ac + (m >> 2) - WL;
  float v;
  switch ((int)(m & 3)) {
    case 0: v = cascade_node4<NS, 0>(c); break;
    case 1: v = cascade_node4<NS, 1>(c); break;
    case 2: v = cascade_node4<NS, 2>(c); break;
    default: v = cascade_node4<NS, 3>(c); break;
  }
  row[i] = sc * (row[i] + v);
}

// K(x, y) through the hot-path shape code: a line with alpha_D = sqrt(ln 2)
// (so x = d and y = gamma_L in cm^-1) and unit intensity has F = K / sqrt(pi)
template <typename R>
__device__ double device_K(double x, double y, const DeviceTables* tabs) {
  typename RecOf<R>::T L{};
  L.k0 = 0; L.frac = 0; L.A = R(y * kInvPi);
  L.gam = R(y);
  if constexpr (sizeof(R) == 8) L.gam2 = R(y) * R(y);
  L.amp = R(kInvSqrtPi);
  L.ae = R(0.5); L.xs = R(1); L.s = 0;
  Geometry G{};
  G.weid = tabs->weid;
  G.ktab = reinterpret_cast<const float4*>(tabs->taylor);
  G.shape = MARFA_SHAPE_VOIGT;
  G.chi = MARFA_CHI_NONE;
  Counts c{0, 0, 0, 0, 0};
  R d = R(x) * R(2048);  // fine units
  R f = line_value<R, false>(d, L, R(1), G, R(INFINITY), c);
  return (double)f * 1.772453850905516;
}

// device Voigt for tests
template <typename R>
__global__ void k_voigt_eval(int64_t n, const double* x, const double* y, double* out, const DeviceTables* tabs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = device_K<R>(x[i], y[i], tabs);
}

// ------------------------------------------------------------------
// training samples of the learned line shape
// ------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double uniform01(uint64_t seed, uint64_t ctr) {
  return (double)(splitmix64(seed ^ splitmix64(ctr)) >> 11) * 0x1.0p-53;
}

// Sample i: a line centre nu0 and temperature T uniform over the configured
// ranges (alpha_D from Section 2.2's Doppler width), y log-uniform, and the
// distance |d| from a mixture -- log-uniform over [1e-6, c], uniform over
// [0, c], uniform over the Doppler core (x in [0, 8]), and the transition
// from core to wing (x in [0, 4] with y in [0.01, 10]).  Inputs are the
// network features; the target is log(K chi) - log(Kb) with K from the
// double-precision device line shape and chi from Eq.(10).
__global__ void k_mlp_samples(MlpSampleCfg c, uint64_t seed, int64_t n, float* __restrict__ X,
                              float* __restrict__ T, const DeviceTables* __restrict__ tabs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t b = (uint64_t)i * 8;
  const double nu0 = c.nu_lo + (c.nu_hi - c.nu_lo) * uniform01(seed, b + 0);
  const double Tk = c.T_lo + (c.T_hi - c.T_lo) * uniform01(seed, b + 1);
  const double aD = nu0 / kCLight * sqrt(2.0 * kLn2d * kBoltzmann * kNA * Tk / (c.molar_mass * 1e-3));
  double y = exp(log(c.y_lo) + (log(c.y_hi) - log(c.y_lo)) * uniform01(seed, b + 2));
  const double u = uniform01(seed, b + 3), v = uniform01(seed, b + 4);
  const double sq = sqrt(kLn2d);
  double ad;
  if (u < 0.3) ad = exp(log(1e-6) + (log(c.cutoff) - log(1e-6)) * v);
  else if (u < 0.55) ad = c.cutoff * v;
  else if (u < 0.8) ad = fmin(c.cutoff, 8.0 * aD / sq * v);
  else {
    // where the Doppler core meets the Lorentz wing: x < 4, 0.01 < y < 10
    ad = fmin(c.cutoff, 4.0 * aD / sq * v);
    y = exp(log(fmax(c.y_lo, 1e-2)) + (log(fmin(c.y_hi, 10.0)) - log(fmax(c.y_lo, 1e-2))) * uniform01(seed, b + 5));
  }
  const double x = sq * ad / aD;
  const double K = device_K<double>(x, y, tabs);
  const double chi = c.chi == MARFA_CHI_TONKOV ? tonkov<double>(ad) : 1.0;
  const double x2 = x * x, r = x2 + y * y, up = 1.0 + 1.7724538509055160 * y;
  const double kb = y * (1.0 + (3.0 * x2 - y * y) / (2.0 * r * r + 1.0)) / (1.7724538509055160 * (r + 0.5 * exp(-r))) +
                    exp(-x2) / (up * up);
  X[3 * i + 0] = (float)(asinh(x) * 0.125);
  X[3 * i + 1] = (float)(log10(y) * 0.5);
  X[3 * i + 2] = (float)(fmax(ad - 3.0, 0.0) / c.cutoff);
  T[i] = (float)(log(K * chi) - log(kb));
}

// ------------------------------------------------------------------
// host-side launchers
// ------------------------------------------------------------------
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n > 0) k_fill_u64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}
void launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s) {
  if (n > 0) k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}

void launch_prep(const LineIn& in, const double* layers, int nL, const Geometry& G, const PrepArgs& pa,
                 hipStream_t s) {
  int nblk = (int)((in.n + 255) / 256);
  launch_fill_u64(pa.smax, nL, 0ull, s);
  k_layer_const<<<(nL + 63) / 64, 64, 0, s>>>(layers, nL, in.molar_mass, pa.lc);
  if (nblk > 0) {
    dim3 grid(nblk, nL);
    k_prep_smax<<<dim3(nblk < 64 ? nblk : 64, nL), 256, 0, s>>>(in, pa.lc, pa.smax);
    k_prep_count<<<grid, 256, 0, s>>>(in, G, pa, nblk);
  }
  k_prep_scan<<<nL, 256, 0, s>>>(pa, nblk);
  if (nblk > 0) {
    dim3 grid(nblk, nL);
    if (pa.fp64) k_prep_scatter<double><<<grid, 256, 0, s>>>(in, G, pa, nblk);
    else k_prep_scatter<float><<<grid, 256, 0, s>>>(in, G, pa, nblk);
  }
  dim3 gb((unsigned)((in.n + 1 + 255) / 256), nL);
  k_prep_bucket<<<gb, 256, 0, s>>>(in.n, G, pa);
  k_layer_scale<<<(nL + 255) / 256, 256, 0, s>>>(layers, pa.smax, nL, pa.out_kind, pa.scale);
}

void launch_level_f32(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);
void launch_level_f32_count(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);
void launch_level_f32_surr(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);
void launch_level_f64(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);
void launch_level_f64_count(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);
void launch_level_f32_user(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);
void launch_level_f64_user(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);
void launch_level_f32_s4(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);
void launch_level_f64_s4(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s);

// Plans with the user line shape or chi run the kernels built with them (and
// every stencil); 4-point plans run kernels built for that stencil alone; the
// pair-counting kernels never evaluate a shape's value and hold every stencil.
// The learned shape serves 3- and 5-point plans only.
void launch_level(const Geometry& G, const LevelArgs& a, int grid, bool fp64, bool count, hipStream_t s) {
  const bool user = G.shape == MARFA_SHAPE_USER || G.chi == MARFA_CHI_USER;
  const bool four = G.ns == 4;
  if (fp64) {
    if (count) launch_level_f64_count(G, a, grid, s);
    else if (user) launch_level_f64_user(G, a, grid, s);
    else if (four) launch_level_f64_s4(G, a, grid, s);
    else launch_level_f64(G, a, grid, s);
  } else {
    if (count) launch_level_f32_count(G, a, grid, s);
    else if (a.surr) launch_level_f32_surr(G, a, grid, s);
    else if (user) launch_level_f32_user(G, a, grid, s);
    else if (four) launch_level_f32_s4(G, a, grid, s);
    else launch_level_f32(G, a, grid, s);
  }
}

void launch_rank(const LineIn& in, const double* layers, int nL, const double* span, int32_t* perm, hipStream_t s) {
  if (in.n <= 0) return;
  dim3 grid((unsigned)((in.n + 255) / 256), nL);
  k_rank<<<grid, 256, 0, s>>>(in, layers, span, perm);
}

template <typename R, int RHO>
static void launch_cascade_level(const Geometry& G, int l, dim3 grid, R* A, R* out, int64_t stride,
                                 const double* scale, hipStream_t s) {
  if (G.ns == 5) k_cascade<R, RHO, 5><<<grid, 256, 0, s>>>(G, l, A, out, stride, scale);
  else if (G.ns == 4) k_cascade<R, RHO, 4><<<grid, 256, 0, s>>>(G, l, A, out, stride, scale);
  else k_cascade<R, RHO, 3><<<grid, 256, 0, s>>>(G, l, A, out, stride, scale);
}

template <typename R>
static void launch_cascade_r(const Geometry& G, int nL, R* A, R* out, int64_t stride, const double* scale,
                             hipStream_t s) {
  for (int l = kLevels - 2; l >= 0; --l) {
    // the level tables have ratios 2 and 4 only (4 between levels 1 and 0 in the default table)
    const int64_t rho = G.r[l + 1] / G.r[l];
    const int64_t q_lo = G.lo[l] >= 0 ? G.lo[l] / rho : -((-G.lo[l] + rho - 1) / rho);
    const int64_t m_hi = G.lo[l] + G.n[l] - 1;
    const int64_t q_hi = m_hi >= 0 ? m_hi / rho : -((-m_hi + rho - 1) / rho);
    if constexpr (sizeof(R) == 4) {
      if (l == 0 && rho == 4 && G.lo[0] >= 0) {
        // groups of four aligned output nodes plus up to six single ones
        const dim3 g0((unsigned)((G.n[0] / 4 + 6 + 255) / 256), nL);
        if (G.ns == 5) k_cascade_out<5><<<g0, 256, 0, s>>>(G, A, out, stride, scale);
        else if (G.ns == 4) k_cascade_out<4><<<g0, 256, 0, s>>>(G, A, out, stride, scale);
        else k_cascade_out<3><<<g0, 256, 0, s>>>(G, A, out, stride, scale);
        continue;
      }
    }
    const dim3 grid((unsigned)((q_hi - q_lo + 1 + 255) / 256), nL);
    if (rho == 4) launch_cascade_level<R, 4>(G, l, grid, A, out, stride, scale, s);
    else launch_cascade_level<R, 2>(G, l, grid, A, out, stride, scale, s);
  }
}

void launch_cascade(const Geometry& G, int nL, void* A, void* out, int64_t stride, const double* scale, bool fp64,
                    hipStream_t s) {
  if (fp64) launch_cascade_r<double>(G, nL, (double*)A, (double*)out, stride, scale, s);
  else launch_cascade_r<float>(G, nL, (float*)A, (float*)out, stride, scale, s);
}

void launch_mlp_samples(const MlpSampleCfg& c, uint64_t seed, int64_t n, float* X, float* T,
                        const DeviceTables* tabs, hipStream_t s) {
  if (n <= 0) return;
  k_mlp_samples<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(c, seed, n, X, T, tabs);
}

void launch_voigt_eval(int64_t n, const double* x, const double* y, double* out, bool fp64,
                       const DeviceTables* tabs, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = (unsigned)((n + 255) / 256);
  if (fp64) k_voigt_eval<double><<<g, 256, 0, s>>>(n, x, y, out, tabs);
  else k_voigt_eval<float><<<g, 256, 0, s>>>(n, x, y, out, tabs);
}

}  // namespace marfa
