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
//   k_prep_smax       FP64 S(T) per (line, layer), max per layer
//   k_prep_count      per-block counts of kept lines by start level
//   k_prep_scan       exclusive offsets per (layer, start level)
//   k_prep_scatter    FP64 placement nu~0*2048 -> (int k0, frac) and the
//                     compacted per-layer line records, grouped by start level
//   k_layer_scale     output scale per layer (max S(T), number density)
//   k_level           persistent work queue over (layer, level, node tile):
//                     each lane owns one level node and sums the contributions
//                     of the lines in its windows (wave-uniform line loads)
//   k_cascade         3-point interpolation from level l+1 into level l;
//                     the level-0 pass applies the layer scale and writes out.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "marfa_internal.h"

namespace marfa {

// physical constants (CODATA 2018) and HITRAN reference temperature
constexpr double kC2 = 1.438776877;           // hc/k_B [cm K]
constexpr double kTref = 296.0;
constexpr double kBoltzmann = 1.380649e-23;   // [J/K]
constexpr double kNA = 6.02214076e23;         // [1/mol]
constexpr double kCLight = 299792458.0;       // [m/s]
constexpr double kAtmPa = 101325.0;
constexpr double kLn2d = 0.693147180559945309417;
constexpr double kInvPi = 0.318309886183790671538;
constexpr double kInvSqrtPi = 0.564189583547756286948;
constexpr double kH0 = 1.0 / 2048.0;

__constant__ double c_weid32[kWeidemanN32 + 1];
__constant__ double c_weid64[kWeidemanN64 + 1];
__constant__ double c_weidL[2];

template <typename R> struct RecOf;
template <> struct RecOf<float> { using T = LineRec32; };
template <> struct RecOf<double> { using T = LineRec64; };

// Wing series cut and the |z|^2 above which it replaces the rational core.
template <typename R> struct Prec;
template <> struct Prec<float> {
  static constexpr float kEps = 1e-8f;
  static constexpr float kZ2 = 36.0f;
  static constexpr int kTerms = 12;
};
template <> struct Prec<double> {
  static constexpr double kEps = 1e-17;
  static constexpr double kZ2 = 64.0;
  static constexpr int kTerms = 60;
};

// ------------------------------------------------------------------
// line shapes
// ------------------------------------------------------------------

// Re w(z) for |z| small, w the Faddeeva function, by Weideman's rational
// series in Z = (L+iz)/(L-iz):  w = 1/(sqrt(pi)(L-iz)) + 2/(L-iz)^2 sum_n a_n Z^(n-1).
// Evaluated in double precision in both paths (the real part is small next to
// |w| near the real axis, so single precision would lose it).
template <int N>
__device__ __forceinline__ double voigt_core(double x, double y, const double* a, double L) {
  double Ar = L + y, Ai = -x;
  double inv = 1.0 / (Ar * Ar + Ai * Ai);
  double iAr = Ar * inv, iAi = -Ai * inv;
  double Br = L - y, Bi = x;
  double Zr = Br * iAr - Bi * iAi, Zi = Br * iAi + Bi * iAr;
  double pr = a[N], pim = 0.0;
#pragma unroll
  for (int n = N - 1; n >= 1; --n) {
    double tr = fma(pr, Zr, fma(-pim, Zi, a[n]));
    pim = fma(pr, Zi, pim * Zr);
    pr = tr;
  }
  double i2r = iAr * iAr - iAi * iAi, i2i = 2.0 * iAr * iAi;
  return iAr * kInvSqrtPi + 2.0 * (pr * i2r - pim * i2i);
}

// Voigt far from the core (|z| large): f = Re[i/(pi (d + i g))] times the
// asymptotic series sum_k (2k-1)!! e^k U_2k(cos th), e = alpha_D^2/(2 ln2 |d+ig|^2),
// cos^2 th = d^2/(d^2+g^2), U the Chebyshev polynomials of the second kind
// (Re[i/u^(2k+1)] = g sin((2k+1)th)/(|u|^(2k+2) sin th)).  k = 1 is the
// 1 + 3/(2x^2) correction of Appendix C.  Returns f and the number of extra terms.
template <typename R>
__device__ __forceinline__ R voigt_wing(R dd, R gam, R gam2, R ae, int& terms) {
  R Q = R(1) / (dd + gam2);
  R e = ae * Q;
  R acc = R(1);
  if (e * R(3) >= Prec<R>::kEps) {
    R s = dd * Q;
    R t = R(4) * s - R(2);
    R ck = R(1), Um = R(-1), U = R(1);
    for (int k = 1; k <= Prec<R>::kTerms; ++k) {
      ck *= R(2 * k - 1) * e;
      R Un = t * U - Um;
      Um = U;
      U = Un;
      acc += ck * U;
      ++terms;
      if (ck * R(2 * k + 1) < Prec<R>::kEps) break;
    }
  }
  return gam * Q * R(kInvPi) * acc;
}

template <typename R>
__device__ __forceinline__ R tonkov(R a) {
  // Eq.(10): 1.084 e^{-0.027|d|} on [3,150], 0.208 e^{-0.016|d|} on (150,300],
  // 0.025 e^{-0.009|d|} above 300, 1 otherwise
  if (a < R(3)) return R(1);
  if (a <= R(150)) return R(1.084) * exp(R(-0.027) * a);
  if (a <= R(300)) return R(0.208) * exp(R(-0.016) * a);
  return R(0.025) * exp(R(-0.009) * a);
}

struct Counts {
  uint32_t core, wing, terms;
};

// g(d) = S' F(d) chi(|d|) [|d| <= c], d in fine units
template <typename R, bool COUNT>
__device__ __forceinline__ R line_value(R d, const typename RecOf<R>::T& L, const Geometry& G, R cfine,
                                        Counts& cnt) {
  R ad = fabs(d);
  if (ad > cfine) return R(0);
  R dcm = d * R(kH0);
  R dd = dcm * dcm;
  R f;
  if (G.shape == MARFA_SHAPE_LORENTZ) {
    f = R(L.gam) * R(kInvPi) / (dd + R(L.gam2));
  } else if (G.shape == MARFA_SHAPE_DOPPLER) {
    R x = R(L.xs) * dcm;
    f = R(L.xs) * R(kInvSqrtPi) * exp(-x * x);
  } else {
    R x = R(L.xs) * dcm;
    R y = R(L.xs) * R(L.gam);
    R z2 = x * x + y * y;
    if (L.xs == 0 || z2 >= Prec<R>::kZ2) {
      int terms = 0;
      f = voigt_wing<R>(dd, R(L.gam), R(L.gam2), R(L.ae), terms);
      if (COUNT) { cnt.wing++; cnt.terms += terms; }
    } else {
      double K;
      if (sizeof(R) == 4)
        K = voigt_core<kWeidemanN32>(fabs((double)x), (double)y, c_weid32, c_weidL[0]);
      else
        K = voigt_core<kWeidemanN64>(fabs((double)x), (double)y, c_weid64, c_weidL[1]);
      f = R((double)L.xs * kInvSqrtPi * K);
      if (COUNT) cnt.core++;
    }
  }
  R chi = (G.chi == MARFA_CHI_TONKOV) ? tonkov<R>(ad * R(kH0)) : R(1);
  return R(L.Sp) * f * chi;
}

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
__device__ __forceinline__ LineState line_state(const LineIn& in, int64_t j, const double* lay) {
  double p = lay[0], T = lay[1], ps = lay[2], q = lay[3];
  double nu = in.nu0[j];
  double qr = q > 0.0 ? q : kTref / T;
  double boltz = exp(-kC2 * (double)in.El[j] * (1.0 / T - 1.0 / kTref));
  double stim = nu > 0.0 ? expm1(-kC2 * nu / T) / expm1(-kC2 * nu / kTref) : kTref / T;
  LineState s;
  s.S = (double)in.S296[j] * qr * boltz * stim;
  s.gL = pow(kTref / T, (double)in.nair[j]) * ((double)in.gair[j] * (p - ps) + (double)in.gself[j] * ps);
  s.aD = nu / kCLight * sqrt(2.0 * kLn2d * kBoltzmann * kNA * T / (in.molar_mass * 1e-3));
  s.nut = nu + (double)in.dair[j] * p;
  return s;
}

__global__ void k_prep_smax(LineIn in, const double* __restrict__ layers, unsigned long long* smax) {
  __shared__ double red[256];
  int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int L = blockIdx.y;
  double S = 0.0;
  if (j < in.n) S = line_state(in, j, layers + 4 * L).S;
  red[threadIdx.x] = S;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0.0) atomicMax(&smax[L], (unsigned long long)__double_as_longlong(red[0]));
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

__device__ __forceinline__ int line_key(const LineIn& in, int64_t j, const double* lay, double smax,
                                        double prune, double R, const Geometry& G, LineState& st) {
  st = line_state(in, j, lay);
  bool keep = prune <= 0.0 || st.S >= prune * smax;
  if (!keep) return kGroups;  // dropped
  return start_level(fmax(st.gL, st.aD), R, G);
}

__global__ void k_prep_count(LineIn in, const double* __restrict__ layers, const unsigned long long* smax,
                             double prune, double R, Geometry G, int32_t* bcount, int nblk) {
  __shared__ int cnt[kGroups + 1];
  if (threadIdx.x <= kGroups) cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int L = blockIdx.y;
  if (j < in.n) {
    LineState st;
    int key = line_key(in, j, layers + 4 * L, __longlong_as_double((long long)smax[L]), prune, R, G, st);
    atomicAdd(&cnt[key], 1);
  }
  __syncthreads();
  if (threadIdx.x <= kGroups)
    bcount[((int64_t)L * nblk + blockIdx.x) * (kGroups + 1) + threadIdx.x] = cnt[threadIdx.x];
}

// exclusive offsets per (layer, group) over blocks, in place; group totals and starts
__global__ void k_prep_scan(int32_t* bcount, int nblk, int32_t* gcount, int32_t* gstart) {
  __shared__ int part[256];
  __shared__ int tot[kGroups + 1];
  int L = blockIdx.x;
  int t = threadIdx.x;
  int chunk = (nblk + 255) / 256;
  int b0 = t * chunk, b1 = min(nblk, b0 + chunk);
  for (int g = 0; g <= kGroups; ++g) {
    int s = 0;
    for (int b = b0; b < b1; ++b) s += bcount[((int64_t)L * nblk + b) * (kGroups + 1) + g];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan
    for (int o = 1; o < 256; o <<= 1) {
      int v = (t >= o) ? part[t - o] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int run = part[t] - s;
    for (int b = b0; b < b1; ++b) {
      int64_t k = ((int64_t)L * nblk + b) * (kGroups + 1) + g;
      int v = bcount[k];
      bcount[k] = run;
      run += v;
    }
    if (t == 255) tot[g] = part[255];
    __syncthreads();
  }
  if (t == 0) {
    int run = 0;
    for (int g = 0; g <= kGroups; ++g) {
      gcount[L * (kGroups + 1) + g] = tot[g];
      gstart[L * (kGroups + 1) + g] = run;
      run += tot[g];
    }
  }
}

template <typename R>
__global__ void k_prep_scatter(LineIn in, const double* __restrict__ layers, const unsigned long long* smax,
                               double prune, double R_, Geometry G, const int32_t* bcount, int nblk,
                               const int32_t* gstart, typename RecOf<R>::T* rec, double* cnu) {
  __shared__ int wcnt[4][kGroups + 1];
  int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int L = blockIdx.y;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double sm = __longlong_as_double((long long)smax[L]);
  int key = kGroups + 1;  // out of range: not a line
  LineState st{0, 0, 0, 0};
  if (j < in.n) key = line_key(in, j, layers + 4 * L, sm, prune, R_, G, st);
  unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int rank = 0;
  for (int g = 0; g <= kGroups; ++g) {
    unsigned long long m = __ballot(key == g);
    if (key == g) rank = __popcll(m & lt);
    if (lane == 0) wcnt[wv][g] = __popcll(m);
  }
  __syncthreads();
  if (key >= kGroups) return;
  int off = rank;
  for (int w = 0; w < wv; ++w) off += wcnt[w][key];
  int64_t dest = (int64_t)gstart[L * (kGroups + 1) + key] +
                 bcount[((int64_t)L * nblk + blockIdx.x) * (kGroups + 1) + key] + off;
  int64_t base = (int64_t)L * in.n;
  // FP64 placement of the shifted centre on the finest lattice
  double t = st.nut * 2048.0;
  double k0 = floor(t);
  typename RecOf<R>::T r;
  R fr = R(t - k0);
  if (fr >= R(1)) { k0 += 1.0; fr = R(0); }
  r.k0 = (int32_t)k0;
  r.frac = fr;
  r.Sp = sm > 0.0 ? R(st.S / sm) : R(0);
  r.gam = R(st.gL);
  r.gam2 = R(st.gL * st.gL);
  r.ae = R(st.aD * st.aD / (2.0 * kLn2d));
  r.xs = st.aD > 0.0 ? R(sqrt(kLn2d) / st.aD) : R(0);
  r.aD = R(st.aD);
  rec[base + dest] = r;
  cnu[base + dest] = in.nu0[j];
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
// level accumulation
// ------------------------------------------------------------------
__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ __forceinline__ int64_t lower_bound(const double* a, int64_t n, double v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t upper_bound(const double* a, int64_t n, double v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}


template <typename R, bool COUNT>
__global__ void __launch_bounds__(256) k_level(Geometry G, LevelArgs a) {
  using Rec = typename RecOf<R>::T;
  __shared__ int64_t s_item;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t total = a.n_tiles * a.n_layers;
  const R cfine = R(G.c_fine);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t item = s_item;
    if (item >= total) break;
    const Tile tile = a.tiles[item / a.n_layers];
    const int layer = (int)(item % a.n_layers);
    const int l = tile.level;
    const int64_t rl = G.r[l];
    const Rec* rec = reinterpret_cast<const Rec*>(a.rec) + (int64_t)layer * a.n_lines;
    const double* cnu = a.cnu + (int64_t)layer * a.n_lines;
    const double sh_lo = a.shift[2 * layer], sh_hi = a.shift[2 * layer + 1];
    const int nsub = (tile.count + kWave - 1) / kWave;
    for (int sub = wv; sub < nsub; sub += 4) {
      const int64_t rel0 = tile.first + (int64_t)sub * kWave;
      const int64_t m = G.lo[l] + rel0 + lane;
      const bool active = (rel0 + lane < G.n[l]) && (sub * kWave + lane < tile.count);
      const int64_t X = m * rl;
      const int64_t Xf = (G.lo[l] + rel0) * rl;
      const int64_t Xl = Xf + (int64_t)(kWave - 1) * rl;
      // stencil on level l+1
      int ns = 0;
      int64_t Xs[3] = {0, 0, 0};
      R ws[3] = {0, 0, 0};
      if (l < kLevels - 1) {
        int64_t rho = G.r[l + 1] / rl;
        int64_t q = floor_div(m, rho);
        int64_t rem = m - q * rho;
        int64_t r1 = G.r[l + 1];
        if (rem == 0) {
          ns = 1; Xs[0] = q * r1; ws[0] = R(1);
        } else {
          double f = (double)rem / (double)rho, t;
          int64_t kc;
          if (f <= 0.5) { kc = q; t = f; } else { kc = q + 1; t = f - 1.0; }
          ns = 3;
          Xs[0] = (kc - 1) * r1; ws[0] = R(0.5 * t * (t - 1.0));
          Xs[1] = kc * r1;       ws[1] = R(1.0 - t * t);
          Xs[2] = (kc + 1) * r1; ws[2] = R(0.5 * t * (t + 1.0));
        }
      }
      R acc = R(0);
      Counts cnt{0, 0, 0};
      uint32_t n_used = 0, n_band = 0;
      for (int s = 0; s < kGroups; ++s) {
        const int64_t gc = a.gcount[layer * (kGroups + 1) + s];
        if (gc == 0) continue;
        const int64_t gs = a.gstart[layer * (kGroups + 1) + s];
        const IntervalSet& iv = a.ivs[l * kGroups + s];
        if (iv.n_iv == 0) continue;
        const R b_in = (l > 0) ? R(G.b[l - 1]) : R(0);
        const R b_out = (l < kLevels - 1) ? R(G.b[l]) : R(0);
        const R Bl = (l < kLevels - 1) ? R(G.B[l]) : R(0);
        for (int k = 0; k < iv.n_iv; ++k) {
          const double ia = iv.a[k], ib = iv.b[k];
          const R ra = R(ia), rb = R(ib);
          const int nside = (ia == 0.0) ? 1 : 2;
          for (int side = 0; side < nside; ++side) {
            double plo, phi;
            int sgn;
            if (nside == 1) { plo = (double)Xf - ib; phi = (double)Xl + ib; sgn = 0; }
            else if (side == 0) { plo = (double)Xf - ib; phi = (double)Xl - ia; sgn = 1; }
            else { plo = (double)Xf + ia; phi = (double)Xl + ib; sgn = -1; }
            const double vlo = plo * kH0 - sh_hi - 1e-7, vhi = phi * kH0 - sh_lo + 1e-7;
            const int64_t j0 = lower_bound(cnu + gs, gc, vlo);
            const int64_t j1 = upper_bound(cnu + gs, gc, vhi);
            for (int64_t j = gs + j0; j < gs + j1; ++j) {
              const Rec L = rec[j];
              const R d = R((int32_t)(X - L.k0)) - R(L.frac);
              const R ad = fabs(d);
              bool use = active && ad >= ra && ad <= rb && (sgn == 0 || (sgn > 0 ? d > R(0) : d < R(0)));
              if (!use) continue;
              bool in_reg = (l >= s) && ad <= cfine && (l == s || ad >= b_in) &&
                            (l == kLevels - 1 || ad < b_out);
              bool in_band = false;
              for (int qi = 0; qi < iv.n_q; ++qi) in_band |= fabs(ad - R(iv.q[qi])) <= Bl;
              if (!(in_reg || in_band)) continue;
              // T_l(d): zero inside the hole of a wing level
              R v = (l > s && ad < b_in) ? R(0) : line_value<R, COUNT>(d, L, G, cfine, cnt);
              if (in_band) {
                for (int i = 0; i < ns; ++i) {
                  const R di = R((int32_t)(Xs[i] - L.k0)) - R(L.frac);
                  const R adi = fabs(di);
                  if (!(l + 1 > s && adi < b_out)) v -= ws[i] * line_value<R, COUNT>(di, L, G, cfine, cnt);
                }
              }
              acc += v;
              if (COUNT) { n_used++; n_band += in_band ? 1u : 0u; }
            }
          }
        }
      }
      if (COUNT) {
        // wave reductions, one atomic per counter per sub-tile
        unsigned long long v[5] = {n_used, n_band, cnt.core, cnt.wing, cnt.terms};
        for (int i = 0; i < 5; ++i) {
          unsigned long long x = v[i];
          for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
          v[i] = x;
        }
        if (lane == 0) {
          atomicAdd(&a.stats[l], v[0]);
          atomicAdd(&a.stats[11], v[1]);
          atomicAdd(&a.stats[12], v[2]);
          atomicAdd(&a.stats[13], v[3]);
          atomicAdd(&a.stats[14], v[4]);
        }
      } else if (active) {
        const int64_t rel = m - G.lo[l];
        if (l == 0)
          reinterpret_cast<R*>(a.out)[(int64_t)layer * a.stride + rel] = acc;
        else
          reinterpret_cast<R*>(a.A)[(int64_t)layer * G.a_total + G.aoff[l] + rel] = acc;
      }
    }
  }
}

// ------------------------------------------------------------------
// cascade: A_l += P(A_(l+1)); level 0 also scales into the output
// ------------------------------------------------------------------
template <typename R>
__global__ void k_cascade(Geometry G, int l, R* A, R* out, int64_t stride, const double* scale) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int layer = blockIdx.y;
  if (i >= G.n[l]) return;
  int64_t m = G.lo[l] + i;
  int64_t rho = G.r[l + 1] / G.r[l];
  int64_t q = floor_div(m, rho);
  int64_t rem = m - q * rho;
  const R* Ac = A + (int64_t)layer * G.a_total + G.aoff[l + 1] - G.lo[l + 1];
  R v;
  if (rem == 0) {
    v = Ac[q];
  } else {
    double f = (double)rem / (double)rho, t;
    int64_t kc;
    if (f <= 0.5) { kc = q; t = f; } else { kc = q + 1; t = f - 1.0; }
    v = R(0.5 * t * (t - 1.0)) * Ac[kc - 1] + R(1.0 - t * t) * Ac[kc] + R(0.5 * t * (t + 1.0)) * Ac[kc + 1];
  }
  if (l > 0) {
    A[(int64_t)layer * G.a_total + G.aoff[l] + i] += v;
  } else {
    R* o = out + (int64_t)layer * stride + i;
    *o = R(scale[layer]) * (*o + v);
  }
}

// device Voigt for tests: K(x, y) through the hot-path shape code
template <typename R>
__global__ void k_voigt_eval(int64_t n, const double* x, const double* y, double* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  typename RecOf<R>::T L{};
  // alpha_D = sqrt(ln 2): x = d, y = gamma_L, F = K / sqrt(pi)
  L.k0 = 0; L.frac = 0; L.Sp = R(1);
  L.gam = R(y[i]); L.gam2 = R(y[i]) * R(y[i]);
  L.ae = R(0.5); L.xs = R(1); L.aD = R(sqrt(kLn2d));
  Geometry G{};
  G.shape = MARFA_SHAPE_VOIGT;
  G.chi = MARFA_CHI_NONE;
  Counts c{0, 0, 0};
  R d = R(x[i]) * R(2048);  // fine units
  R f = line_value<R, false>(d, L, G, R(INFINITY), c);
  out[i] = (double)f * 1.772453850905516;
}

// ------------------------------------------------------------------
// host-side launchers
// ------------------------------------------------------------------
hipError_t upload_weideman(const double* a32, const double* a64, const double* L2) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_weid32), a32, sizeof(double) * (kWeidemanN32 + 1));
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_weid64), a64, sizeof(double) * (kWeidemanN64 + 1));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_weidL), L2, sizeof(double) * 2);
}

void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n > 0) k_fill_u64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}
void launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s) {
  if (n > 0) k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}

void launch_prep(const LineIn& in, const double* layers, int nL, unsigned long long* smax, double prune, double R,
                 const Geometry& G, int32_t* bcount, int32_t* gcount, int32_t* gstart, void* rec, double* cnu,
                 double* scale, int out_kind, bool fp64, hipStream_t s) {
  int nblk = (int)((in.n + 255) / 256);
  launch_fill_u64(smax, nL, 0ull, s);
  if (nblk > 0) {
    dim3 grid(nblk, nL);
    k_prep_smax<<<grid, 256, 0, s>>>(in, layers, smax);
    k_prep_count<<<grid, 256, 0, s>>>(in, layers, smax, prune, R, G, bcount, nblk);
  }
  k_prep_scan<<<nL, 256, 0, s>>>(bcount, nblk, gcount, gstart);
  if (nblk > 0) {
    dim3 grid(nblk, nL);
    if (fp64)
      k_prep_scatter<double><<<grid, 256, 0, s>>>(in, layers, smax, prune, R, G, bcount, nblk, gstart,
                                                   (LineRec64*)rec, cnu);
    else
      k_prep_scatter<float><<<grid, 256, 0, s>>>(in, layers, smax, prune, R, G, bcount, nblk, gstart,
                                                  (LineRec32*)rec, cnu);
  }
  k_layer_scale<<<(nL + 255) / 256, 256, 0, s>>>(layers, smax, nL, out_kind, scale);
}

void launch_level(const Geometry& G, const LevelArgs& a, int grid, bool fp64, bool count, hipStream_t s) {
  if (fp64) {
    if (count) k_level<double, true><<<grid, 256, 0, s>>>(G, a);
    else k_level<double, false><<<grid, 256, 0, s>>>(G, a);
  } else {
    if (count) k_level<float, true><<<grid, 256, 0, s>>>(G, a);
    else k_level<float, false><<<grid, 256, 0, s>>>(G, a);
  }
}

void launch_cascade(const Geometry& G, int nL, void* A, void* out, int64_t stride, const double* scale, bool fp64,
                    hipStream_t s) {
  for (int l = kLevels - 2; l >= 0; --l) {
    dim3 grid((unsigned)((G.n[l] + 255) / 256), nL);
    if (fp64)
      k_cascade<double><<<grid, 256, 0, s>>>(G, l, (double*)A, (double*)out, stride, scale);
    else
      k_cascade<float><<<grid, 256, 0, s>>>(G, l, (float*)A, (float*)out, stride, scale);
  }
}

void launch_voigt_eval(int64_t n, const double* x, const double* y, double* out, bool fp64, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = (unsigned)((n + 255) / 256);
  if (fp64) k_voigt_eval<double><<<g, 256, 0, s>>>(n, x, y, out);
  else k_voigt_eval<float><<<g, 256, 0, s>>>(n, x, y, out);
}

}  // namespace marfa
