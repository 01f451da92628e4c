// marfa_level.h -- the level-accumulation kernel of the eleven-grid library
// (Section 2.4): a persistent work queue over (layer, level, node tile) whose
// region pass gathers the lines of each node's windows and whose residual-band
// pass corrects the jumps of the coarser level's line parts.  Each
// instantiation is compiled in a translation unit of its own
// (marfa_level_*.hip) so that they build in parallel.
#pragma once
#include "marfa_device.h"

namespace marfa {

// ------------------------------------------------------------------
// level accumulation
// ------------------------------------------------------------------

// T_l(d) of a line with start level s: zero in the hole of a wing level
template <typename R, bool COUNT>
__device__ __forceinline__ R T_level(R d, int l, int s, const typename RecOf<R>::T& L, R Sp, const Geometry& G,
                                     R cfine, R b_prev, Counts& cnt) {
  if (l > s && fabs(d) < b_prev) return R(0);
  return line_value<R, COUNT>(d, L, Sp, G, cfine, cnt);
}

template <typename R> __device__ __forceinline__ R fast_rcp(R x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double fast_rcp<double>(double x) { return 1.0 / x; }
template <typename R> __device__ __forceinline__ R fast_exp2(R x);
template <> __device__ __forceinline__ float fast_exp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <> __device__ __forceinline__ double fast_exp2<double>(double x) { return exp2(x); }

// Wing series of the fast path.  Term k (coefficient (2k-1)!! e^k) is kept
// while some live lane has (2k+1)!! e^k >= eps, i.e. e >= thr(k) with
// thr(k) = (eps / (2k+1)!!)^(1/k), computed at compile time (Newton's method
// for the k-th root).  The core takes |z| < 6 (FP32) / 8 (FP64); at |z| = 6
// the FP32 series needs 6 terms for 1e-6 (a cut well under the 3e-5 the
// single-precision path is held to, and common to every pass, so it cancels
// between a coarse sum and the band correction that removes it).
constexpr double ct_pow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}
constexpr double ct_root(double a, int k) {
  double r = 1.0;
  for (int i = 0; i < 400; ++i) r -= (ct_pow(r, k) - a) / (k * ct_pow(r, k - 1));
  return r;
}
constexpr double ct_series_thr(double eps, int k) {
  double df = 1.0;
  for (int i = 1; i <= k; ++i) df *= 2.0 * i + 1.0;
  return ct_root(eps / df, k);
}
template <typename R> struct Series;
template <> struct Series<float> {
  static constexpr int kMax = 10;
  static constexpr float thr[kMax + 1] = {
      0.f, (float)ct_series_thr(1e-6, 1), (float)ct_series_thr(1e-6, 2), (float)ct_series_thr(1e-6, 3),
      (float)ct_series_thr(1e-6, 4), (float)ct_series_thr(1e-6, 5), (float)ct_series_thr(1e-6, 6),
      (float)ct_series_thr(1e-6, 7), (float)ct_series_thr(1e-6, 8), (float)ct_series_thr(1e-6, 9),
      (float)ct_series_thr(1e-6, 10)};
};
static_assert(Series<float>::thr[2] > 2.5e-4f && Series<float>::thr[2] < 2.6e-4f, "sqrt(1e-6 / 15)");
template <> struct Series<double> { static constexpr int kMax = 60; };

// chi of Eq.(10) without branches: exp2(c0 + c1 |d|) with the piece chosen by
// selects; the user chi through its compiled-in function
template <typename R>
__device__ __forceinline__ R chi_any(R ad_fine, const Geometry& G) {
  if (MARFA_USER_PLUGINS && G.chi == MARFA_CHI_USER) return MarfaUserChi::chi<R>(ad_fine * R(kH0));
  if (G.chi != MARFA_CHI_TONKOV) return R(1);
  const R a = ad_fine * R(kH0);
  R c0 = R(0), c1 = R(0);
  c0 = a >= R(3) ? R(G.chi_c0[0]) : c0;
  c1 = a >= R(3) ? R(G.chi_c1[0]) : c1;
  c0 = a > R(150) ? R(G.chi_c0[1]) : c0;
  c1 = a > R(150) ? R(G.chi_c1[1]) : c1;
  c0 = a > R(300) ? R(G.chi_c0[2]) : c0;
  c1 = a > R(300) ? R(G.chi_c1[2]) : c1;
  return fast_exp2<R>(c0 + c1 * a);
}

// S' F(d) of the core (|z| < 6): the single-precision Taylor-table core
// inline; the double-precision Weideman core kept out of line (its path is
// not timed and stays small)
__device__ __attribute__((noinline)) double core_value64(double dcm, double xs, double gam, double amp,
                                                         const double* __restrict__ wd) {
  return amp * voigt_core<kWeidemanN64>(fabs(xs * dcm), xs * gam, wd, wd[kWeidemanN64 + 1]);
}
// amp = S' sqrt(ln 2) / (sqrt(pi) alpha_D) from the record
template <typename R>
__device__ __forceinline__ R core_value(R dcm, R xs, R gam, R amp, const Geometry& G) {
  if constexpr (sizeof(R) == 4)
    return amp * voigt_core32(fabsf(xs * dcm), xs * gam, G.ktab);
  else
    return core_value64(dcm, xs, gam, amp, G.weid);
}

// S' F(d) (without chi and the cut-off) for the Voigt shape (Lorentz: ae = 0)
// outside the core: the asymptotic wing series, each lane stopping at its own
// term count (so a pair's value does not depend on the pairs that share its
// wavefront).  `live` marks lanes whose value is used.  The wing is A Q sum with A = S' gamma_L / pi and
// Q = 1/(d^2 + gamma_L^2).  `core` returns whether the pair is live and in the
// core (|z| < sqrt(kZ2)), where the returned value is not the line shape.
template <typename R, bool COUNT>
__device__ __forceinline__ R shape_wing(R dcm, const typename RecOf<R>::T& L, bool live, Counts& cnt, bool& core_out) {
  const R g2 = gam2_of(L);
  const R den = fma(dcm, dcm, g2);
  const R Q = fast_rcp<R>(den);
  const R e = R(L.ae) * Q;
  const bool core = e > R(0.5 / Prec<R>::kZ2);     // |z|^2 = 1/(2e) < kZ2
  // U_2 = 4 d^2 Q - 1 = 3 - 4 gamma^2 Q
  R U = fma(R(-4) * g2, Q, R(3));
  R sum = fma(e, U, R(1));
  const bool wing = live && !core;
  // term k, with coefficient c_k = (2k-1)!! e^k, is kept while some live
  // wing lane has (2k+1)!! e^k >= eps: e >= thr(k) (FP32), or from the
  // running coefficient (2k+1)(2k-1) c_(k-1) e >= eps (FP64)
  const R eps = Prec<R>::kEps;
  auto more = [&](int k, R ck_prev) -> bool {
    if constexpr (sizeof(R) == 4) return e >= Series<float>::thr[k];
    else return R((2 * k + 1) * (2 * k - 1)) * ck_prev * e >= eps;
  };
  if (wing && more(2, e)) {
    const R t = U - R(1);
    R Um = R(1), ck = e;
#pragma unroll
    for (int k = 2; k < Series<R>::kMax; ++k) {
      ck *= R(2 * k - 1) * e;
      const R Un = t * U - Um;
      Um = U;
      U = Un;
      sum += ck * U;
      if (COUNT) cnt.terms++;
      if (k + 1 >= Series<R>::kMax || !more(k + 1, ck)) break;
    }
  }
  core_out = live && core;
  if (COUNT && live) { if (core) cnt.core++; else cnt.wing++; }
  return R(L.A) * Q * sum;
}

// S' F(d) (without chi and the cut-off) for the Voigt shape: the wing series,
// and the core for lanes with |z| < sqrt(kZ2).  The core needs S' itself (sp[j]).
template <typename R, bool COUNT>
__device__ __forceinline__ R shape_fast(R d, const typename RecOf<R>::T& L, const R* __restrict__ sp, int32_t j,
                                        const Geometry& G, bool live, Counts& cnt) {
  const R dcm = d * R(kH0);
  bool core;
  R f = shape_wing<R, COUNT>(dcm, L, live, cnt, core);
  if (core) f = core_value<R>(dcm, L.xs, L.gam, R(L.amp), G);
  return f;
}

// Wave-local queue of core pairs (single-precision plain kernel): the pairs of
// one line step whose |z| is below the core radius are packed densely over
// the wavefront's lanes, evaluated 64 at a time, and handed back to the lanes
// they came from, which add them in their usual order (the sums are the same
// bits as with the core evaluated in place).
constexpr int kCoreQueue = 256;   // 64 lanes x up to 4 nodes per lane
struct CoreQueue {
  float* x;        // [kCoreQueue] |x| of the queued pair, then its value
  uint8_t* src;    // [kCoreQueue] lane that queued the pair
  float* y;        // [64] y of each lane's line
  float* amp;      // [64] the core scale of each lane's line
};

// For the K node slots of a lane (pairs d[k] with the lane's line L): replace
// f[k] by the core value wherever core[k].
template <int K>
__device__ __forceinline__ void core_batch(const CoreQueue& q, const LineRec32& L, const float* d, const bool* core,
                                           float* f, const Geometry& G) {
  const int lane = threadIdx.x & 63;
  q.y[lane] = L.xs * L.gam;
  q.amp[lane] = L.amp;
  int pos[K];
  int n = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(core[k]);
    pos[k] = n + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (core[k]) {
      q.x[pos[k]] = fabsf(L.xs * (d[k] * float(kH0)));
      q.src[pos[k]] = (uint8_t)lane;
    }
    n += __builtin_popcountll(m);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int r = 0; r < n; r += 64) {
    const int i = r + lane;
    if (i < n) {
      const int s = q.src[i];
      const float Kv = voigt_core32(q.x[i], q.y[s], G.ktab);
      q.x[i] = q.amp[s] * Kv;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (core[k]) f[k] = q.x[pos[k]];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// g(d) = S' F(d) chi(|d|) [|d| <= c] for any shape
template <typename R, bool COUNT>
__device__ __forceinline__ R g_any(R d, const typename RecOf<R>::T& L, const R* __restrict__ sp, int32_t j,
                                   const Geometry& G, R cfine, bool live, Counts& cnt) {
  if (generic_shape(G)) return live ? line_value<R, COUNT>(d, L, sp[j], G, cfine, cnt) : R(0);
  const R ad = fabs(d);
  const R v = shape_fast<R, COUNT>(d, L, sp, j, G, live && ad <= cfine, cnt) * chi_any<R>(ad, G);
  return ad <= cfine ? v : R(0);
}

// S' F(d) chi(|d|) through the learned line shape, for one (line, node) pair
// per lane; wave-collective (all 64 lanes call it together).  Pairs outside
// the trained domain that are live use the plain shape.  With A = S'
// gamma_L / pi and y = xs gamma_L: S' F chi = A sqrt(pi) xs^2 / y Kb e^t.
template <bool COUNT>
__device__ float g_surr(float d, const LineRec32& L, const float* __restrict__ sp, int32_t j, const Geometry& G,
                        const LevelArgs& a, bool live, Counts& cnt) {
  const float dcm = d * float(kH0);
  const float x = L.xs * dcm;
  const float y = L.xs * L.gam;
  const bool dom = y >= kMlpYMin && y <= kMlpYMax && fabsf(x) <= a.mlp_xmax;
  float f1, f2, f3;
  mlp_features(x, dom ? y : 1.0f, fabsf(dcm), a.mlp_inv_c, f1, f2, f3);
  const float t = mlp_forward_wave<true>(a.mlp, f1, f2, f3);
  float v = L.A * 1.7724538509055160f * L.xs * L.xs * __builtin_amdgcn_rcpf(dom ? y : 1.0f) * mlp_base(x, y) *
            __expf(t);
  v = dom ? v : 0.0f;
  if (__builtin_amdgcn_ballot_w64(live && !dom)) {
    const float pv = shape_fast<float, COUNT>(d, L, sp, j, G, live && !dom, cnt) * chi_any<float>(fabsf(d), G);
    v = dom ? v : pv;
  }
  return v;
}

// Wave-local queue of learned-shape pairs: every lane pushes the pairs it
// needs in one session, the network then runs on 64 queued pairs at a time,
// and each lane reads its values back by slot in its own order.  Per entry:
// |x|, y and |d| in cm; the batch overwrites |x| with Kb(x, y) e^t / y, and
// the lane scales it by its line's S' sqrt(pi) xs^2 (= A sqrt(pi) xs^2 with
// A = S' gamma_L / pi).  A session pushes at most kSurrSlots pairs per lane
// (with the 3-point stencil, the only one the learned shape runs with: four
// nodes of the region pass, five stencil values or two candidate centres of
// three nodes each in the band pass), so the queue never overflows.  Six
// slots keep the four queues at 18 KB, so three workgroups share a CU.
constexpr int kSurrSlots = 6;
constexpr int kSurrQueue = 64 * kSurrSlots;   // entries per wavefront: three arrays of this many floats

// Push `want` pairs of the calling lanes; returns the slot of each, `n` the
// wave's running count (uniform).
__device__ __forceinline__ int surr_push(float* q, bool want, int& n, float x, float y, float ad) {
  const uint64_t m = __builtin_amdgcn_ballot_w64(want);
  const int pos = n + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  if (want) {
    q[pos] = fabsf(x);
    q[kSurrQueue + pos] = y;
    q[2 * kSurrQueue + pos] = ad;
  }
  n += __builtin_popcountll(m);
  return pos;
}

// Evaluate the n queued pairs (n uniform): Kb(x, y) e^t / y into the |x| slot.
__device__ __forceinline__ void surr_batch(float* q, int n, const LevelArgs& a) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int lane = threadIdx.x & 63;
  for (int r = 0; r < n; r += 64) {
    const int i = r + lane;
    const bool ok = i < n;
    const float x = ok ? q[i] : 1.0f;
    const float y = ok ? q[kSurrQueue + i] : 1.0f;
    const float ad = ok ? q[2 * kSurrQueue + i] : 0.0f;
    float f1, f2, f3;
    mlp_features(x, y, ad, a.mlp_inv_c, f1, f2, f3);
    // a partial last batch runs only the 16-sample groups that hold entries
    const int ns = n - r >= 64 ? 4 : (n - r + 15) >> 4;
    const float t = mlp_forward_wave<true>(a.mlp, f1, f2, f3, ns);
    if (ok) q[i] = __builtin_amdgcn_rcpf(y) * mlp_base(x, y) * __expf(t);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// the learned shape's inputs of one pair: whether it lies in the trained domain
__device__ __forceinline__ bool surr_domain(float d, const LineRec32& L, const LevelArgs& a, float& x, float& y) {
  x = L.xs * (d * float(kH0));
  y = L.xs * L.gam;
  return y >= kMlpYMin && y <= kMlpYMax && fabsf(x) <= a.mlp_xmax;
}

// g(d) with the cut-off for the band pass, chi given for the jump's
// neighbourhood (mode 0: 1, 1: one piece exp2(c0 + c1 |d|), 2: any piece)
template <typename R, bool COUNT, bool SURR>
__device__ __forceinline__ R g_band(R d, const typename RecOf<R>::T& L, const R* __restrict__ sp, int32_t j,
                                    const Geometry& G, R cfine, bool live, Counts& cnt, const LevelArgs& a,
                                    int chi_mode, R c0, R c1) {
  if (SURR || generic_shape(G)) return g_eval<R, COUNT, SURR>(d, L, sp, j, G, cfine, live, cnt, a);
  const R ad = fabs(d);
  const R f = shape_fast<R, COUNT>(d, L, sp, j, G, live && ad <= cfine, cnt);
  R chi;
  if (chi_mode == 0) chi = R(1);
  else if (chi_mode == 1) chi = fast_exp2<R>(fma(c1, ad, c0));
  else chi = chi_any<R>(ad, G);
  return ad <= cfine ? f * chi : R(0);
}

// g(d) with the cut-off, plain or learned (wave-collective when SURR)
template <typename R, bool COUNT, bool SURR>
__device__ __forceinline__ R g_eval(R d, const typename RecOf<R>::T& L, const R* __restrict__ sp, int32_t j,
                                    const Geometry& G, R cfine, bool live, Counts& cnt, const LevelArgs& a) {
  if constexpr (SURR) {
    const float v = g_surr<COUNT>(d, L, sp, j, G, a, live && fabsf(d) <= cfine, cnt);
    return fabsf(d) <= cfine ? v : 0.0f;
  } else {
    (void)a;
    return g_any<R, COUNT>(d, L, sp, j, G, cfine, live, cnt);
  }
}

// Region pass: scan lines [j0, j1) of one window side (SGN = +1: d > 0,
// -1: d < 0, 0: both) and add g(d) for every (node, line) pair in the line's
// region at this level.
template <typename R, bool COUNT, int SGN, bool SURR>
__device__ __forceinline__ void scan_region(const typename RecOf<R>::T* __restrict__ rec, const R* __restrict__ sp,
                                            int32_t j0, int32_t j1,
                                            int S, int slice, int32_t X, bool active, R ra, R rb, bool chi_one,
                                            bool chi_mixed, R c0, R c1, int l, const Geometry& G, R cfine,
                                            R b_prev, R b_cur, R& acc, Counts& cnt, uint32_t& n_used,
                                            const LevelArgs& a) {
  using Rec = typename RecOf<R>::T;
  const bool generic = generic_shape(G);
  int32_t jn = j0 + slice;
  Rec Lnext = load_rec(rec, jn < j1 ? jn : j1 - 1);
  for (int32_t J = j0; J < j1; J += S) {
    const int32_t j = J + slice;
    const Rec L = Lnext;
    jn = j + S;
    if (J + S < j1) Lnext = load_rec(rec, jn < j1 ? jn : j1 - 1);
    const R d = R(X - L.k0) - R(L.frac);
    const R ad = fabs(d);
    bool in_win = active && j < j1 && ad >= ra && ad <= rb;
    if (SGN > 0) in_win = in_win && d > R(0);
    if (SGN < 0) in_win = in_win && d < R(0);
    const int ls = L.s;
    const R rlo = (l == ls) ? R(0) : b_prev;
    const bool in_reg = in_win && ls <= l && ad >= rlo && ad < b_cur && ad <= cfine;
    R val;
    if constexpr (SURR) {
      (void)generic;
      const float g = g_surr<COUNT>(d, L, sp, j, G, a, in_reg, cnt);
      val = in_reg ? g : R(0);
    } else if (!generic) {
      const R g = shape_fast<R, COUNT>(d, L, sp, j, G, in_reg, cnt);
      R chi;
      if (chi_one) chi = R(1);
      else if (!chi_mixed) chi = fast_exp2<R>(c0 + c1 * ad);
      else chi = chi_any<R>(ad, G);
      val = in_reg ? g * chi : R(0);
    } else {
      val = in_reg ? line_value<R, COUNT>(d, L, sp[j], G, cfine, cnt) : R(0);
    }
    acc += val;
    if (COUNT) {
      if (in_reg) n_used++;
      if ((threadIdx.x & 63) == 0) cnt.iters++;
    }
  }
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Line record j of a layer through a 32-bit byte offset from the layer's
// base in the global address space (plans keep a layer's records under
// 4 GiB), so the load can take the scalar-base + vector-offset form.
template <typename Rec>
__device__ __forceinline__ Rec load_rec(const Rec* __restrict__ rec, int32_t j) {
#if __HIP_DEVICE_COMPILE__
  typedef const __attribute__((address_space(1))) char gchar;
  typedef const __attribute__((address_space(1))) Rec grec;
  gchar* base = (gchar*)rec;
  return *(grec*)(base + (uint32_t)j * (uint32_t)sizeof(Rec));
#else
  return rec[j];   // host pass: parsed, never run
#endif
}

// Fast region scan over one window: SGN = +1 / -1 one side of the annulus
// |d| in [ra, rbx); SGN = 0 the own region |d| < rbx.  Each lane takes K
// consecutive level nodes (X0, X0 + rl, ...) against one line per step, so a
// line record is loaded and unpacked once per K pairs.  Lanes past the
// window's last line read that line again and are masked; act masks nodes
// outside the tile.  Lines with start level
// above smax are skipped.  CHIM: 0 no chi, 1 one exponential piece over the
// window, 2 any piece.  With one piece and a signed distance, chi of node k is
// chi of node k-1 times the constant exp2(c1 rl).
template <typename R, bool COUNT, int SGN, bool SURR, int CHIM, int K>
__device__ __forceinline__ void scan_fast(const typename RecOf<R>::T* __restrict__ rec, const R* __restrict__ sp,
                                          int32_t j0, int32_t j1, int S, int slice, int32_t X0, int32_t rl,
                                          uint32_t act, R ra, R rbx, int smax, R c0, R c1, const Geometry& G,
                                          R* acc, Counts& cnt, uint32_t& n_used, const LevelArgs& a,
                                          const CoreQueue& cq) {
  using Rec = typename RecOf<R>::T;
  const R c1s = SGN < 0 ? -c1 : c1;   // chi exponent slope in the signed distance
  const R chi_step = (CHIM == 1 && SGN != 0) ? fast_exp2<R>(c1s * R(rl)) : R(1);
  auto chi_of = [&](int k, R d, R& chi_run) -> R {
    if constexpr (CHIM == 0) {
      return R(1);
    } else if constexpr (CHIM == 1 && SGN != 0) {
      chi_run = (k == 0) ? fast_exp2<R>(fma(c1s, d, c0)) : chi_run * chi_step;
      return chi_run;
    } else if constexpr (CHIM == 1) {
      return fast_exp2<R>(fma(c1s, fabs(d), c0));
    } else {
      return chi_any<R>(fabs(d), G);
    }
  };
  auto step = [&](const Rec& L, int32_t j) {
    const int32_t n0 = X0 - L.k0;
    const R fr = R(L.frac);
    const bool lok = L.s <= smax && j < j1;
    R chi_run = R(1);
    if constexpr (sizeof(R) == 4 && !COUNT && !SURR) {
      // wing values first, core pairs through the wave's queue, then chi and
      // the accumulation in node order
      R d[K], f[K];
      bool reg[K], core[K];
      bool any = false;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        d[k] = R(n0 + k * rl) - fr;
        bool in_reg;
        if (SGN > 0) in_reg = d[k] >= ra && d[k] < rbx;
        else if (SGN < 0) in_reg = d[k] <= -ra && d[k] > -rbx;
        else in_reg = fabs(d[k]) < rbx;
        reg[k] = in_reg && lok && ((act >> k) & 1u);
        f[k] = shape_wing<R, false>(d[k] * R(kH0), L, reg[k], cnt, core[k]);
        any = any || core[k];
      }
      if (__builtin_amdgcn_ballot_w64(any)) core_batch<K>(cq, L, d, core, f, G);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const R chi = chi_of(k, d[k], chi_run);
        acc[k] += reg[k] ? f[k] * chi : R(0);
      }
      return;
    }
    if constexpr (SURR && !COUNT) {
      // learned shape: pairs in the trained domain through the wave's queue,
      // the others by the plain shape
      static_assert(K <= kSurrSlots, "one queue session holds a lane's nodes");
      float f[K];
      bool reg[K], queued[K];
      int pos[K];
      int n = 0;
      const float amp = L.A * 1.7724538509055160f * L.xs * L.xs;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float d = float(n0 + k * rl) - fr;
        bool in_reg;
        if (SGN > 0) in_reg = d >= ra && d < rbx;
        else if (SGN < 0) in_reg = d <= -ra && d > -rbx;
        else in_reg = fabsf(d) < rbx;
        reg[k] = in_reg && lok && ((act >> k) & 1u);
        float x, y;
        const bool dom = surr_domain(d, L, a, x, y);
        queued[k] = reg[k] && dom;
        f[k] = 0.0f;
        if (reg[k] && !dom) f[k] = shape_fast<float, false>(d, L, sp, j, G, true, cnt) * chi_any<float>(fabsf(d), G);
        pos[k] = surr_push(a.sq, queued[k], n, x, y, fabsf(d * float(kH0)));
      }
      if (n > 0) surr_batch(a.sq, n, a);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (queued[k]) f[k] = amp * a.sq[pos[k]];
        acc[k] += reg[k] ? f[k] : 0.0f;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R d = R(n0 + k * rl) - fr;
      bool in_reg;
      if (SGN > 0) in_reg = d >= ra && d < rbx;
      else if (SGN < 0) in_reg = d <= -ra && d > -rbx;
      else in_reg = fabs(d) < rbx;
      in_reg = in_reg && lok && ((act >> k) & 1u);
      if constexpr (SURR) {
        const float g = g_surr<COUNT>(d, L, sp, j, G, a, in_reg, cnt);
        acc[k] += in_reg ? g : R(0);
      } else {
        (void)a;
        const R g = shape_fast<R, COUNT>(d, L, sp, j, G, in_reg, cnt);
        const R chi = chi_of(k, d, chi_run);
        acc[k] += in_reg ? g * chi : R(0);
      }
      if (COUNT && in_reg) n_used++;
    }
  };
  int32_t j = j0 + slice;
  Rec La = load_rec(rec, j < j1 ? j : j1 - 1);
  for (int32_t J = j0; J < j1; J += 2 * S) {
    const Rec Lb = load_rec(rec, J + S + slice < j1 ? J + S + slice : j1 - 1);
    step(La, J + slice);
    La = load_rec(rec, J + 2 * S + slice < j1 ? J + 2 * S + slice : j1 - 1);
    if (COUNT && (threadIdx.x & 63) == 0) cnt.iters++;
    if (J + S < j1) {
      step(Lb, J + S + slice);
      if (COUNT && (threadIdx.x & 63) == 0) cnt.iters++;
    }
  }
}

// scan_fast with the window's chi mode as a template argument
template <typename R, bool COUNT, int SGN, bool SURR, int K>
__device__ __forceinline__ void scan_fast_chi(const typename RecOf<R>::T* __restrict__ rec, const R* __restrict__ sp,
                                              int32_t j0, int32_t j1, int S, int slice, int32_t X0, int32_t rl,
                                              uint32_t act, R ra, R rbx, int smax, bool chi_none, bool chi_mixed,
                                              R c0, R c1, const Geometry& G, R* acc, Counts& cnt, uint32_t& n_used,
                                              const LevelArgs& a, const CoreQueue& cq) {
  // the learned shape carries chi itself (its plain fallback uses chi_any):
  // one instantiation serves every chi mode
  if (SURR || chi_mixed)
    scan_fast<R, COUNT, SGN, SURR, 2, K>(rec, sp, j0, j1, S, slice, X0, rl, act, ra, rbx, smax, c0, c1, G, acc, cnt,
                                         n_used, a, cq);
  else if (chi_none)
    scan_fast<R, COUNT, SGN, SURR, 0, K>(rec, sp, j0, j1, S, slice, X0, rl, act, ra, rbx, smax, c0, c1, G, acc, cnt,
                                         n_used, a, cq);
  else
    scan_fast<R, COUNT, SGN, SURR, 1, K>(rec, sp, j0, j1, S, slice, X0, rl, act, ra, rbx, smax, c0, c1, G, acc, cnt,
                                         n_used, a, cq);
}

// Fast region pass of one wavefront tile of nw = 2^lnw nodes: groups of K
// consecutive nodes per lane, lane = group * S + slice, S = 64 K / nw line
// slices.  iv->fast_ok: 2 = the own region of lines starting at l (one
// window), 1 = the annulus [b_(l-1), b_l) of lines starting below l (two
// sides).  The line windows (my_j) are fetched by the caller.
template <typename R, bool COUNT, bool SURR, int K>
__device__ __forceinline__ void region_fast(const Geometry& G, const LevelArgs& a, int l, int layer, int lnw,
                                            int64_t rel0, int tile_left, const IntervalSet* iv, R* lds_acc,
                                            int64_t item_first, int32_t my_j, Counts& cnt, uint32_t& n_used,
                                            const CoreQueue& cq) {
  using Rec = typename RecOf<R>::T;
  constexpr int lK = K == 4 ? 2 : (K == 2 ? 1 : 0);
  const int lane = threadIdx.x & 63;
  const int lS = 6 - (lnw - lK);
  const int S = 1 << lS;
  const int node0 = (lane >> lS) * K;
  const int slice = lane & (S - 1);
  const int32_t rl = G.r[l];
  const Rec* rec = reinterpret_cast<const Rec*>(a.rec) + (int64_t)layer * a.n_lines;
  const R* sp = reinterpret_cast<const R*>(a.csp) + (int64_t)layer * a.n_lines;
  const int64_t m0 = G.lo[l] + rel0 + node0;
  const int32_t X0 = (int32_t)(m0 * rl);
  uint32_t act = 0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (rel0 + node0 + k < G.n[l] && node0 + k < tile_left) act |= 1u << k;
  R acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = R(0);
  const bool chi_mixed = iv->fchi_mixed != 0;
  const bool chi_none = !chi_mixed && iv->fc0 == 0.0 && iv->fc1 == 0.0;
  const R c0 = R(iv->fc0), c1 = R(iv->fc1);
  const int smax = uniform(iv->fast_need_s) ? l : kLevels;
  const R rbx = sizeof(R) == 4 ? R(iv->rbx32) : R(iv->rbx64);
  if (uniform(iv->fast_ok) == 2) {
    const int32_t j0 = uniform(__shfl(my_j, 0)), j1 = uniform(__shfl(my_j, 1));
    if (j0 < j1)
      scan_fast_chi<R, COUNT, 0, SURR, K>(rec, sp, j0, j1, S, slice, X0, rl, act, R(0), rbx, smax, chi_none,
                                          chi_mixed, c0, c1, G, acc, cnt, n_used, a, cq);
  } else {
    const R ra = sizeof(R) == 4 ? R(iv->ra32) : R(iv->ra64);
    for (int side = 0; side < 2; ++side) {
      const int32_t j0 = uniform(__shfl(my_j, 2 * side)), j1 = uniform(__shfl(my_j, 2 * side + 1));
      if (j0 >= j1) continue;
      if (side == 0)
        scan_fast_chi<R, COUNT, 1, SURR, K>(rec, sp, j0, j1, S, slice, X0, rl, act, ra, rbx, smax, chi_none,
                                            chi_mixed, c0, c1, G, acc, cnt, n_used, a, cq);
      else
        scan_fast_chi<R, COUNT, -1, SURR, K>(rec, sp, j0, j1, S, slice, X0, rl, act, ra, rbx, smax, chi_none,
                                             chi_mixed, c0, c1, G, acc, cnt, n_used, a, cq);
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    R v = acc[k];
    for (int o = S >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (((act >> k) & 1u) && slice == 0) lds_acc[m0 + k - G.lo[l] - item_first] = v;
  }
}



__device__ __forceinline__ int64_t bucket_of(double nu, const Geometry& G) {
  int64_t b = (int64_t)floor((nu - G.bucket_origin) * kBucketPerCm);
  return b < 0 ? 0 : (b > G.nbucket ? G.nbucket : b);
}

// Stencil of level-l node m on level l+1 (positions in fine units): G.ns
// coarse nodes centred on the nearest one (a tie goes to the lower) for 3
// and 5 points, the two on each side for 4 points; one node where m
// coincides with a coarse node
template <typename R>
__device__ __forceinline__ int stencil_of(const Geometry& G, int l, int64_t m, int32_t* Xs, R* ws) {
  const int64_t rl = G.r[l];
  const int64_t rho = G.r[l + 1] / rl;
  const int64_t q = floor_div(m, rho);
  const int64_t rem = m - q * rho;
  const int64_t r1 = G.r[l + 1];
  // at rem == 0 the stencil at t = 0 has weights (.., 0, 1, 0, ..) exactly
  const double f = (double)rem / (double)rho;
  if (G.ns == 4) {
    // the two coarse nodes on each side: q - 1 .. q + 2 at t = f
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      Xs[i] = (int32_t)((q - 1 + (i < 4 ? i : 3)) * r1);
      ws[i] = R(i < 4 ? lagrange_w4(i - 1, f) : 0.0);
    }
    return rem == 0 ? 1 : 4;
  }
  double tt;
  int64_t kc;
  if (f <= 0.5) { kc = q; tt = f; } else { kc = q + 1; tt = f - 1.0; }
  // both stencils, selected per slot (the 3-point one padded with zero weights)
  const bool five = G.ns == 5;
  const int64_t k0 = five ? kc - 2 : kc - 1;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    Xs[i] = (int32_t)((k0 + (i < 3 || five ? i : 2)) * r1);
    const double w3 = i < 3 ? lagrange_w<1>(i - 1, tt) : 0.0;
    ws[i] = R(five ? lagrange_w<2>(i - 2, tt) : w3);
  }
  return rem == 0 ? 1 : G.ns;
}

// Region pass of one wavefront tile: nw = 2^lnw consecutive nodes of level l;
// lane = node * S + slice, S = 64 / nw.  For every region window the tile
// walks the union of its nodes' line ranges, S consecutive lines per step
// (coalesced loads); node sums are reduced over slices and stored to LDS.
template <typename R, bool COUNT, bool SURR>
__device__ __forceinline__ void region_tile(const Geometry& G, const LevelArgs& a, int l, int layer, int lnw, int64_t rel0,
                            int tile_left, const IntervalSet* iv, R* lds_acc, int64_t item_first, Counts& cnt,
                            uint32_t& n_used, const CoreQueue& cq) {
  using Rec = typename RecOf<R>::T;
  const int lane = threadIdx.x & 63;
  const int nw = 1 << lnw;
  const int lS = 6 - lnw;
  const int S = 1 << lS;
  const int node = lane >> lS;
  const int slice = lane & (S - 1);
  const int32_t rl = G.r[l];
  const Rec* rec = reinterpret_cast<const Rec*>(a.rec) + (int64_t)layer * a.n_lines;
  const R* sp = reinterpret_cast<const R*>(a.csp) + (int64_t)layer * a.n_lines;
  const int32_t* bk = a.bucket + (int64_t)layer * (G.nbucket + 1);
  const R cfine = R(G.c_fine);
  const R b_prev = (l > 0) ? R(G.b[l - 1]) : R(0);
  const R b_cur = (l < kLevels - 1) ? R(G.b[l]) : R(INFINITY);
  const int64_t m = G.lo[l] + rel0 + node;
  const bool active = (rel0 + node < G.n[l]) && (node < tile_left);
  const int32_t X = (int32_t)(m * rl);
  const int64_t Xf = (G.lo[l] + rel0) * rl;
  const int64_t Xl = Xf + (int64_t)(nw - 1) * rl;
  // line ranges of every (window, side), fetched in one round.  Region
  // membership is decided on the single-precision distance, which can round
  // onto a window edge from outside; one fine unit of margin keeps such
  // lines in the scan, where the membership test decides.
  constexpr double kEdge = 1.0;
  const int n_iv = uniform(iv->n_iv);
  int nws = 0;
  int my_bucket = 0;
  for (int k = 0; k < n_iv; ++k) {
    const double ia = iv->a[k], ib = iv->b[k];
    const int nside = (ia == 0.0) ? 1 : 2;
    for (int side = 0; side < nside; ++side, ++nws) {
      double plo, phi;
      if (nside == 1) { plo = (double)Xf - ib - kEdge; phi = (double)Xl + ib + kEdge; }
      else if (side == 0) { plo = (double)Xf - ib - kEdge; phi = (double)Xl - ia + kEdge; }
      else { plo = (double)Xf + ia - kEdge; phi = (double)Xl + ib + kEdge; }
      const int64_t blo = bucket_of(plo * kH0, G);
      const int64_t bhi = bucket_of(phi * kH0, G) + 1 > G.nbucket ? G.nbucket : bucket_of(phi * kH0, G) + 1;
      if (lane == 2 * nws) my_bucket = (int)blo;
      if (lane == 2 * nws + 1) my_bucket = (int)bhi;
    }
  }
  const int32_t my_j = (lane < 2 * nws) ? bk[my_bucket] : 0;
  if (iv->fast_ok && !generic_shape(G)) {
    // K nodes per lane (up to 4, fewer for narrow tiles) in the single-
    // precision plain kernel; one elsewhere (the counting, learned-shape and
    // double-precision kernels are not timed and stay small)
    if constexpr (sizeof(R) == 4 && !COUNT) {
      if (lnw >= 2) {
        region_fast<R, COUNT, SURR, 4>(G, a, l, layer, lnw, rel0, tile_left, iv, lds_acc, item_first, my_j, cnt,
                                       n_used, cq);
        return;
      }
      if (lnw == 1) {
        region_fast<R, COUNT, SURR, 2>(G, a, l, layer, lnw, rel0, tile_left, iv, lds_acc, item_first, my_j, cnt,
                                       n_used, cq);
        return;
      }
    }
    region_fast<R, COUNT, SURR, 1>(G, a, l, layer, lnw, rel0, tile_left, iv, lds_acc, item_first, my_j, cnt, n_used,
                                   cq);
    return;
  }
  R acc = R(0);
  int ws_i = 0;
  for (int k = 0; k < n_iv; ++k) {
    const R ra = R(iv->a[k]), rb = R(iv->b[k]);
    const bool chi_mixed = iv->chi_mixed[k] != 0;
    const R c0 = R(iv->chi_c0[k]), c1 = R(iv->chi_c1[k]);
    const bool chi_one = !chi_mixed && iv->chi_c0[k] == 0.0 && iv->chi_c1[k] == 0.0;
    if (iv->a[k] == 0.0) {
      const int32_t j0 = uniform(__shfl(my_j, 2 * ws_i)), j1 = uniform(__shfl(my_j, 2 * ws_i + 1));
      ++ws_i;
      if (j0 < j1)
        scan_region<R, COUNT, 0, SURR>(rec, sp, j0, j1, S, slice, X, active, ra, rb, chi_one, chi_mixed, c0, c1, l, G, cfine,
                                 b_prev, b_cur, acc, cnt, n_used, a);
    } else {
      int32_t j0 = uniform(__shfl(my_j, 2 * ws_i)), j1 = uniform(__shfl(my_j, 2 * ws_i + 1));
      ++ws_i;
      if (j0 < j1)
        scan_region<R, COUNT, 1, SURR>(rec, sp, j0, j1, S, slice, X, active, ra, rb, chi_one, chi_mixed, c0, c1, l, G, cfine,
                                 b_prev, b_cur, acc, cnt, n_used, a);
      j0 = uniform(__shfl(my_j, 2 * ws_i));
      j1 = uniform(__shfl(my_j, 2 * ws_i + 1));
      ++ws_i;
      if (j0 < j1)
        scan_region<R, COUNT, -1, SURR>(rec, sp, j0, j1, S, slice, X, active, ra, rb, chi_one, chi_mixed, c0, c1, l, G, cfine,
                                  b_prev, b_cur, acc, cnt, n_used, a);
    }
  }
  for (int o = S >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (active && slice == 0) lds_acc[m - G.lo[l] - item_first] = acc;
}

// Residual-band pass: lane = one node of level l whose stencil on level l+1
// has three points.  For every jump q of T_(l+1) and side, the lane walks the
// lines whose |d| lies within reach of q (its own window), and for each line
// whose stencil hull holds a jump — counted at the smallest such jump only —
// adds D_l = T_l(d) - sum_i w_i T_(l+1)(d_i) minus the region value already
// added.
template <typename R, bool COUNT>
__device__ __forceinline__ void band_group(const Geometry& G, const LevelArgs& a, int l, int layer, int64_t rel0, int group_left,
                           const IntervalSet* iv, R* lds_acc, int64_t item_first, Counts& cnt, uint32_t& n_used,
                           uint32_t& n_band) {
  using Rec = typename RecOf<R>::T;
  const int lane = threadIdx.x & 63;
  const int32_t rl = G.r[l];
  const Rec* rec = reinterpret_cast<const Rec*>(a.rec) + (int64_t)layer * a.n_lines;
  const R* sp = reinterpret_cast<const R*>(a.csp) + (int64_t)layer * a.n_lines;
  const int32_t* bk = a.bucket + (int64_t)layer * (G.nbucket + 1);
  const R cfine = R(G.c_fine);
  const R b_prev = (l > 0) ? R(G.b[l - 1]) : R(0);
  const R b_cur = R(G.b[l]);
  const double hb = G.hb[l];
  const int64_t m = G.lo[l] + rel0 + lane;
  int32_t Xs[5];
  R ws[5];
  const int ns = stencil_of<R>(G, l, m, Xs, ws);
  const bool active = (rel0 + lane < G.n[l]) && (lane < group_left) && ns > 1;
  const int nsg = G.ns;
  const int32_t x_last = Xs[0] + (nsg - 1) * G.r[l + 1];   // stencil nodes are r_(l+1) apart
  if (!__any(active)) return;
  const int32_t X = (int32_t)(m * rl);
  const int nj = uniform(iv->n_jump);
  R acc = R(0);
  for (int k = 0; k < nj; ++k) {
    const double q = iv->jq[k];
    const R rq = R(q);
    for (int side = 0; side < 2; ++side) {
      // side 0: d > 0 (line below the node), side 1: d <= 0
      const double plo = side == 0 ? (double)X - q - hb : (double)X + q - hb;
      const double phi = side == 0 ? (double)X - q + hb : (double)X + q + hb;
      const int64_t b0 = bucket_of(plo * kH0, G);
      int64_t b1 = bucket_of(phi * kH0, G) + 1;
      b1 = b1 > G.nbucket ? G.nbucket : b1;
      const int32_t j0 = active ? bk[b0] : 0;
      const int32_t j1 = active ? bk[b1] : 0;
      for (int32_t j = j0; __any(j < j1); ++j) {
        if (j < j1) {
          const Rec L = rec[j];
          const R d = R(X - L.k0) - R(L.frac);
          const bool side_ok = side == 0 ? d > R(0) : !(d > R(0));
          const int ls = L.s;
          const int cls = (l >= ls) ? 1 : 2;
          const R d0 = R(Xs[0] - L.k0) - R(L.frac);
          const R d2 = R(x_last - L.k0) - R(L.frac);
          const R lo = (d0 * d2 <= R(0)) ? R(0) : fmin(fabs(d0), fabs(d2));
          const R hi = fmax(fabs(d0), fabs(d2));
          // the smallest straddled jump of this line's class
          R qmin = R(INFINITY);
          for (int i = 0; i < nj; ++i) {
            const R qi = R(iv->jq[i]);
            if ((iv->jmask[i] & cls) && qi >= lo && qi <= hi) qmin = fmin(qmin, qi);
          }
          if (side_ok && qmin == rq) {
            const R ad = fabs(d);
            const R rlo = (l == ls) ? R(0) : b_prev;
            const bool in_reg = ls <= l && ad >= rlo && ad < b_cur && ad <= cfine;
            const bool tl = ad <= cfine && !(l > ls && ad < b_prev);
            R v = R(0);
            if (tl && !in_reg) v = g_any<R, COUNT>(d, L, sp, j, G, cfine, true, cnt);
#pragma unroll
            for (int i = 0; i < 5; ++i) {
              if (i >= nsg) break;
              const R di = R(Xs[i] - L.k0) - R(L.frac);
              const R adi = fabs(di);
              if (adi <= cfine && !(l + 1 > ls && adi < b_cur)) v -= ws[i] * g_any<R, COUNT>(di, L, sp, j, G, cfine, true, cnt);
            }
            acc += v;
            if (COUNT) { n_band++; if (!in_reg) n_used++; }
          }
        }
        if (COUNT && lane == 0) cnt.band_iters++;
      }
    }
  }
  if (active) lds_acc[m - G.lo[l] - item_first] += acc;
}

// Segmented inclusive sum over the lanes of a wavefront, for a key that is
// non-decreasing over the lanes (a segment = lanes with equal keys), with DPP
// lane shifts (no LDS round trips): shifts by 1, 2, 4 and 8 inside each row of
// 16 lanes, then the broadcasts of lane 15 of a row to the next row and of lane
// 31 to the upper half.  Each step adds the shifted partial sum where its
// source lane lies in the same segment.  `last` marks the last lane of each
// segment, which ends with the segment's sum.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShl1 = 0x130;
struct SegSum {
  float m[6];   // 1 where step i's source lane is in this lane's segment
  bool last;
};
__device__ __forceinline__ SegSum seg_prepare(int32_t key) {
  SegSum g;
  const int32_t none = ~key;   // never equal to key: lanes without a source keep it
  const int32_t k1 = __builtin_amdgcn_update_dpp(none, key, kDppRowShr1, 0xf, 0xf, false);
  const int32_t k2 = __builtin_amdgcn_update_dpp(none, key, kDppRowShr2, 0xf, 0xf, false);
  const int32_t k4 = __builtin_amdgcn_update_dpp(none, key, kDppRowShr4, 0xf, 0xf, false);
  const int32_t k8 = __builtin_amdgcn_update_dpp(none, key, kDppRowShr8, 0xf, 0xf, false);
  const int32_t k15 = __builtin_amdgcn_update_dpp(none, key, kDppRowBcast15, 0xa, 0xf, false);
  const int32_t k31 = __builtin_amdgcn_update_dpp(none, key, kDppRowBcast31, 0xc, 0xf, false);
  const int32_t kn = __builtin_amdgcn_update_dpp(none, key, kDppWaveShl1, 0xf, 0xf, false);
  g.m[0] = k1 == key ? 1.0f : 0.0f;
  g.m[1] = k2 == key ? 1.0f : 0.0f;
  g.m[2] = k4 == key ? 1.0f : 0.0f;
  g.m[3] = k8 == key ? 1.0f : 0.0f;
  g.m[4] = k15 == key ? 1.0f : 0.0f;
  g.m[5] = k31 == key ? 1.0f : 0.0f;
  g.last = kn != key;
  return g;
}
template <int CTRL, int RMASK>
__device__ __forceinline__ float dpp_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RMASK, 0xf, false));
}
template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_shift(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, RMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, RMASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename R>
__device__ __forceinline__ R seg_sum(R v, const SegSum& g) {
  v = fma(dpp_shift<kDppRowShr1, 0xf>(v), R(g.m[0]), v);
  v = fma(dpp_shift<kDppRowShr2, 0xf>(v), R(g.m[1]), v);
  v = fma(dpp_shift<kDppRowShr4, 0xf>(v), R(g.m[2]), v);
  v = fma(dpp_shift<kDppRowShr8, 0xf>(v), R(g.m[3]), v);
  v = fma(dpp_shift<kDppRowBcast15, 0xa>(v), R(g.m[4]), v);
  v = fma(dpp_shift<kDppRowBcast31, 0xc>(v), R(g.m[5]), v);
  return v;
}

// One chunk of 64 lines of the line-major band pass for one jump and side:
// Layout of an NSP-point stencil on level l+1 for the RHO - 1 level-l nodes
// between coarse nodes: offsets -kLeft .. kRight from the stencil's base
// node -- the nearest coarse node for 3 and 5 points, the one below for the
// symmetric 4-point rule -- and the level-l offsets jj (kJlo .. kJhi, jj = 0
// coinciding) that the base serves.
template <int NSP, int RHO>
struct StencilShape {
  static constexpr bool kCentred = NSP != 4;
  static constexpr int kLeft = kCentred ? NSP / 2 : 1;
  static constexpr int kRight = kCentred ? NSP / 2 : 2;
  static constexpr int kJlo = kCentred ? -RHO / 2 + 1 : 1;
  static constexpr int kJhi = kCentred ? RHO / 2 : RHO - 1;
  // weight of stencil point i (0 .. NSP-1) for level-l offset jj
  static constexpr double weight(int i, int jj) {
    return kCentred ? lagrange_w<NSP / 2>(i - NSP / 2, (double)jj / (double)RHO)
                    : lagrange_w4(i - 1, (double)jj / (double)RHO);
  }
};

// NC candidate base nodes from kc0 with NSP-point stencils (see band_lines).
template <typename R, bool COUNT, int RHO, bool SURR, int NSP, int NC>
__device__ __forceinline__ void band_chunk(const typename RecOf<R>::T& L, int32_t jl, int ls, int cls, bool ok,
                                           int64_t kc0, int side, R rq, bool iso, const IntervalSet* iv,
                                           int chi_mode, R cc0, R cc1, int l, int32_t rl, int32_t r1, R cfine,
                                           R b_prev, R b_cur, int64_t m_a, int64_t m_b, int64_t base,
                                           const R* __restrict__ sp, const Geometry& G, const LevelArgs& a,
                                           R* lds_acc, Counts& cnt, uint32_t& n_used, uint32_t& n_band) {
  const int lane = threadIdx.x & 63;
  using SS = StencilShape<NSP, RHO>;
  constexpr int H = SS::kLeft;   // first stencil node: kc0 - H
  constexpr int NT = NC + NSP - 1;
  // T_(l+1) at level-(l+1) nodes kc0-H .. kc0+NC-1+kRight
  R dd[NT], T1[NT];
  if constexpr (SURR && !COUNT) {
    // learned shape: the stencil values through the wave's queue; a queued
    // slot holds its queue position (bit i of qmask) until the batch returns
    static_assert(NT <= kSurrSlots, "one queue session holds the stencil values");
    uint32_t qmask = 0;
    int n = 0;
    const float amp = L.A * 1.7724538509055160f * L.xs * L.xs;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      dd[i] = float((int32_t)((kc0 - H + i) * r1) - L.k0) - L.frac;
      const float adi = fabsf(dd[i]);
      const bool act = ok && adi <= cfine && !(l + 1 > ls && adi < b_cur);
      float x, y;
      const bool dom = surr_domain(dd[i], L, a, x, y);
      const bool queued = act && dom;
      T1[i] = 0.0f;
      if (act && !dom) T1[i] = g_any<float, false>(dd[i], L, sp, jl, G, cfine, true, cnt);
      const int pos = surr_push(a.sq, queued, n, x, y, adi * float(kH0));
      if (queued) {
        T1[i] = __int_as_float(pos);
        qmask |= 1u << i;
      }
    }
    if (n > 0) surr_batch(a.sq, n, a);
#pragma unroll
    for (int i = 0; i < NT; ++i)
      if ((qmask >> i) & 1u) T1[i] = amp * a.sq[__float_as_int(T1[i])];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  } else {
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      dd[i] = R((int32_t)((kc0 - H + i) * r1) - L.k0) - R(L.frac);
      const R adi = fabs(dd[i]);
      const bool act = ok && adi <= cfine && !(l + 1 > ls && adi < b_cur);
      const R g = g_band<R, COUNT, SURR>(dd[i], L, sp, jl, G, cfine, act, cnt, a, chi_mode, cc0, cc1);
      T1[i] = act ? g : R(0);
    }
  }
  // segments of lanes with equal kc0 (non-decreasing over lanes)
  const SegSum seg = seg_prepare((int32_t)kc0);
  const bool seg_end = seg.last;
  // at fine levels lines are sparse: no two lanes share a centre and the merge is skipped
  const bool merge = __builtin_amdgcn_ballot_w64(!seg.last) != 0;
  // does the stencil hull of centre kc0 + c straddle this jump (the smallest
  // straddled one of the line's class)?
  bool strad_c[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const R d0 = dd[c], d2 = dd[c + NSP - 1];
    const R lo = (d0 * d2 <= R(0)) ? R(0) : fmin(fabs(d0), fabs(d2));
    const R hi = fmax(fabs(d0), fabs(d2));
    if (iso) {
      strad_c[c] = ok && rq >= lo && rq <= hi;
    } else {
      R qmin = R(INFINITY);
      const int nj = uniform(iv->n_jump);
      for (int i = 0; i < nj; ++i) {
        const R qi = R(iv->jq[i]);
        if ((iv->jmask[i] & cls) && qi >= lo && qi <= hi) qmin = fmin(qmin, qi);
      }
      strad_c[c] = ok && qmin == rq;
    }
  }
  // the candidate node m = (kc0 + c) RHO + jj of a lane: distance, whether its
  // correction is used, and whether it needs the line's own value there
  auto node = [&](int c, int jj, R& d, bool& use, bool& need, bool& in_reg, bool& own) {
    const int64_t m = (kc0 + c) * RHO + jj;
    d = R((int32_t)(m * rl) - L.k0) - R(L.frac);
    const bool side_ok = side == 0 ? d > R(0) : !(d > R(0));
    own = m >= m_a && m <= m_b;
    use = strad_c[c] && own && side_ok;
    const R ad = fabs(d);
    const R rlo = (l == ls) ? R(0) : b_prev;
    in_reg = ls <= l && ad >= rlo && ad < b_cur && ad <= cfine;
    const bool tl = ad <= cfine && !(l > ls && ad < b_prev);
    need = use && tl && !in_reg;
  };
  R glv[NC][RHO];
  if constexpr (SURR && !COUNT) {
    // learned shape: the line's own values at the candidate nodes through the
    // queue (queued slots hold their position, bit c RHO + ji of qmask), in
    // sessions of CS centres so that a lane never holds more than kSurrSlots
    static_assert(NC * RHO <= 32, "one mask bit per candidate node");
    constexpr int kPer = SS::kJhi - SS::kJlo;   // interpolated nodes per centre
    constexpr int CS = kSurrSlots / kPer;
    static_assert(CS >= 1, "one queue session holds a centre's nodes");
    const float amp = L.A * 1.7724538509055160f * L.xs * L.xs;
#pragma unroll
    for (int cb = 0; cb < NC; cb += CS) {
      uint32_t qmask = 0;
      int n = 0;
#pragma unroll
      for (int c = cb; c < (cb + CS < NC ? cb + CS : NC); ++c)
#pragma unroll
        for (int jj = SS::kJlo; jj <= SS::kJhi; ++jj) {
          const int ji = jj - SS::kJlo;
          glv[c][ji] = 0.0f;
          if (jj == 0) continue;
          R d;
          bool use, need, in_reg, own;
          node(c, jj, d, use, need, in_reg, own);
          float x, y;
          const bool dom = surr_domain(d, L, a, x, y);
          const bool queued = need && dom;
          if (need && !dom) glv[c][ji] = g_any<float, false>(d, L, sp, jl, G, cfine, true, cnt);
          const int pos = surr_push(a.sq, queued, n, x, y, fabsf(d) * float(kH0));
          if (queued) {
            glv[c][ji] = __int_as_float(pos);
            qmask |= 1u << (c * RHO + ji);
          }
        }
      if (n > 0) surr_batch(a.sq, n, a);
#pragma unroll
      for (int c = cb; c < (cb + CS < NC ? cb + CS : NC); ++c)
#pragma unroll
        for (int ji = 0; ji < RHO; ++ji)
          if ((qmask >> (c * RHO + ji)) & 1u) glv[c][ji] = amp * a.sq[__float_as_int(glv[c][ji])];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int jj = SS::kJlo; jj <= SS::kJhi; ++jj) {
      if (jj == 0) continue;
      const int64_t m = (kc0 + c) * RHO + jj;
      R d;
      bool use, need, in_reg, own;
      node(c, jj, d, use, need, in_reg, own);
      R gl = R(0);
      if constexpr (SURR && !COUNT) {
        gl = glv[c][jj - SS::kJlo];
      } else {
        (void)glv;
        if (need) gl = g_band<R, COUNT, SURR>(d, L, sp, jl, G, cfine, need, cnt, a, chi_mode, cc0, cc1);
      }
      R interp = R(0);
#pragma unroll
      for (int i = 0; i < NSP; ++i) interp += R(SS::weight(i, jj)) * T1[c + i];
      const R v0 = (need ? gl : R(0)) - interp;
      R v = use ? v0 : R(0);
      if (merge) v = seg_sum<R>(v, seg);
      if (seg_end && own) lds_acc[m - base] += v;
      if (COUNT && use) { n_band++; if (!in_reg) n_used++; }
    }
  }
}

// Residual-band pass, line-major form, for one wavefront owning the item's
// nodes [own_lo, own_hi).  For a jump q of T_(l+1) and a side, put the
// line's jump point at P = nu~0 + q (nodes above the line) or nu~0 - q (nodes
// below).  A level-l node's stencil hull [(kc-H) r1, (kc+H) r1] (H = 1 for the
// 3-point stencil, 2 for the 5-point one) holds P only if its nearest
// level-(l+1) centre kc is within H steps of P / r1, so the nodes to correct
// are the (RHO - 1) interpolated nodes around each of 2H (2H + 1 when P / r1
// is an integer) centres.  Lane = line: T_(l+1) is evaluated once at
// the level-(l+1) nodes around P, every candidate node gets D_l = T_l(d) - sum w_i T_(l+1)(d_i)
// minus the region value (zero unless its hull straddles q and q is the
// smallest straddled jump), and a segmented sum over lanes with the same
// centre estimate -- non-decreasing in line order -- merges corrections of a
// node before one lane adds them to its LDS slot.  Per slot there is one
// writer and a fixed summation order, so results are reproducible.
template <typename R, bool COUNT, int RHO, bool SURR, int NSP>
__device__ __forceinline__ void band_lines(const Geometry& G, const LevelArgs& a, int l, int layer, int64_t item_first, int own_lo,
                           int own_hi, const IntervalSet* iv, R* lds_acc, Counts& cnt, uint32_t& n_used,
                           uint32_t& n_band) {
  using Rec = typename RecOf<R>::T;
  const int lane = threadIdx.x & 63;
  if (own_hi <= own_lo) return;
  const int32_t rl = G.r[l];
  const int32_t r1 = G.r[l + 1];
  const Rec* rec = reinterpret_cast<const Rec*>(a.rec) + (int64_t)layer * a.n_lines;
  const R* sp = reinterpret_cast<const R*>(a.csp) + (int64_t)layer * a.n_lines;
  const int32_t* bk = a.bucket + (int64_t)layer * (G.nbucket + 1);
  const R cfine = R(G.c_fine);
  const R b_prev = (l > 0) ? R(G.b[l - 1]) : R(0);
  const R b_cur = R(G.b[l]);
  const double eps = iv->lc_eps;
  const double inv_r1 = 1.0 / (double)r1;
  const int nj = uniform(iv->n_jump);
  const int64_t base = G.lo[l] + item_first;   // absolute index of the item's first node
  const int64_t m_a = base + own_lo, m_b = base + own_hi - 1;
  const bool iso = uniform(iv->jumps_isolated) != 0;
  for (int k = 0; k < nj; ++k) {
    const double q = iv->jq[k];
    const R rq = R(q);
    const int mask = iv->jmask[k];
    const int chi_mode = uniform(iv->jchi_mode[k]);
    const R cc0 = R(iv->jchi_c0[k]), cc1 = R(iv->jchi_c1[k]);
    for (int side = 0; side < 2; ++side) {
      const double sq = side == 0 ? q : -q;
      // lines whose candidate nodes can reach [m_a, m_b]
      const double marg = (NSP / 2 + 1.5) * r1 + 2.0;
      const double plo = (double)(m_a * rl) - marg - sq;
      const double phi = (double)(m_b * rl) + marg - sq;
      const int64_t b0 = bucket_of(plo * kH0, G);
      int64_t b1 = bucket_of(phi * kH0, G) + 1;
      b1 = b1 > G.nbucket ? G.nbucket : b1;
      const int32_t j0 = uniform(bk[b0]), j1 = uniform(bk[b1]);
      for (int32_t J = j0; J < j1; J += kWave) {
        const int32_t jl = (J + lane < j1) ? J + lane : j1 - 1;
        const Rec L = load_rec(rec, jl);
        const int ls = L.s;
        const int cls = (l >= ls) ? 1 : 2;
        const bool ok = (J + lane < j1) && (mask & cls);
        const double P = (double)L.k0 + (double)L.frac + sq;
        // Candidate centres: kc in [P/r1 - H, P/r1 + H].  Unless P/r1 lies
        // within single-precision rounding of an integer (eps), these are the
        // 2H centres from floor(P/r1) - H + 1; otherwise 2H + 1, from
        // floor(P/r1 + eps) - H.  The wavefront takes the wider set when any
        // of its used lanes needs it.
        // (4 points: base nodes k with [k - 1, k + 2] holding P / r1, i.e. the
        // kLeft + kRight = 3 bases from floor(P / r1) - 1, or 4 from
        // floor(P / r1 + eps) - 2.)
        constexpr int KL = StencilShape<NSP, RHO>::kLeft, KR = StencilShape<NSP, RHO>::kRight;
        const double Pr = P * inv_r1;
        const double fl = floor(Pr);
        const bool edge = (Pr - fl) < eps || (Pr - fl) > 1.0 - eps;
        if (__builtin_amdgcn_ballot_w64(ok && edge))
          band_chunk<R, COUNT, RHO, SURR, NSP, KL + KR + 1>(L, jl, ls, cls, ok, (int64_t)floor(Pr + eps) - KR, side,
                                                            rq, iso, iv, chi_mode, cc0, cc1, l, rl, r1, cfine, b_prev,
                                                            b_cur, m_a, m_b, base, sp, G, a, lds_acc, cnt, n_used,
                                                            n_band);
        else
          band_chunk<R, COUNT, RHO, SURR, NSP, KL + KR>(L, jl, ls, cls, ok, (int64_t)fl - KR + 1, side, rq, iso, iv,
                                                        chi_mode, cc0, cc1, l, rl, r1, cfine, b_prev, b_cur, m_a, m_b,
                                                        base, sp, G, a, lds_acc, cnt, n_used, n_band);
        if (COUNT && lane == 0) cnt.band_iters++;
      }
    }
  }
}

#ifndef MARFA_STENCILS
#define MARFA_STENCILS 7
#endif

// Persistent work queue: each workgroup takes items (consecutive nodes of one
// level of one layer, heaviest levels first).  Its four wavefronts split the
// item into region tiles, then into band groups of 64 nodes; node sums meet in
// LDS and are written once.
template <typename R, bool COUNT, bool SURR>
__device__ __forceinline__ void level_body(const Geometry& G, const LevelArgs& a_in) {
  extern __shared__ char smem_raw[];
  R* lds_acc = reinterpret_cast<R*>(smem_raw);
  LevelArgs a = a_in;
  if constexpr (SURR) {
    // the learned line shape's weights, staged once per workgroup in the
    // scaled form that mlp_forward_wave<true> takes
    __shared__ float4 s_w0b[kMlpHid];
    __shared__ uint4 s_wp[kMlpHidLayers * 8 * 64];
    __shared__ float s_bh[kMlpHidLayers * kMlpHid];
    __shared__ float s_w4[kMlpHid];
    __shared__ float s_b4[1];
    for (int i = threadIdx.x; i < kMlpHid; i += 256) {
      s_w0b[i] = mlp_scaled_w0b(a_in.mlp.w0b[i]);
      s_w4[i] = mlp_scaled_w4(a_in.mlp.w4[i]);
    }
    for (int i = threadIdx.x; i < kMlpHidLayers * 8 * 64; i += 256) s_wp[i] = a_in.mlp.wp[i];
    for (int i = threadIdx.x; i < kMlpHidLayers * kMlpHid; i += 256) s_bh[i] = mlp_scaled_bh(a_in.mlp.bh[i]);
    if (threadIdx.x == 0) s_b4[0] = a_in.mlp.b4[0];
    __syncthreads();
    a.mlp.w0b = s_w0b;
    a.mlp.wp = s_wp;
    a.mlp.bh = s_bh;
    a.mlp.w4 = s_w4;
    a.mlp.b4 = s_b4;
  }
  __shared__ int64_t s_item;
  const int wv = threadIdx.x >> 6;
  if constexpr (SURR) {
    __shared__ float s_sq[4][3 * kSurrQueue];
    a.sq = s_sq[wv];
  }
  CoreQueue cq{nullptr, nullptr, nullptr, nullptr};
  if constexpr (sizeof(R) == 4 && !COUNT && !SURR) {
    __shared__ float s_cq[4][kCoreQueue + 128];
    __shared__ uint8_t s_cqs[4][kCoreQueue];
    cq.x = s_cq[wv];
    cq.y = s_cq[wv] + kCoreQueue;
    cq.amp = s_cq[wv] + kCoreQueue + 64;
    cq.src = s_cqs[wv];
  }
  const int lane = threadIdx.x & 63;
  const int64_t total = a.n_tiles * a.n_layers;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t item_v = s_item;
    const int64_t item = (int64_t)(((uint64_t)(uint32_t)uniform((int)(item_v >> 32)) << 32) |
                                   (uint32_t)uniform((int)item_v));
    if (item >= total) break;
    const int tix = uniform((int)(item / a.n_layers));
    const int layer = uniform((int)(item % a.n_layers));
    const int l = uniform(a.tiles[tix].level);
    const int count = uniform(a.tiles[tix].count);
    const int64_t first = a.tiles[tix].first;
    const int32_t* gc = a.gcount + layer * (kGroups + 1);
    int below = 0, above = 0;
    for (int g = 0; g < l; ++g) below += gc[g];
    for (int g = l + 1; g < kGroups; ++g) above += gc[g];
    const int combo = uniform((below > 0 ? 1 : 0) | (gc[l] > 0 ? 2 : 0) | (above > 0 ? 4 : 0));
    const IntervalSet* iv = a.ivs + (l * 8 + combo);
    Counts cnt{0, 0, 0, 0, 0};
    uint32_t n_used = 0, n_band = 0;
    // region pass
    const int lnw = G.lnw[l];
    const int ntile = (count + (1 << lnw) - 1) >> lnw;
    for (int t = wv; t < ntile; t += 4)
      region_tile<R, COUNT, SURR>(G, a, l, layer, lnw, first + ((int64_t)t << lnw), count - (t << lnw), iv, lds_acc,
                            first, cnt, n_used, cq);
    __syncthreads();
    // residual-band pass
    if (l < kLevels - 1 && iv->n_jump > 0) {
      if (iv->lc_ok) {
        // each wavefront owns a contiguous quarter of the item's nodes
        const int own_lo = (int)(((int64_t)count * wv) >> 2);
        const int own_hi = (int)(((int64_t)count * (wv + 1)) >> 2);
        const bool two = G.r[l + 1] == 2 * G.r[l];
        // the stencils this kernel is built with (MARFA_STENCILS: bit 0 the
        // 3-point, bit 1 the 4-point, bit 2 the 5-point rule)
        bool done = false;
        if constexpr ((MARFA_STENCILS & 4) != 0) {
          if (G.ns == 5) {
            if (two)
              band_lines<R, COUNT, 2, SURR, 5>(G, a, l, layer, first, own_lo, own_hi, iv, lds_acc, cnt, n_used, n_band);
            else
              band_lines<R, COUNT, 4, SURR, 5>(G, a, l, layer, first, own_lo, own_hi, iv, lds_acc, cnt, n_used, n_band);
            done = true;
          }
        }
        if constexpr ((MARFA_STENCILS & 2) != 0) {
          if (!done && G.ns == 4) {
            if (two)
              band_lines<R, COUNT, 2, SURR, 4>(G, a, l, layer, first, own_lo, own_hi, iv, lds_acc, cnt, n_used, n_band);
            else
              band_lines<R, COUNT, 4, SURR, 4>(G, a, l, layer, first, own_lo, own_hi, iv, lds_acc, cnt, n_used, n_band);
            done = true;
          }
        }
        if constexpr ((MARFA_STENCILS & 1) != 0) {
          if (!done) {
            if (two)
              band_lines<R, COUNT, 2, SURR, 3>(G, a, l, layer, first, own_lo, own_hi, iv, lds_acc, cnt, n_used, n_band);
            else
              band_lines<R, COUNT, 4, SURR, 3>(G, a, l, layer, first, own_lo, own_hi, iv, lds_acc, cnt, n_used, n_band);
          }
        }
        (void)done;
      } else {
        const int ngroup = (count + 63) >> 6;
        for (int g = wv; g < ngroup; g += 4)
          band_group<R, COUNT>(G, a, l, layer, first + ((int64_t)g << 6), count - (g << 6), iv, lds_acc, first, cnt,
                               n_used, n_band);
      }
    }
    __syncthreads();
    if (COUNT) {
      unsigned long long v[7] = {n_used, n_band, cnt.core, cnt.wing, cnt.terms, cnt.iters, cnt.band_iters};
      for (int i = 0; i < 7; ++i) {
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
        atomicAdd(&a.stats[16 + l], v[5]);
        atomicAdd(&a.stats[27 + l], v[6]);
      }
    } else {
      for (int i = threadIdx.x; i < count; i += 256) {
        const R v = lds_acc[i];
        if (l == 0)
          reinterpret_cast<R*>(a.out)[(int64_t)layer * a.stride + first + i] = v;
        else
          reinterpret_cast<R*>(a.A)[(int64_t)layer * G.a_total + G.aoff[l] + first + i] = v;
      }
    }
  }
}


}  // namespace marfa

// Defines one instantiation of the level kernel and its launcher; WAVES is
// the occupancy (wavefronts per SIMD) the register allocation must allow.
#define MARFA_LEVEL_LAUNCHER(TAG, R, COUNT, SURR, WAVES)                                          \
  namespace marfa {                                                                              \
  __global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES)))             \
      k_level_##TAG(Geometry G, LevelArgs a) {                                                   \
    level_body<R, COUNT, SURR>(G, a);                                                            \
  }                                                                                              \
  void launch_level_##TAG(const Geometry& G, const LevelArgs& a, int grid, hipStream_t s) {      \
    const size_t smem = (size_t)a.max_item * sizeof(R);                                           \
    k_level_##TAG<<<grid, 256, smem, s>>>(G, a);                                                 \
  }                                                                                              \
  }
