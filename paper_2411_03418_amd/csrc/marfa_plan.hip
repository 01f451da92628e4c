// marfa_plan.hip -- host runtime and C ABI of the eleven-grid library.
//
// A plan owns the uploaded line list, the per-layer workspace and one HIP
// graph holding the whole hot path (line preparation, level accumulation,
// cascade).  See include/marfa.h for the contract of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "marfa.h"
#include "marfa_internal.h"
#include "marfa_user.h"

using namespace marfa;

// ------------------------------------------------------------------
// errors
// ------------------------------------------------------------------
static thread_local std::string g_err;

static marfa_status fail(marfa_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(MARFA_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------
// Weideman coefficients: psi(t) = (L^2 + t^2) exp(-t^2) expanded in
// Z(t)^n = ((L+it)/(L-it))^n; with t = L tan(theta/2) the a_n are the Fourier
// cosine coefficients of psi(L tan(theta/2)), computed by the trapezoid rule.
// ------------------------------------------------------------------
static void weideman_coeffs(int N, double* a, double* Lout) {
  const double L = std::pow(2.0, -0.25) * std::sqrt((double)N);
  const int M = 16 * N;
  const double pi = 3.14159265358979323846;
  std::vector<double> psi(M), th(M);
  for (int k = 0; k < M; ++k) {
    th[k] = -pi + 2.0 * pi * k / M;
    if (k == 0) { psi[k] = 0.0; continue; }
    double t = L * std::tan(0.5 * th[k]);
    psi[k] = (L * L + t * t) * std::exp(-t * t);
  }
  for (int n = 0; n <= N; ++n) {
    double s = 0.0;
    for (int k = 0; k < M; ++k) s += psi[k] * std::cos(n * th[k]);
    a[n] = s / M;
  }
  *Lout = L;
}

// Faddeeva function w(z) = exp(-z^2) erfc(-iz) in double precision on the host,
// by the Weideman series (coefficients a, scale L) for Im z >= 0 and the
// reflection w(z) = 2 exp(-z^2) - w(-z) below the real axis.
static std::complex<double> host_faddeeva(std::complex<double> z, const double* a, int N, double L) {
  if (z.imag() < 0.0) return 2.0 * std::exp(-z * z) - host_faddeeva(-z, a, N, L);
  const std::complex<double> I(0.0, 1.0);
  const std::complex<double> A = L - I * z;
  const std::complex<double> Z = (L + I * z) / A;
  std::complex<double> P = a[N];
  for (int n = N - 1; n >= 1; --n) P = P * Z + a[n];
  return 1.0 / (std::sqrt(M_PI) * A) + 2.0 * P / (A * A);
}

// Taylor coefficients c_n = w^(n)(z0)/n!, n < kTaylorTerms, about every centre
// z0 = (i + j sqrt(-1)) / kTaylorPerUnit, by the trapezoid rule for Cauchy's
// integral on a circle of radius 0.6 around z0 (64 points; w is entire, so the
// rule converges geometrically).  On the real axis (j = 0) the real parts are
// the closed forms d^n/dx^n exp(-x^2)/n! = (-1)^n H_n(x) exp(-x^2)/n! (Hermite
// polynomials by their recurrence), which are tiny there and must not carry the
// integral's absolute rounding.  Packed per centre as float4 quads (re c_2k,
// im c_2k, re c_2k+1, im c_2k+1), the last quad (re c_8, im c_8, 0, 0).
static void taylor_table(const double* a, int N, double L, float* out) {
  const int M = 64;
  const double rho = 0.6;
  for (int j = 0; j < kTaylorSide; ++j)
    for (int i = 0; i < kTaylorSide; ++i) {
      const std::complex<double> z0((double)i / kTaylorPerUnit, (double)j / kTaylorPerUnit);
      std::complex<double> c[kTaylorTerms];
      for (int n = 0; n < kTaylorTerms; ++n) c[n] = 0.0;
      for (int k = 0; k < M; ++k) {
        const double th = 2.0 * M_PI * k / M;
        const std::complex<double> wv = host_faddeeva(z0 + std::polar(rho, th), a, N, L);
        for (int n = 0; n < kTaylorTerms; ++n) c[n] += wv * std::polar(1.0, -n * th);
      }
      for (int n = 0; n < kTaylorTerms; ++n) c[n] /= (double)M * std::pow(rho, n);
      if (j == 0) {
        const double x = z0.real();
        double H[kTaylorTerms + 1];
        H[0] = 1.0;
        H[1] = 2.0 * x;
        for (int n = 1; n < kTaylorTerms; ++n) H[n + 1] = 2.0 * x * H[n] - 2.0 * n * H[n - 1];
        double fact = 1.0;
        for (int n = 0; n < kTaylorTerms; ++n) {
          if (n > 0) fact *= n;
          const double re = ((n & 1) ? -1.0 : 1.0) * H[n] * std::exp(-x * x) / fact;
          c[n] = std::complex<double>(re, c[n].imag());
        }
      }
      float* q = out + (size_t)(j * kTaylorSide + i) * kTaylorQuads * 4;
      for (int n = 0; n < kTaylorQuads * 2; ++n) {
        const std::complex<double> v = n < kTaylorTerms ? c[n] : std::complex<double>(0.0, 0.0);
        q[2 * n] = (float)v.real();
        q[2 * n + 1] = (float)v.imag();
      }
    }
}

static std::mutex g_dev_mu;
static bool g_dev_ready[64];
static DeviceTables* g_tabs[64];   // per-device coefficient tables, kept until the process ends

static marfa_status ensure_device(int device) {
  int cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0) return fail(MARFA_E_DEVICE, "no HIP device");
  if (device < 0 || device >= cnt || device >= 64) return fail(MARFA_E_DEVICE, "device %d out of range", device);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(MARFA_E_DEVICE, "device %d is %s, not gfx950", device, prop.gcnArchName);
  HIP_TRY(hipSetDevice(device));
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (!g_dev_ready[device]) {
    std::vector<DeviceTables> host(1);
    DeviceTables& t = host[0];
    weideman_coeffs(kWeidemanN64, t.weid, &t.weid[kWeidemanN64 + 1]);
    taylor_table(t.weid, kWeidemanN64, t.weid[kWeidemanN64 + 1], t.taylor);
    DeviceTables* d = nullptr;
    HIP_TRY(hipMalloc((void**)&d, sizeof(DeviceTables)));
    hipError_t e = hipMemcpy(d, &t, sizeof(DeviceTables), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return fail(MARFA_E_DEVICE, "coefficient upload: %s", hipGetErrorString(e));
    }
    g_tabs[device] = d;
    g_dev_ready[device] = true;
  }
  return MARFA_OK;
}

namespace marfa {
const DeviceTables* device_tables(int device) { return (device >= 0 && device < 64) ? g_tabs[device] : nullptr; }
marfa_status marfa_set_error(marfa_status st, const char* msg) { return fail(st, "%s", msg); }
marfa_status marfa_use_device(int device) { return ensure_device(device); }
}  // namespace marfa

// ------------------------------------------------------------------
// plan
// ------------------------------------------------------------------
struct marfa_plan {
  int device = 0;
  marfa_request req{};
  int64_t n_lines = 0;
  double molar_mass = 44.0;
  int32_t n_layers = 0;
  int nblk = 0;
  Geometry G{};
  std::vector<IntervalSet> ivs;
  std::vector<Tile> tiles;
  std::vector<Tile> stiles;   // work items of the learned-shape kernel
  std::vector<double> layers_h;
  std::vector<double> span_h;
  DeviceBuffers d;
  int grid = 0;
  int cu_count = 0;
  // graph cache
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void* g_out = nullptr;
  int64_t g_stride = 0;
  hipStream_t cap = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraph_t sgraph[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t sexec[3] = {nullptr, nullptr, nullptr};
  void* s_out = nullptr;
  int64_t s_stride = 0;
  // tile parameters (autotuned by marfa_plan_tune)
  int base_nodes = 256;
  int blocks_per_cu = 8;
  int64_t tiles_cap = 0;   // capacity of d.tiles (tile count at the smallest item size)
  int tuned = 0;
  float tune_ms = 0.f;
  // learned line shape
  const marfa_surrogate* surr = nullptr;
  MlpDev mlp{};
  float mlp_xmax = 0.f, mlp_inv_c = 0.f;
};

// evaluation view of a trained surrogate (defined with the surrogate object)
bool marfa_surrogate_view(const marfa_surrogate* s, MlpDev* W, double* x_max, int32_t* chi, double* cutoff,
                          int* device);

static int64_t fdiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// Nodes per wavefront tile by level: all 64 lanes on consecutive nodes at the
// finest level (short windows), 16 nodes x 4 line slices above it.
static int default_lnw(int l) { return l == 0 ? 6 : 4; }

static void make_geometry(const marfa_request& rq, double nu_max, Geometry& G) {
  G.ns = rq.stencil == 0 ? 3 : rq.stencil;
  const int half = G.ns / 2;   // coarse nodes a stencil reaches beyond its interval: 1, 2, 2
  for (int l = 0; l < kLevels; ++l) {
    if (rq.level_table == 1) G.r[l] = 1 << l;
    else G.r[l] = l == 0 ? 1 : (1 << (l + 1));
    G.lnw[l] = default_lnw(l);
  }
  G.lo[0] = (int64_t)std::llround(rq.nu_begin * 2048.0);
  int64_t hi[kLevels];
  hi[0] = (int64_t)std::llround(rq.nu_end * 2048.0);
  for (int l = 0; l < kLevels - 1; ++l) {
    int64_t rho = G.r[l + 1] / G.r[l];
    G.lo[l + 1] = fdiv(G.lo[l], rho) - half;
    hi[l + 1] = -fdiv(-hi[l], rho) + half;
  }
  int64_t off = 0;
  for (int l = 0; l < kLevels; ++l) {
    G.n[l] = hi[l] - G.lo[l] + 1;
    if (l >= 1) {
      G.aoff[l] = off;
      off += G.n[l];
    } else {
      G.aoff[l] = 0;
    }
  }
  G.a_total = off;
  const double c = rq.cutoff * 2048.0;
  for (int l = 0; l < kLevels - 1; ++l) {
    G.b[l] = rq.R * G.r[l + 1];
    G.hb[l] = (half + 0.5) * G.r[l + 1] + 1.0;
  }
  G.b[kLevels - 1] = INFINITY;
  G.hb[kLevels - 1] = 0.0;
  G.c_fine = c;
  // |d| where chi jumps (fine units): Eq.(10)'s piece ends, or the user chi's breaks
  std::vector<double> br;
  if (rq.chi == MARFA_CHI_TONKOV) br = {3.0 * 2048.0, 150.0 * 2048.0, 300.0 * 2048.0};
  if (rq.chi == MARFA_CHI_USER)
    for (int i = 0; i < MarfaUserChi::kBreaks; ++i) br.push_back(MarfaUserChi::kBreak[i] * 2048.0);
  for (int l = 0; l < kLevels; ++l) {
    G.nq1[l] = G.nq2[l] = 0;
    if (l == kLevels - 1) continue;
    // lines starting at or below l: T_(l+1) = g on [b_l, c]
    if (G.b[l] <= c) {
      std::vector<double> q{G.b[l], c};
      for (double v : br)
        if (v >= G.b[l] && v <= c) q.push_back(v);
      std::sort(q.begin(), q.end());
      q.erase(std::unique(q.begin(), q.end()), q.end());
      for (size_t i = 0; i < q.size(); ++i) G.q1[l][i] = q[i];
      G.nq1[l] = (int)q.size();
    }
    // lines starting above l: T_(l+1) = g on [0, c]
    std::vector<double> q2{c};
    for (double v : br)
      if (v <= c) q2.push_back(v);
    std::sort(q2.begin(), q2.end());
    q2.erase(std::unique(q2.begin(), q2.end()), q2.end());
    for (size_t i = 0; i < q2.size(); ++i) G.q2[l][i] = q2[i];
    G.nq2[l] = (int)q2.size();
  }
  G.shape = rq.shape;
  G.chi = rq.chi;
  G.out_kind = rq.out_kind;
  G.fp64 = rq.fp64;
  G.nbucket = (int32_t)std::ceil((nu_max + 1.0) * kBucketPerCm) + 1;
  // Eq.(10): 1.084 e^{-0.027|d|}, 0.208 e^{-0.016|d|}, 0.025 e^{-0.009|d|}
  const double l2e = 1.0 / std::log(2.0);
  G.chi_c0[0] = std::log2(1.084); G.chi_c1[0] = -0.027 * l2e;
  G.chi_c0[1] = std::log2(0.208); G.chi_c1[1] = -0.016 * l2e;
  G.chi_c0[2] = std::log2(0.025); G.chi_c1[2] = -0.009 * l2e;
}

// |d| windows a level must scan, for each combination of start-level classes
// present in a layer (bit 0: s < l, bit 1: s == l, bit 2: s > l): regions and
// the reach 1.5 h_(l+1) around the jumps of T_(l+1).  Each window carries the
// jumps within its reach and, when chi is one exponential piece over the
// whole window, that piece as exp2(c0 + c1 |d|).
static bool make_intervals(const Geometry& G, int chi, std::vector<IntervalSet>& out) {
  out.assign(kLevels * 8, IntervalSet{});
  const double c = G.c_fine;
  for (int l = 0; l < kLevels; ++l) {
    for (int combo = 0; combo < 8; ++combo) {
      std::vector<std::pair<double, double>> iv;
      const bool top = (l == kLevels - 1);
      if ((combo & 1) && l > 0) {
        double hi = top ? c : std::min(G.b[l], c);
        if (G.b[l - 1] <= hi) iv.push_back({G.b[l - 1], hi});
      }
      if (combo & 2) iv.push_back({0.0, top ? c : std::min(G.b[l], c)});
      std::sort(iv.begin(), iv.end());
      std::vector<std::pair<double, double>> merged;
      for (auto& p : iv) {
        if (!merged.empty() && p.first <= merged.back().second)
          merged.back().second = std::max(merged.back().second, p.second);
        else
          merged.push_back(p);
      }
      if ((int)merged.size() > kMaxIntervals) return false;
      IntervalSet& S = out[l * 8 + combo];
      S.n_iv = (int)merged.size();
      for (size_t i = 0; i < merged.size(); ++i) {
        const double a = merged[i].first, b = merged[i].second;
        S.a[i] = a;
        S.b[i] = b;
        const double A = a / 2048.0, B = b / 2048.0;
        S.chi_mixed[i] = 0;
        S.chi_c0[i] = 0.0;
        S.chi_c1[i] = 0.0;
        if (chi == MARFA_CHI_TONKOV) {
          const int piece_a = A < 3.0 ? 0 : (A <= 150.0 ? 1 : (A <= 300.0 ? 2 : 3));
          const int piece_b = B < 3.0 ? 0 : (B <= 150.0 ? 1 : (B <= 300.0 ? 2 : 3));
          if (piece_a != piece_b) {
            S.chi_mixed[i] = 1;
          } else if (piece_a > 0) {
            S.chi_c0[i] = G.chi_c0[piece_a - 1];
            S.chi_c1[i] = G.chi_c1[piece_a - 1] / 2048.0;
          }
        } else if (chi == MARFA_CHI_USER) {
          S.chi_mixed[i] = 1;  // no separable form known: evaluated pair by pair
        }
      }
      // fast region test: every line with a region here starts below l (one
      // annulus window), or none starts below l (the own region); lines that
      // start above l are skipped by their start level
      S.fast_ok = 0;
      S.fast_need_s = 0;
      const bool annulus = (combo == 1 || combo == 5) && l > 0 && S.n_iv == 1;
      const bool own = (combo == 2 || combo == 6) && S.n_iv == 1;
      if (annulus || own) {
        const double ra = annulus ? G.b[l - 1] : 0.0;
        const double bl = top ? INFINITY : G.b[l];
        double rbx64;
        float rbx32;
        bool incl_c = c < bl;
        if (incl_c) {
          rbx64 = std::nextafter(c, INFINITY);
          rbx32 = std::nextafterf((float)c, INFINITY);
        } else {
          rbx64 = bl;
          rbx32 = (float)bl;
        }
        S.fast_ok = annulus ? 1 : 2;
        S.fast_need_s = (combo & 4) ? 1 : 0;
        S.ra64 = ra;
        S.rbx64 = rbx64;
        S.ra32 = (float)ra;
        S.rbx32 = rbx32;
        // chi over [ra, rbx): lowest and highest |d| of the range, in cm
        auto piece_incl = [](double x) { return x < 3.0 ? 0 : (x <= 150.0 ? 1 : (x <= 300.0 ? 2 : 3)); };
        auto piece_below = [](double x) { return x <= 3.0 ? 0 : (x <= 150.0 ? 1 : (x <= 300.0 ? 2 : 3)); };
        const int pa = piece_incl(ra / 2048.0);
        const int pb = incl_c ? piece_incl(c / 2048.0) : piece_below(bl / 2048.0);
        S.fchi_mixed = 0;
        S.fc0 = 0.0;
        S.fc1 = 0.0;
        if (chi == MARFA_CHI_TONKOV) {
          if (pa != pb) S.fchi_mixed = 1;
          else if (pa > 0) {
            S.fc0 = G.chi_c0[pa - 1];
            S.fc1 = G.chi_c1[pa - 1] / 2048.0;
          }
        } else if (chi == MARFA_CHI_USER) {
          S.fchi_mixed = 1;
        }
      }
      // jumps of T_(l+1) for the classes present, merged by value
      std::vector<std::pair<double, int>> jumps;
      if (!top) {
        if (combo & 3)
          for (int i = 0; i < G.nq1[l]; ++i) jumps.push_back({G.q1[l][i], 1});
        if (combo & 4)
          for (int i = 0; i < G.nq2[l]; ++i) jumps.push_back({G.q2[l][i], 2});
      }
      std::sort(jumps.begin(), jumps.end());
      std::vector<std::pair<double, int>> qs;
      for (auto& jq : jumps) {
        if (!qs.empty() && qs.back().first == jq.first) qs.back().second |= jq.second;
        else qs.push_back(jq);
      }
      if ((int)qs.size() > kMaxJumps) return false;
      S.n_jump = (int)qs.size();
      for (size_t k = 0; k < qs.size(); ++k) {
        S.jq[k] = qs[k].first;
        S.jmask[k] = qs[k].second;
      }
      S.jumps_isolated = 1;
      for (size_t k = 1; k < qs.size(); ++k)
        if (qs[k].first - qs[k - 1].first <= 2.0 * (G.ns - 1) * G.r[l + (top ? 0 : 1)] + 4.0) S.jumps_isolated = 0;
      for (size_t k = 0; k < qs.size(); ++k) {
        S.jchi_mode[k] = 0;
        S.jchi_c0[k] = 0.0;
        S.jchi_c1[k] = 0.0;
        if (chi == MARFA_CHI_NONE || top) continue;
        if (chi == MARFA_CHI_USER) {
          S.jchi_mode[k] = 2;
          continue;
        }
        const double reach = G.ns * G.r[l + 1] + 4.0;
        const double lo = std::max(0.0, qs[k].first - reach) / 2048.0, hi = (qs[k].first + reach) / 2048.0;
        auto piece = [](double x) { return x < 3.0 ? 0 : (x <= 150.0 ? 1 : (x <= 300.0 ? 2 : 3)); };
        const int pa = piece(lo), pb = piece(hi);
        if (pa != pb) {
          S.jchi_mode[k] = 2;
        } else if (pa > 0) {
          S.jchi_mode[k] = 1;
          S.jchi_c0[k] = G.chi_c0[pa - 1];
          S.jchi_c1[k] = G.chi_c1[pa - 1] / 2048.0;
        }
      }
      S.lc_ok = 0;
      S.lc_eps = 0.0;
      if (!top && !qs.empty()) {
        const double r1 = G.r[l + 1];
        const int rho = G.r[l + 1] / G.r[l];
        const double qlo = qs.front().first, qhi = qs.back().first;
        // single-precision d carries at most half an ulp of |d| <= qhi + ns r1
        const double eps = 4.0 * std::ldexp(qhi + G.ns * r1, -24) / r1 + 1e-9;
        if ((rho == 2 || rho == 4) && qlo > (G.ns - 1) * r1 + 2.0 && eps < 0.4 && qhi + G.ns * r1 < 16777216.0) {
          S.lc_ok = 1;
          S.lc_eps = eps;
        }
      }
    }
  }
  return true;
}

// Nodes per wavefront tile for each level: the fewest nodes (most line slices
// per node, least union overhead) that still give every slice several lines
// per window side, from the mean line density.
static void choose_tiles(Geometry& G, double lines_per_cm) {
  const double rho = lines_per_cm / 2048.0;  // lines per fine unit
  G.lnw[0] = 6;
  for (int l = 1; l < kLevels; ++l) {
    const double width = (G.b[l - 1] > 0 ? (l < kLevels - 1 ? G.b[l] - G.b[l - 1] : G.c_fine - G.b[l - 1]) : 0.0);
    int lnw = 0;
    for (; lnw < 6; ++lnw) {
      const double nw = (double)(1 << lnw);
      const double iters = (width + (nw - 1) * G.r[l]) * rho * nw / 64.0;
      if (iters >= 4.0) break;
    }
    G.lnw[l] = lnw;
  }
}

// candidate work-item sizes of the autotuner (ascending)
static const int kTuneItems[3] = {128, 256, 512};
static const int kSurrItemNodes = 128;   // work-item size of the learned-shape kernel
static const int kSurrItemMult = 8;      // at most this many times larger on the finest levels

// Work items: nodes per item scale inversely with the per-node cost, which
// grows with the level step (window width in lines); heaviest levels first.
static void make_tiles(const Geometry& G, std::vector<Tile>& tiles, int base_nodes, int max_mult = 16) {
  tiles.clear();
  for (int l = kLevels - 1; l >= 0; --l) {
    int64_t per = (int64_t)base_nodes * std::max<int64_t>(1, std::min(max_mult, 16 / G.r[l]));
    per = ((per + kWave - 1) / kWave) * kWave;
    for (int64_t f = 0; f < G.n[l]; f += per) {
      Tile t;
      t.level = l;
      t.first = f;
      t.count = (int32_t)std::min<int64_t>(per, G.n[l] - f);
      tiles.push_back(t);
    }
  }
}

static bool finite_all_f(const float* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static marfa_status validate(const marfa_lines* L, const marfa_layer* lay, int32_t nL, const marfa_request* rq) {
  if (!L || !lay || !rq) return fail(MARFA_E_INVALID, "null argument");
  if (L->n < 0) return fail(MARFA_E_INVALID, "negative line count");
  if (nL < 1) return fail(MARFA_E_INVALID, "n_layers must be >= 1");
  if (L->n > 0 && (!L->nu0 || !L->S296 || !L->gamma_air || !L->gamma_self || !L->E_lower || !L->n_air ||
                   !L->delta_air))
    return fail(MARFA_E_INVALID, "null line array");
  // a layer's line records (64 bytes in double precision) stay under 4 GiB:
  // kernels address them with 32-bit byte offsets
  if (L->n > ((int64_t)1 << 26) - 1) return fail(MARFA_E_INVALID, "too many lines (at most 2^26 - 1)");
  if (!(L->molar_mass_g > 0.0) || !std::isfinite(L->molar_mass_g)) return fail(MARFA_E_INVALID, "molar mass");
  for (int64_t j = 0; j < L->n; ++j)
    if (!std::isfinite(L->nu0[j]) || L->nu0[j] < 0.0) return fail(MARFA_E_INVALID, "line %lld: bad nu0", (long long)j);
  if (!finite_all_f(L->S296, L->n) || !finite_all_f(L->gamma_air, L->n) || !finite_all_f(L->gamma_self, L->n) ||
      !finite_all_f(L->E_lower, L->n) || !finite_all_f(L->n_air, L->n) || !finite_all_f(L->delta_air, L->n))
    return fail(MARFA_E_INVALID, "non-finite line parameter");
  for (int64_t j = 0; j < L->n; ++j)
    if (L->S296[j] < 0.0f || L->gamma_air[j] < 0.0f || L->gamma_self[j] < 0.0f)
      return fail(MARFA_E_INVALID, "line %lld: negative intensity or width", (long long)j);
  for (int32_t i = 0; i < nL; ++i) {
    const marfa_layer& y = lay[i];
    if (!std::isfinite(y.p_atm) || !std::isfinite(y.T_K) || !std::isfinite(y.p_self_atm) || !std::isfinite(y.q_ratio))
      return fail(MARFA_E_INVALID, "layer %d: non-finite", i);
    if (!(y.T_K > 0.0) || y.p_atm < 0.0 || y.p_self_atm < 0.0 || y.p_self_atm > y.p_atm)
      return fail(MARFA_E_INVALID, "layer %d: need T > 0 and 0 <= p_self <= p", i);
  }
  if (!std::isfinite(rq->nu_begin) || !std::isfinite(rq->nu_end) || rq->nu_begin < 0.0 || rq->nu_end <= rq->nu_begin)
    return fail(MARFA_E_INVALID, "need 0 <= nu_begin < nu_end");
  if (std::floor(rq->nu_begin * 2048.0) != rq->nu_begin * 2048.0 ||
      std::floor(rq->nu_end * 2048.0) != rq->nu_end * 2048.0)
    return fail(MARFA_E_INVALID, "nu_begin and nu_end must be multiples of 2^-11 cm^-1");
  if (rq->nu_end * 2048.0 > 1.0e9) return fail(MARFA_E_INVALID, "nu_end too large");
  if (!(rq->cutoff > 0.0) || !std::isfinite(rq->cutoff) || rq->cutoff > 1.0e5)
    return fail(MARFA_E_INVALID, "cutoff must be in (0, 1e5]");
  if (!(rq->R >= 4.0) || rq->R > 4096.0 || std::floor(rq->R) != rq->R)
    return fail(MARFA_E_INVALID, "R must be an integer in [4, 4096]");
  if (rq->shape < 0 || rq->shape > 3) return fail(MARFA_E_INVALID, "shape");
  if (rq->chi < 0 || rq->chi > 2) return fail(MARFA_E_INVALID, "chi");
  if (rq->out_kind < 0 || rq->out_kind > 1) return fail(MARFA_E_INVALID, "out_kind");
  if (rq->eval < 0 || rq->eval > 1) return fail(MARFA_E_INVALID, "eval");
  if (rq->level_table < 0 || rq->level_table > 1) return fail(MARFA_E_INVALID, "level_table");
  if (rq->stencil != 0 && rq->stencil != 3 && rq->stencil != 4 && rq->stencil != 5)
    return fail(MARFA_E_INVALID, "stencil must be 3, 4 or 5");
  if (rq->fp64 < 0 || rq->fp64 > 1) return fail(MARFA_E_INVALID, "fp64");
  if (!(rq->prune_rel >= 0.0) || !(rq->prune_rel < 1.0)) return fail(MARFA_E_INVALID, "prune_rel in [0,1)");
  return MARFA_OK;
}

template <typename T>
static marfa_status dmalloc(T** p, size_t count) {
  size_t bytes = std::max<size_t>(1, count * sizeof(T));
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) return fail(MARFA_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  return MARFA_OK;
}

static void free_plan(marfa_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < 3; ++i) {
    if (p->sexec[i]) (void)hipGraphExecDestroy(p->sexec[i]);
    if (p->sgraph[i]) (void)hipGraphDestroy(p->sgraph[i]);
  }
  void* bufs[] = {p->d.nu0, p->d.S296, p->d.gair, p->d.gself, p->d.El, p->d.nair, p->d.dair, p->d.layers, p->d.lconst,
                  p->d.smax, p->d.bcount, p->d.scount, p->d.kept, p->d.gcount, p->d.bucket, p->d.rec, p->d.cnu, p->d.csp,
                  p->d.A, p->d.ivs, p->d.tiles, p->d.stiles, p->d.counter, p->d.scale, p->d.span, p->d.perm,
                  p->d.stats};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete p;
}

extern "C" marfa_status marfa_plan_create(marfa_plan** out, const marfa_lines* lines, const marfa_layer* layers,
                                          int32_t n_layers, const marfa_request* req, int32_t device) {
  if (!out) return fail(MARFA_E_INVALID, "null out");
  *out = nullptr;
  marfa_status st = validate(lines, layers, n_layers, req);
  if (st != MARFA_OK) return st;
  st = ensure_device(device);
  if (st != MARFA_OK) return st;
  marfa_plan* p = new marfa_plan();
  p->device = device;
  p->req = *req;
  p->n_lines = lines->n;
  p->molar_mass = lines->molar_mass_g;
  p->n_layers = n_layers;
  p->nblk = (int)((lines->n + 255) / 256);
  double nu_max = 0.0, nu_min = 0.0;
  {
    double dlo = 0.0, dhi = 0.0, pmax = 0.0;
    for (int64_t j = 0; j < lines->n; ++j) {
      nu_max = std::max(nu_max, lines->nu0[j]);
      dlo = std::min<double>(dlo, lines->delta_air[j]);
      dhi = std::max<double>(dhi, lines->delta_air[j]);
    }
    for (int i = 0; i < n_layers; ++i) pmax = std::max(pmax, layers[i].p_atm);
    nu_min = std::min(0.0, dlo * pmax) - 1.0;   // lowest shifted centre, minus a margin
    nu_max = nu_max + std::max(0.0, dhi * pmax);
  }
  make_geometry(*req, nu_max - nu_min, p->G);
  {
    const char* base = reinterpret_cast<const char*>(device_tables(device));
    p->G.weid = reinterpret_cast<const double*>(base + offsetof(DeviceTables, weid));
    p->G.ktab = reinterpret_cast<const float4*>(base + offsetof(DeviceTables, taylor));
  }
  p->G.bucket_origin = std::floor(nu_min);
  {
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t j = 0; j < lines->n; ++j) { lo = std::min(lo, lines->nu0[j]); hi = std::max(hi, lines->nu0[j]); }
    const double span = lines->n > 0 ? std::max(1.0, hi - lo) : 1.0;
    choose_tiles(p->G, (double)lines->n / span);
  }
  if (!make_intervals(p->G, req->chi, p->ivs)) {
    free_plan(p);
    return fail(MARFA_E_INVALID, "too many band intervals");
  }
  make_tiles(p->G, p->tiles, p->base_nodes);
  {
    std::vector<Tile> most;
    make_tiles(p->G, most, kTuneItems[0]);
    p->tiles_cap = (int64_t)std::max(most.size(), p->tiles.size());
  }
  // sort lines by nu0
  const int64_t n = lines->n;
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return lines->nu0[a] < lines->nu0[b]; });
  std::vector<double> nu(n);
  std::vector<float> S(n), ga(n), gs(n), E(n), na(n), da(n);
  double dmin = 0.0, dmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = idx[i];
    nu[i] = lines->nu0[j];
    S[i] = lines->S296[j];
    ga[i] = lines->gamma_air[j];
    gs[i] = lines->gamma_self[j];
    E[i] = lines->E_lower[j];
    na[i] = lines->n_air[j];
    da[i] = lines->delta_air[j];
    if (i == 0) dmin = dmax = da[i];
    dmin = std::min<double>(dmin, da[i]);
    dmax = std::max<double>(dmax, da[i]);
  }
  p->layers_h.resize(4 * n_layers);
  p->span_h.resize(n_layers);
  for (int i = 0; i < n_layers; ++i) {
    p->layers_h[4 * i + 0] = layers[i].p_atm;
    p->layers_h[4 * i + 1] = layers[i].T_K;
    p->layers_h[4 * i + 2] = layers[i].p_self_atm;
    p->layers_h[4 * i + 3] = layers[i].q_ratio;
    p->span_h[i] = (dmax - dmin) * layers[i].p_atm * (1.0 + 1e-12) + 1e-12;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    free_plan(p);
    return fail(MARFA_E_DEVICE, "device properties");
  }
  p->cu_count = prop.multiProcessorCount;
  const size_t recsz = req->fp64 ? sizeof(LineRec64) : sizeof(LineRec32);
  const size_t realsz = req->fp64 ? sizeof(double) : sizeof(float);
  const size_t NL = (size_t)n_layers;
#define ALLOC(ptr, cnt)                      \
  do {                                       \
    st = dmalloc(&(ptr), (cnt));             \
    if (st != MARFA_OK) { free_plan(p); return st; } \
  } while (0)
  ALLOC(p->d.nu0, n);
  ALLOC(p->d.S296, n);
  ALLOC(p->d.gair, n);
  ALLOC(p->d.gself, n);
  ALLOC(p->d.El, n);
  ALLOC(p->d.nair, n);
  ALLOC(p->d.dair, n);
  ALLOC(p->d.layers, 4 * NL);
  ALLOC(p->d.lconst, 8 * NL);
  ALLOC(p->d.smax, NL);
  ALLOC(p->d.bcount, NL * (size_t)std::max(1, p->nblk));
  ALLOC(p->d.scount, NL * (size_t)std::max(1, p->nblk) * (kGroups + 1));
  ALLOC(p->d.kept, NL);
  ALLOC(p->d.gcount, NL * (kGroups + 1));
  ALLOC(p->d.bucket, NL * ((size_t)p->G.nbucket + 1));
  {
    char* r = nullptr;
    ALLOC(r, NL * (size_t)n * recsz);
    p->d.rec = r;
    char* a = nullptr;
    ALLOC(a, NL * (size_t)p->G.a_total * realsz);
    p->d.A = a;
  }
  ALLOC(p->d.cnu, NL * (size_t)n);
  {
    char* c = nullptr;
    ALLOC(c, NL * (size_t)n * realsz);
    p->d.csp = c;
  }
  ALLOC(p->d.ivs, p->ivs.size());
  ALLOC(p->d.tiles, (size_t)p->tiles_cap);
  ALLOC(p->d.counter, 4);
  ALLOC(p->d.scale, NL);
  ALLOC(p->d.span, NL);
  ALLOC(p->d.perm, NL * (size_t)n);
  ALLOC(p->d.stats, 40);
#undef ALLOC
  auto up = [&](void* dst, const void* src, size_t bytes) -> marfa_status {
    if (bytes == 0) return MARFA_OK;
    hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(MARFA_E_DEVICE, "upload: %s", hipGetErrorString(e));
    return MARFA_OK;
  };
  marfa_status u = MARFA_OK;
  if (u == MARFA_OK) u = up(p->d.nu0, nu.data(), n * sizeof(double));
  if (u == MARFA_OK) u = up(p->d.S296, S.data(), n * sizeof(float));
  if (u == MARFA_OK) u = up(p->d.gair, ga.data(), n * sizeof(float));
  if (u == MARFA_OK) u = up(p->d.gself, gs.data(), n * sizeof(float));
  if (u == MARFA_OK) u = up(p->d.El, E.data(), n * sizeof(float));
  if (u == MARFA_OK) u = up(p->d.nair, na.data(), n * sizeof(float));
  if (u == MARFA_OK) u = up(p->d.dair, da.data(), n * sizeof(float));
  if (u == MARFA_OK) u = up(p->d.layers, p->layers_h.data(), p->layers_h.size() * sizeof(double));
  if (u == MARFA_OK) u = up(p->d.span, p->span_h.data(), p->span_h.size() * sizeof(double));
  if (u == MARFA_OK) u = up(p->d.ivs, p->ivs.data(), p->ivs.size() * sizeof(IntervalSet));
  if (u == MARFA_OK) u = up(p->d.tiles, p->tiles.data(), p->tiles.size() * sizeof(Tile));
  if (u != MARFA_OK) {
    free_plan(p);
    return u;
  }
  {
    LineIn in{p->d.nu0, p->d.S296, p->d.gair, p->d.gself, p->d.El, p->d.nair, p->d.dair, p->molar_mass, n};
    launch_rank(in, p->d.layers, n_layers, p->d.span, p->d.perm, nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      free_plan(p);
      return fail(MARFA_E_DEVICE, "line ordering: %s", hipGetErrorString(e));
    }
  }
  p->grid = p->cu_count * p->blocks_per_cu;
  if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
    free_plan(p);
    return fail(MARFA_E_DEVICE, "stream create");
  }
  for (hipEvent_t& e : p->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      free_plan(p);
      return fail(MARFA_E_DEVICE, "event create");
    }
  *out = p;
  return MARFA_OK;
}

extern "C" marfa_status marfa_plan_points(const marfa_plan* p, int64_t* pts) {
  if (!p || !pts) return fail(MARFA_E_INVALID, "null argument");
  *pts = p->G.n[0];
  return MARFA_OK;
}

// enqueue the hot path for layers [first, first+count)
// stage mask: 1 = line preparation, 2 = level accumulation, 4 = cascade
// A tile list on the device (the plan's own unless overridden by the tuner).
struct TileSet {
  const Tile* dev;
  int64_t n;
  int max_item;
};

static TileSet plan_tiles(const marfa_plan* p, bool surr) {
  const std::vector<Tile>& v = surr ? p->stiles : p->tiles;
  TileSet t{surr ? p->d.stiles : p->d.tiles, (int64_t)v.size(), 0};
  for (const Tile& x : v) t.max_item = std::max(t.max_item, x.count);
  return t;
}

static void enqueue(marfa_plan* p, int first, int count, void* out, int64_t stride, hipStream_t s, bool count_mode,
                    int stages = 7, const TileSet* ts = nullptr, int grid_cap = 0) {
  const bool f64 = p->req.fp64 != 0;
  const size_t recsz = f64 ? sizeof(LineRec64) : sizeof(LineRec32);
  const size_t realsz = f64 ? sizeof(double) : sizeof(float);
  const int64_t n = p->n_lines;
  const size_t F = (size_t)first;
  LineIn in{p->d.nu0, p->d.S296, p->d.gair, p->d.gself, p->d.El, p->d.nair, p->d.dair, p->molar_mass, n};
  const int G12 = kGroups + 1;
  const size_t nb = (size_t)std::max(1, p->nblk);
  PrepArgs pa;
  pa.perm = p->d.perm + F * (size_t)n;
  pa.smax = p->d.smax + F;
  pa.bcount = p->d.bcount + F * nb;
  pa.scount = p->d.scount + F * nb * G12;
  pa.kept = p->d.kept + F;
  pa.gcount = p->d.gcount + F * G12;
  pa.bucket = p->d.bucket + F * ((size_t)p->G.nbucket + 1);
  pa.rec = (char*)p->d.rec + F * (size_t)n * recsz;
  pa.cnu = p->d.cnu + F * (size_t)n;
  pa.csp = (char*)p->d.csp + F * (size_t)n * realsz;
  pa.scale = p->d.scale + F;
  pa.lc = p->d.lconst + 8 * F;
  pa.prune = p->req.prune_rel;
  pa.R = p->req.R;
  pa.out_kind = p->req.out_kind;
  pa.fp64 = f64 ? 1 : 0;
  char* A = (char*)p->d.A + F * (size_t)p->G.a_total * realsz;
  if (stages & 1) launch_prep(in, p->d.layers + 4 * F, count, p->G, pa, s);
  const bool surr = p->surr && p->req.eval == MARFA_EVAL_SURROGATE && !count_mode;
  const TileSet tl = ts ? *ts : plan_tiles(p, surr);
  LevelArgs a;
  a.tiles = tl.dev;
  a.n_tiles = tl.n;
  a.n_layers = count;
  a.counter = p->d.counter;
  a.rec = pa.rec;
  a.csp = pa.csp;
  a.bucket = pa.bucket;
  a.gcount = pa.gcount;
  a.ivs = p->d.ivs;
  a.n_lines = n;
  a.A = A;
  a.out = out;
  a.stride = stride;
  a.stats = p->d.stats;
  a.max_item = tl.max_item;
  a.surr = surr ? 1 : 0;
  a.mlp_xmax = p->mlp_xmax;
  a.mlp_inv_c = p->mlp_inv_c;
  a.mlp = p->mlp;
  int64_t items = a.n_tiles * count;
  int grid = (int)std::min<int64_t>(std::max<int64_t>(1, items), (int64_t)(grid_cap > 0 ? grid_cap : p->grid));
  if (stages & 2) {
    launch_fill_u32(p->d.counter, 1, 0u, s);
    launch_level(p->G, a, grid, f64, count_mode, s);
  }
  if ((stages & 4) && !count_mode) launch_cascade(p->G, count, A, out, stride, p->d.scale + F, f64, s);
}

static marfa_status capture(marfa_plan* p, void* out, int64_t stride, int stages, hipGraph_t* g, hipGraphExec_t* x) {
  // a launch of the graph being replaced may still be queued
  if (*x) HIP_TRY(hipDeviceSynchronize());
  if (*x) { (void)hipGraphExecDestroy(*x); *x = nullptr; }
  if (*g) { (void)hipGraphDestroy(*g); *g = nullptr; }
  HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
  enqueue(p, 0, p->n_layers, out, stride, p->cap, false, stages);
  hipError_t e = hipStreamEndCapture(p->cap, g);
  if (e != hipSuccess) return fail(MARFA_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
  HIP_TRY(hipGraphInstantiate(x, *g, nullptr, nullptr, 0));
  return MARFA_OK;
}

static marfa_status check_out(marfa_plan* p, void* out, int64_t stride) {
  if (!out) return fail(MARFA_E_INVALID, "null output");
  if (stride < p->G.n[0]) return fail(MARFA_E_INVALID, "layer_stride %lld < points %lld", (long long)stride,
                                      (long long)p->G.n[0]);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, out) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MARFA_E_INVALID, "output is not a HIP allocation");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(MARFA_E_INVALID, "output must be device memory");
  if (attr.device != p->device) return fail(MARFA_E_INVALID, "output lives on device %d, plan on %d", attr.device,
                                            p->device);
  return MARFA_OK;
}

static marfa_status check_eval(const marfa_plan* p) {
  if (p->req.eval == MARFA_EVAL_SURROGATE && !p->surr)
    return fail(MARFA_E_UNSUPPORTED, "surrogate evaluation requested but no trained surrogate is set");
  return MARFA_OK;
}

extern "C" marfa_status marfa_execute(marfa_plan* p, void* out, int64_t stride, void* stream) {
  if (!p) return fail(MARFA_E_INVALID, "null plan");
  if (check_eval(p) != MARFA_OK) return MARFA_E_UNSUPPORTED;
  marfa_status st = check_out(p, out, stride);
  if (st != MARFA_OK) return st;
  HIP_TRY(hipSetDevice(p->device));
  if (!p->exec || p->g_out != out || p->g_stride != stride) {
    st = capture(p, out, stride, 7, &p->graph, &p->exec);
    if (st != MARFA_OK) return st;
    p->g_out = out;
    p->g_stride = stride;
  }
  HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream));
  return MARFA_OK;
}

extern "C" marfa_status marfa_execute_timed(marfa_plan* p, void* out, int64_t stride, void* stream, marfa_timing* t) {
  if (!p || !t) return fail(MARFA_E_INVALID, "null argument");
  if (check_eval(p) != MARFA_OK) return MARFA_E_UNSUPPORTED;
  marfa_status st = check_out(p, out, stride);
  if (st != MARFA_OK) return st;
  HIP_TRY(hipSetDevice(p->device));
  if (!p->sexec[0] || p->s_out != out || p->s_stride != stride) {
    for (int i = 0; i < 3; ++i) {
      st = capture(p, out, stride, 1 << i, &p->sgraph[i], &p->sexec[i]);
      if (st != MARFA_OK) return st;
    }
    p->s_out = out;
    p->s_stride = stride;
  }
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipEventRecord(p->ev[0], s));
  for (int i = 0; i < 3; ++i) {
    HIP_TRY(hipGraphLaunch(p->sexec[i], s));
    HIP_TRY(hipEventRecord(p->ev[i + 1], s));
  }
  HIP_TRY(hipEventSynchronize(p->ev[3]));
  HIP_TRY(hipEventElapsedTime(&t->prep_ms, p->ev[0], p->ev[1]));
  HIP_TRY(hipEventElapsedTime(&t->level_ms, p->ev[1], p->ev[2]));
  HIP_TRY(hipEventElapsedTime(&t->cascade_ms, p->ev[2], p->ev[3]));
  HIP_TRY(hipEventElapsedTime(&t->total_ms, p->ev[0], p->ev[3]));
  return MARFA_OK;
}

extern "C" marfa_status marfa_execute_layers(marfa_plan* p, int32_t first, int32_t count, void* out, int64_t stride,
                                             void* stream) {
  if (!p) return fail(MARFA_E_INVALID, "null plan");
  if (first < 0 || count < 1 || first + count > p->n_layers) return fail(MARFA_E_INVALID, "layer range");
  if (check_eval(p) != MARFA_OK) return MARFA_E_UNSUPPORTED;
  marfa_status st = check_out(p, out, stride);
  if (st != MARFA_OK) return st;
  HIP_TRY(hipSetDevice(p->device));
  enqueue(p, first, count, out, stride, (hipStream_t)stream, false);
  HIP_TRY(hipGetLastError());
  return MARFA_OK;
}

extern "C" marfa_status marfa_plan_count(marfa_plan* p, marfa_stats* out) {
  if (!p || !out) return fail(MARFA_E_INVALID, "null argument");
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = p->cap;
  launch_fill_u64(p->d.stats, 40, 0ull, s);
  enqueue(p, 0, p->n_layers, nullptr, 0, s, true);
  HIP_TRY(hipGetLastError());
  unsigned long long h[40];
  int32_t gc[12];
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(h, p->d.stats, sizeof h, hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof *out);
  out->points_per_layer = p->G.n[0];
  out->n_layers = p->n_layers;
  out->lines_total = p->n_lines;
  int64_t kept = 0;
  for (int L = 0; L < p->n_layers; ++L) {
    HIP_TRY(hipMemcpy(gc, p->d.gcount + (size_t)L * 12, sizeof gc, hipMemcpyDeviceToHost));
    for (int g = 0; g < kGroups; ++g) kept += gc[g];
  }
  (void)gc;
  out->lines_kept = kept;
  for (int l = 0; l < kLevels; ++l) out->pairs_level[l] = (int64_t)h[l];
  out->pairs_band = (int64_t)h[11];
  out->pairs_core = (int64_t)h[12];
  out->pairs_wing = (int64_t)h[13];
  out->wing_terms = (int64_t)h[14];
  for (int l = 0; l < kLevels; ++l) {
    out->iters_level[l] = (int64_t)h[16 + l];
    out->band_iters_level[l] = (int64_t)h[27 + l];
  }
  int64_t ln = 0;
  for (int l = 1; l < kLevels; ++l) ln += p->G.n[l];
  out->level_nodes = ln * p->n_layers;
  const bool five = p->G.ns == 5;
  out->flops_per_eval = kFlopsEval;
  out->flops_per_core = kFlopsCore;
  out->flops_per_term = kFlopsTerm;
  const bool four = p->G.ns == 4;
  out->flops_per_band = five ? kFlopsBand5 : (four ? kFlopsBand4 : kFlopsBand3);
  out->flops_per_cascade = five ? kFlopsCascade5 : (four ? kFlopsCascade4 : kFlopsCascade3);
  out->flops_level = out->flops_per_eval * (double)(out->pairs_wing + out->pairs_core) +
                     out->flops_per_core * (double)out->pairs_core + out->flops_per_term * (double)out->wing_terms +
                     out->flops_per_band * (double)out->pairs_band;
  // cascade: every node of levels 0..9 not coinciding with a coarser node is
  // interpolated (injection at coinciding nodes is a copy)
  double interp_nodes = 0.0;
  for (int l = 0; l < kLevels - 1; ++l) {
    const double rho = (double)(p->G.r[l + 1] / p->G.r[l]);
    interp_nodes += (double)p->G.n[l] * (rho - 1.0) / rho;
  }
  out->flops_cascade = out->flops_per_cascade * interp_nodes * p->n_layers;
  const double real_b = p->req.fp64 ? 8.0 : 4.0;
  const double rec_b = p->req.fp64 ? (double)sizeof(LineRec64) : (double)sizeof(LineRec32);
  out->bytes_level = rec_b * (double)kept + real_b * (double)(out->level_nodes + out->points_per_layer * p->n_layers);
  out->bytes_cascade = real_b * (double)(out->level_nodes + out->points_per_layer * p->n_layers) * (double)(p->G.ns + 2);
  return MARFA_OK;
}

// Destroy the plan's captured graphs.  A launch of them may still be queued
// on a caller's stream, so the device finishes its work first.
static void drop_graphs(marfa_plan* p) {
  if (p->exec || p->sexec[0] || p->sexec[1] || p->sexec[2]) {
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
  }
  if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
  if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
  for (int i = 0; i < 3; ++i) {
    if (p->sexec[i]) { (void)hipGraphExecDestroy(p->sexec[i]); p->sexec[i] = nullptr; }
    if (p->sgraph[i]) { (void)hipGraphDestroy(p->sgraph[i]); p->sgraph[i] = nullptr; }
  }
  p->g_out = p->s_out = nullptr;
}

extern "C" marfa_status marfa_plan_tiles(const marfa_plan* p, marfa_tiles* t) {
  if (!p || !t) return fail(MARFA_E_INVALID, "null argument");
  std::memset(t, 0, sizeof *t);
  t->item_nodes = p->base_nodes;
  t->blocks_per_cu = p->blocks_per_cu;
  t->tuned = p->tuned;
  for (int l = 0; l < kLevels; ++l) t->wave_nodes[l] = 1 << p->G.lnw[l];
  t->tune_ms = p->tune_ms;
  return MARFA_OK;
}


extern "C" marfa_status marfa_plan_set_tiles(marfa_plan* p, const marfa_tiles* t) {
  if (!p || !t) return fail(MARFA_E_INVALID, "null argument");
  if (t->item_nodes < 64 || t->item_nodes > 8192 || t->item_nodes % 64 != 0)
    return fail(MARFA_E_INVALID, "item_nodes must be a multiple of 64 in [64, 8192]");
  if (t->blocks_per_cu < 1 || t->blocks_per_cu > 32) return fail(MARFA_E_INVALID, "blocks_per_cu in [1, 32]");
  int lnw[kLevels];
  for (int l = 0; l < kLevels; ++l) {
    const int w = t->wave_nodes[l];
    if (w < 1 || w > 64 || (w & (w - 1)) != 0) return fail(MARFA_E_INVALID, "wave_nodes must be powers of 2 <= 64");
    lnw[l] = __builtin_ctz((unsigned)w);
  }
  std::vector<Tile> tl;
  make_tiles(p->G, tl, t->item_nodes);
  HIP_TRY(hipSetDevice(p->device));
  if ((int64_t)tl.size() > p->tiles_cap) {
    Tile* nt = nullptr;
    marfa_status st = dmalloc(&nt, tl.size());
    if (st != MARFA_OK) return st;
    HIP_TRY(hipDeviceSynchronize());
    (void)hipFree(p->d.tiles);
    p->d.tiles = nt;
    p->tiles_cap = (int64_t)tl.size();
  }
  HIP_TRY(hipMemcpy(p->d.tiles, tl.data(), tl.size() * sizeof(Tile), hipMemcpyHostToDevice));
  drop_graphs(p);
  for (int l = 0; l < kLevels; ++l) p->G.lnw[l] = lnw[l];
  p->tiles = tl;
  p->base_nodes = t->item_nodes;
  p->blocks_per_cu = t->blocks_per_cu;
  p->grid = p->cu_count * t->blocks_per_cu;
  return MARFA_OK;
}

// Level stage alone over every layer with the given tiles and grid; the
// faster of two runs, in ms (events on the caller's stream).
static marfa_status time_level(marfa_plan* p, const std::vector<Tile>& tiles, int grid, void* out, int64_t stride,
                               hipStream_t s, float* ms) {
  if ((int64_t)tiles.size() > p->tiles_cap) return fail(MARFA_E_STATE, "tile list exceeds its buffer");
  HIP_TRY(hipMemcpyAsync(p->d.tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
  TileSet ts{p->d.tiles, (int64_t)tiles.size(), 0};
  for (const Tile& x : tiles) ts.max_item = std::max(ts.max_item, x.count);
  float best = INFINITY;
  for (int rep = 0; rep < 2; ++rep) {
    HIP_TRY(hipEventRecord(p->ev[0], s));
    enqueue(p, 0, p->n_layers, out, stride, s, false, 2, &ts, grid);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(p->ev[1], s));
    HIP_TRY(hipEventSynchronize(p->ev[1]));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, p->ev[0], p->ev[1]));
    best = std::min(best, t);
  }
  *ms = best;
  return MARFA_OK;
}

extern "C" marfa_status marfa_plan_tune(marfa_plan* p, void* out, int64_t stride, void* stream) {
  if (!p) return fail(MARFA_E_INVALID, "null plan");
  marfa_status st = check_out(p, out, stride);
  if (st != MARFA_OK) return st;
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  drop_graphs(p);
  // the tiles are the plain kernel's: tune it even while the learned shape is selected
  const int32_t eval = p->req.eval;
  p->req.eval = MARFA_EVAL_PLAIN;
  struct Restore {
    marfa_plan* p;
    int32_t e;
    ~Restore() { p->req.eval = e; }
  } restore{p, eval};
  enqueue(p, 0, p->n_layers, out, stride, s, false, 1);   // line preparation
  HIP_TRY(hipGetLastError());
  // 1. region tile per level, items of the current size
  for (int l = 0; l < kLevels; ++l) {
    std::vector<Tile> all, lv;
    make_tiles(p->G, all, p->base_nodes);
    for (const Tile& t : all)
      if (t.level == l) lv.push_back(t);
    if (lv.empty()) continue;
    // every tile width (the time is not unimodal in the width: the lanes
    // take 1, 2 or 4 nodes each depending on it)
    const int cur = p->G.lnw[l];
    int best_lnw = cur;
    float best = INFINITY;
    for (int c = 0; c <= 6; ++c) {
      p->G.lnw[l] = c;
      float ms = 0.f;
      st = time_level(p, lv, p->grid, out, stride, s, &ms);
      if (st != MARFA_OK) { p->G.lnw[l] = cur; return st; }
      if (ms < best) { best = ms; best_lnw = c; }
    }
    p->G.lnw[l] = best_lnw;
  }
  // 2. work-item size, then the persistent grid
  int best_base = p->base_nodes, best_bpc = p->blocks_per_cu;
  float best = INFINITY;
  for (int base : kTuneItems) {
    std::vector<Tile> tl;
    make_tiles(p->G, tl, base);
    float ms = 0.f;
    st = time_level(p, tl, p->cu_count * best_bpc, out, stride, s, &ms);
    if (st != MARFA_OK) return st;
    if (ms < best) { best = ms; best_base = base; }
  }
  std::vector<Tile> tl;
  make_tiles(p->G, tl, best_base);
  for (int bpc : {4, 8, 16}) {
    if (bpc == best_bpc) continue;
    float ms = 0.f;
    st = time_level(p, tl, p->cu_count * bpc, out, stride, s, &ms);
    if (st != MARFA_OK) return st;
    if (ms < best) { best = ms; best_bpc = bpc; }
  }
  // 3. one pass over the levels with the whole stage timed: a level's tile
  // chosen alone can interact with the others' (the persistent grid's tail
  // and the mix of levels on a CU), so each width's neighbours are retried
  for (int l = 0; l < kLevels; ++l) {
    const int cur = p->G.lnw[l];
    for (int c : {cur - 1, cur + 1}) {
      if (c < 0 || c > 6) continue;
      p->G.lnw[l] = c;
      float ms = 0.f;
      st = time_level(p, tl, p->cu_count * best_bpc, out, stride, s, &ms);
      if (st != MARFA_OK) { p->G.lnw[l] = cur; return st; }
      if (ms < 0.995f * best) {
        best = ms;
        break;   // keep c
      }
      p->G.lnw[l] = cur;
    }
  }
  p->base_nodes = best_base;
  p->blocks_per_cu = best_bpc;
  p->grid = p->cu_count * best_bpc;
  p->tiles = tl;
  HIP_TRY(hipMemcpyAsync(p->d.tiles, p->tiles.data(), p->tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  p->tuned = 1;
  p->tune_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return MARFA_OK;
}

extern "C" marfa_status marfa_plan_set_surrogate(marfa_plan* p, const marfa_surrogate* s) {
  if (!p) return fail(MARFA_E_INVALID, "null plan");
  if (!s) {
    p->surr = nullptr;
    drop_graphs(p);
    return MARFA_OK;
  }
  MlpDev W;
  double x_max = 0.0, cutoff = 0.0;
  int32_t chi = 0;
  int dev = -1;
  if (!marfa_surrogate_view(s, &W, &x_max, &chi, &cutoff, &dev))
    return fail(MARFA_E_UNSUPPORTED, "the surrogate is not trained");
  if (dev != p->device) return fail(MARFA_E_INVALID, "surrogate on device %d, plan on %d", dev, p->device);
  if (p->req.fp64 || p->req.shape != MARFA_SHAPE_VOIGT)
    return fail(MARFA_E_INVALID, "the surrogate serves single-precision Voigt plans");
  if (p->G.ns != 3) return fail(MARFA_E_UNSUPPORTED, "the learned shape runs with 3-point plans");
  if (chi != p->req.chi || cutoff != p->req.cutoff)
    return fail(MARFA_E_INVALID, "surrogate trained for chi %d, cut-off %g; plan has chi %d, cut-off %g", chi, cutoff,
                p->req.chi, p->req.cutoff);
  for (const IntervalSet& iv : p->ivs)
    if (iv.n_jump > 0 && !iv.lc_ok)
      return fail(MARFA_E_UNSUPPORTED, "cut-off too small for the line-major band pass the surrogate needs");
  // its own work items: 128 nodes (1024 on level 0) keep the accumulators at
  // 4 KB of LDS, so three workgroups fit a CU beside the staged network
  if (p->stiles.empty()) {
    std::vector<Tile> st;
    make_tiles(p->G, st, kSurrItemNodes, kSurrItemMult);
    HIP_TRY(hipSetDevice(p->device));
    marfa_status m = dmalloc(&p->d.stiles, st.size());
    if (m != MARFA_OK) return m;
    HIP_TRY(hipMemcpy(p->d.stiles, st.data(), st.size() * sizeof(Tile), hipMemcpyHostToDevice));
    p->stiles = st;
  }
  p->surr = s;
  p->mlp = W;
  p->mlp_xmax = (float)x_max;
  p->mlp_inv_c = (float)(1.0 / cutoff);
  drop_graphs(p);
  return MARFA_OK;
}

extern "C" marfa_status marfa_plan_set_eval(marfa_plan* p, int32_t eval) {
  if (!p) return fail(MARFA_E_INVALID, "null plan");
  if (eval != MARFA_EVAL_PLAIN && eval != MARFA_EVAL_SURROGATE) return fail(MARFA_E_INVALID, "eval");
  if (eval != p->req.eval) {
    drop_graphs(p);
    p->req.eval = eval;
  }
  return MARFA_OK;
}

extern "C" void marfa_plan_destroy(marfa_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  free_plan(p);
}

extern "C" const char* marfa_status_string(int32_t s) {
  switch (s) {
    case MARFA_OK: return "ok";
    case MARFA_E_INVALID: return "invalid argument";
    case MARFA_E_NOMEM: return "out of memory";
    case MARFA_E_DEVICE: return "device error";
    case MARFA_E_UNSUPPORTED: return "unsupported";
    case MARFA_E_STATE: return "bad state";
    case MARFA_E_IO: return "file error";
    default: return "unknown status";
  }
}

extern "C" marfa_status marfa_last_error(char* buf, size_t n) {
  if (!buf || n == 0) return MARFA_E_INVALID;
  std::snprintf(buf, n, "%s", g_err.c_str());
  return MARFA_OK;
}

extern "C" marfa_status marfa_voigt_eval(int32_t device, int64_t n, const double* x, const double* y, double* out,
                                         int32_t fp64) {
  if (n < 0 || (n > 0 && (!x || !y || !out))) return fail(MARFA_E_INVALID, "bad arguments");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || y[i] < 0.0) return fail(MARFA_E_INVALID, "need finite x, y >= 0");
  marfa_status st = ensure_device(device);
  if (st != MARFA_OK) return st;
  if (n == 0) return MARFA_OK;
  double *dx = nullptr, *dy = nullptr, *dout = nullptr;
  st = dmalloc(&dx, n);
  if (st == MARFA_OK) st = dmalloc(&dy, n);
  if (st == MARFA_OK) st = dmalloc(&dout, n);
  if (st == MARFA_OK) {
    hipError_t e = hipMemcpy(dx, x, n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dy, y, n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      launch_voigt_eval(n, dx, dy, dout, fp64 != 0, device_tables(device), nullptr);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = fail(MARFA_E_DEVICE, "voigt eval: %s", hipGetErrorString(e));
  }
  if (dx) (void)hipFree(dx);
  if (dy) (void)hipFree(dy);
  if (dout) (void)hipFree(dout);
  return st;
}
