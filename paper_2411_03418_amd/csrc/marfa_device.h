// marfa_device.h -- device code shared by the kernels of the eleven-grid
// library: physical constants, the line shapes (Voigt core and wing, Tonkov
// chi) and the evaluation of one line at one distance.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "marfa_internal.h"
#include "marfa_user.h"

// Whether this translation unit's kernels evaluate the user line shape and
// chi.  The level kernels are built twice: without them (the kernels every
// other plan runs, free of their code) and with them (plans that select the
// user shape or chi).
#ifndef MARFA_USER_PLUGINS
#define MARFA_USER_PLUGINS 1
#endif

namespace marfa {

// physical constants (CODATA 2018) and HITRAN reference temperature
constexpr double kC2 = 1.438776877;           // hc/k_B [cm K]
constexpr double kTref = 296.0;
constexpr double kBoltzmann = 1.380649e-23;   // [J/K]
constexpr double kNA = 6.02214076e23;         // [1/mol]
constexpr double kCLight = 299792458.0;       // [m/s]
constexpr double kAtmPa = 101325.0;
constexpr double kLn2d = 0.693147180559945309417;
constexpr double kSqrtLn2 = 0.832554611157697756353;
constexpr double kInvPi = 0.318309886183790671538;
constexpr double kInvSqrtPi = 0.564189583547756286948;
constexpr double kH0 = 1.0 / 2048.0;


template <typename R> struct RecOf;
template <> struct RecOf<float> { using T = LineRec32; };
template <> struct RecOf<double> { using T = LineRec64; };

// gamma_L^2 of a record (the single-precision record keeps gamma_L only)
__device__ __forceinline__ float gam2_of(const LineRec32& L) { return L.gam * L.gam; }
__device__ __forceinline__ double gam2_of(const LineRec64& L) { return L.gam2; }

// Wing series cut and the |z|^2 above which it replaces the core.
template <typename R> struct Prec;
template <> struct Prec<float> {
  static constexpr float kEps = 1e-6f;
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
// series in Z = (L+iz)/(L-iz):  w = 1/(sqrt(pi)(L-iz)) + 2/(L-iz)^2 sum_n a_n Z^(n-1),
// in double precision (double-precision path).  P(Z) = sum_{n=1..N} a_n Z^(n-1)
// by complex Horner.
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

// K(x, y) = Re w(x + iy) for x, y >= 0, |z| < 6, in single precision: the
// Taylor series of w about the nearest lattice centre z0 = (i + j sqrt(-1))/4,
//   w(z0 + u) = sum_n c_n u^n,  c_n = w^(n)(z0)/n!,  |u| <= sqrt(2)/8,
// nine terms, complex Horner in u = (x - i/4) + (y - j/4) sqrt(-1).  The
// coefficients are tabulated in double precision and rounded once; on the real
// axis their real parts are the Hermite forms d^n/dx^n exp(-x^2)/n!.  Because
// the real and imaginary parts of each c_n are stored separately, Re w near the
// real axis (where it is far smaller than Im w) comes out with a relative, not
// an absolute, rounding error: every product that forms it is of its own size.
__device__ __forceinline__ float voigt_core32(float x, float y, const float4* __restrict__ tab) {
  const float fi = fminf(rintf(x * float(kTaylorPerUnit)), float(kTaylorSide - 1));
  const float fj = fminf(rintf(y * float(kTaylorPerUnit)), float(kTaylorSide - 1));
  const float d = fmaf(fi, -1.0f / kTaylorPerUnit, x);
  const float e = fmaf(fj, -1.0f / kTaylorPerUnit, y);
  const float4* c = tab + ((int)fj * kTaylorSide + (int)fi) * kTaylorQuads;
  const float4 q4 = c[4], q3 = c[3], q2 = c[2], q1 = c[1], q0 = c[0];
  float pr = q4.x, pi = q4.y;
  auto step = [&](float cr, float ci) {
    const float nr = fmaf(pr, d, fmaf(-pi, e, cr));
    pi = fmaf(pr, e, fmaf(pi, d, ci));
    pr = nr;
  };
  step(q3.z, q3.w);
  step(q3.x, q3.y);
  step(q2.z, q2.w);
  step(q2.x, q2.y);
  step(q1.z, q1.w);
  step(q1.x, q1.y);
  step(q0.z, q0.w);
  return fmaf(pr, d, fmaf(-pi, e, q0.x));
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
  uint32_t iters;        // wavefront iterations over line windows (lane 0 counts)
  uint32_t band_iters;   // iterations that ran the band correction
};

// shapes evaluated pair by pair through line_value (no wing series or core queue)
__host__ __device__ __forceinline__ bool generic_shape(const Geometry& G) {
  return G.shape == MARFA_SHAPE_DOPPLER || G.shape == MARFA_SHAPE_USER;
}

// g(d) = S' F(d) chi(|d|) [|d| <= c], d in fine units
template <typename R, bool COUNT>
__device__ __forceinline__ R line_value(R d, const typename RecOf<R>::T& L, R Sp, const Geometry& G, R cfine,
                                        Counts& cnt) {
  R ad = fabs(d);
  if (ad > cfine) return R(0);
  R dcm = d * R(kH0);
  R dd = dcm * dcm;
  R f;
  if (G.shape == MARFA_SHAPE_LORENTZ) {
    f = R(L.gam) * R(kInvPi) / (dd + gam2_of(L));
  } else if (G.shape == MARFA_SHAPE_DOPPLER) {
    R x = R(L.xs) * dcm;
    f = R(L.xs) * R(kInvSqrtPi) * exp(-x * x);
  } else if (MARFA_USER_PLUGINS && G.shape == MARFA_SHAPE_USER) {
    // xs = sqrt(ln 2) / alpha_D, and 0 for a line without Doppler width
    const R aD = L.xs > R(0) ? R(kSqrtLn2) / R(L.xs) : R(0);
    f = MarfaUserShape::f<R>(dcm, R(L.gam), aD);
  } else {
    R x = R(L.xs) * dcm;
    R y = R(L.xs) * R(L.gam);
    R z2 = x * x + y * y;
    if (L.xs == 0 || z2 >= Prec<R>::kZ2) {
      int terms = 0;
      f = voigt_wing<R>(dd, R(L.gam), gam2_of(L), R(L.ae), terms);
      if (COUNT) { cnt.wing++; cnt.terms += terms; }
    } else {
      if constexpr (sizeof(R) == 4) {
        f = L.xs * float(kInvSqrtPi) * voigt_core32(fabsf(x), y, G.ktab);
      } else {
        const double K = voigt_core<kWeidemanN64>(fabs(x), y, G.weid, G.weid[kWeidemanN64 + 1]);
        f = L.xs * kInvSqrtPi * K;
      }
      if (COUNT) cnt.core++;
    }
  }
  R chi = R(1);
  if (G.chi == MARFA_CHI_TONKOV) chi = tonkov<R>(ad * R(kH0));
  else if (MARFA_USER_PLUGINS && G.chi == MARFA_CHI_USER) chi = MarfaUserChi::chi<R>(ad * R(kH0));
  return Sp * f * chi;
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// Lagrange weight of offset i (in -H..H) at t for the 2H+1 nodes -H..H
template <int H>
__host__ __device__ constexpr double lagrange_den(int i) {
  double v = 1.0;
  for (int j = -H; j <= H; ++j)
    if (j != i) v *= (double)(i - j);
  return v;
}
template <int H>
__host__ __device__ __forceinline__ constexpr double lagrange_w(int i, double t) {
  double v = 1.0;
  for (int j = -H; j <= H; ++j)
    if (j != i) v *= (t - j);
  return v * (1.0 / lagrange_den<H>(i));
}
// Weight of node i (-1 .. 2) at t for the symmetric 4-point rule on the nodes
// -1, 0, 1, 2 (at t = 1/2: (-1, 9, 9, -1)/16)
__host__ __device__ __forceinline__ constexpr double lagrange_w4(int i, double t) {
  double v = 1.0, den = 1.0;
  for (int j = -1; j <= 2; ++j)
    if (j != i) {
      v *= (t - j);
      den *= (double)(i - j);
    }
  return v / den;
}

}  // namespace marfa
