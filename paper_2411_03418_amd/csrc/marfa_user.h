// User line shape and chi factor, compiled into every kernel (Sections 2.2
// and 2.3: the line shape and the chi factor are user-selectable functions).
//
// A plan whose request has shape MARFA_SHAPE_USER evaluates the normalised
// profile with MarfaUserShape::f; one with chi MARFA_CHI_USER multiplies by
// MarfaUserChi::chi.  To plug in other functions, write a header that defines
// the same two structs and build with MARFA_USER_HEADER=/abs/path/to/it.h.
//
// Contract (R is float or double; both instantiations are compiled):
//   MarfaUserShape::f<R>(d, gamma_L, alpha_D) -- the profile in cm, with unit
//     integral over d; d = nu - nu~0 in cm^-1, gamma_L and alpha_D the Lorentz
//     and Doppler half widths in cm^-1 (alpha_D = 0 for a line without Doppler
//     width).  The start level of a line still comes from max(gamma_L, alpha_D).
//   MarfaUserChi::chi<R>(a) -- the factor at a = |d| >= 0 in cm^-1.
//   MarfaUserChi::kBreaks, kBreak[] -- the a values (cm^-1, ascending, at most
//     3) where chi or its slope jumps.  The band pass corrects the
//     interpolation there exactly as at the cut-off.
//
// The functions below are the shipped example: the pseudo-Voigt of Thompson,
// Cox and Hastings (J. Appl. Cryst. 20 (1987) 79) as a line shape, and a
// sub-Lorentzian chi with a step at 2 cm^-1 and an exponential-times-
// Lorentzian decay beyond it.
#pragma once

#include <hip/hip_runtime.h>

#ifdef MARFA_USER_HEADER
#include MARFA_USER_HEADER
#else

struct MarfaUserShape {
  // eta L(d; Gamma) + (1 - eta) G(d; Gamma) on the full widths fG = 2 alpha_D,
  // fL = 2 gamma_L, with the width Gamma and mixing eta of the TCH fit
  template <typename R>
  __host__ __device__ static R f(R d, R gamma_L, R alpha_D) {
    const R m = R(2) * (alpha_D > gamma_L ? alpha_D : gamma_L);
    if (!(m > R(0))) return R(0);
    const R g = R(2) * alpha_D / m, l = R(2) * gamma_L / m;  // widths scaled by the larger
    const R g2 = g * g, l2 = l * l;
    const R p5 = g2 * g2 * g + R(2.69269) * g2 * g2 * l + R(2.42843) * g2 * g * l2 +
                 R(4.47163) * g2 * l2 * l + R(0.07842) * g * l2 * l2 + l2 * l2 * l;
    const R W = m * pow(p5, R(0.2));
    const R q = R(2) * gamma_L / W;
    const R eta = q * (R(1.36603) + q * (R(-0.47719) + q * R(0.11116)));
    const R hw = R(0.5) * W;
    const R lor = hw / (R(3.14159265358979323846) * (d * d + hw * hw));
    const R gs = R(0.83255461115769775635) / hw;  // sqrt(ln 2) / (W / 2)
    const R gau = gs * R(0.56418958354775628695) * exp(-(gs * d) * (gs * d));
    return eta * lor + (R(1) - eta) * gau;
  }
};

struct MarfaUserChi {
  static constexpr int kBreaks = 1;
  static constexpr double kBreak[kBreaks] = {2.0};
  // 1 up to 2 cm^-1, then 0.95 e^{-(a-2)/30} / (1 + ((a-2)/60)^2)
  template <typename R>
  __host__ __device__ static R chi(R a) {
    if (a <= R(2)) return R(1);
    const R t = (a - R(2)) * R(1.0 / 60.0);
    return R(0.95) * exp(R(-2) * t) / (R(1) + t * t);
  }
};

#endif

static_assert(MarfaUserChi::kBreaks >= 0 && MarfaUserChi::kBreaks <= 3, "at most 3 chi breaks");
