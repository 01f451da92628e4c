/*
 * orc_user.h -- the oracle's user line shape and chi factor (TEST
 * INFRASTRUCTURE ONLY; included by marfa_oracle.c alone).
 *
 * Sections 2.2 and 2.3 let the user supply the line shape and the chi factor.
 * The oracle takes them as plain C functions compiled in; build with
 * ORC_USER_HEADER="/abs/path.h" to substitute others.  A header defines:
 *   double orc_user_shape(double d, double gamma_L, double alpha_D)
 *       normalised profile [cm] at d = nu - nu~0 [cm^-1];
 *   double orc_user_chi(double a)          chi at a = |d| [cm^-1];
 *   ORC_USER_CHI_NBREAK, orc_user_chi_break[]  ascending a where chi or its
 *       slope jumps (the grid method adds residual bands there).
 *
 * Shipped functions, written here from their definitions in double precision:
 *  - the pseudo-Voigt of Thompson, Cox and Hastings (J. Appl. Cryst. 20 (1987)
 *    79): eta L + (1 - eta) G with Lorentz and Gauss profiles of one full
 *    width G5 = (fG^5 + 2.69269 fG^4 fL + 2.42843 fG^3 fL^2 + 4.47163 fG^2 fL^3
 *    + 0.07842 fG fL^4 + fL^5)^(1/5), fG = 2 alpha_D, fL = 2 gamma_L, and
 *    eta = 1.36603 q - 0.47719 q^2 + 0.11116 q^3, q = fL / G5;
 *  - a sub-Lorentzian chi: 1 for a <= 2, beyond it
 *    0.95 exp(-(a - 2) / 30) / (1 + ((a - 2) / 60)^2).
 */
#ifndef ORC_USER_H
#define ORC_USER_H

#ifdef ORC_USER_HEADER
#include ORC_USER_HEADER
#else
#include <math.h>

#define ORC_USER_CHI_NBREAK 1
static const double orc_user_chi_break[ORC_USER_CHI_NBREAK] = {2.0};

static double orc_user_chi(double a) {
  if (a <= 2.0) return 1.0;
  const double u = a - 2.0;
  return 0.95 * exp(-u / 30.0) / (1.0 + (u / 60.0) * (u / 60.0));
}

static double orc_user_shape(double d, double gamma_L, double alpha_D) {
  const double fG = 2.0 * alpha_D, fL = 2.0 * gamma_L;
  const double G5 = pow(pow(fG, 5) + 2.69269 * pow(fG, 4) * fL + 2.42843 * pow(fG, 3) * pow(fL, 2) +
                            4.47163 * pow(fG, 2) * pow(fL, 3) + 0.07842 * fG * pow(fL, 4) + pow(fL, 5),
                        0.2);
  if (!(G5 > 0.0)) return 0.0;
  const double q = fL / G5;
  const double eta = 1.36603 * q - 0.47719 * q * q + 0.11116 * q * q * q;
  const double pi = 3.14159265358979323846;
  /* Lorentz of full width G5: (G5/2) / (pi (d^2 + (G5/2)^2)) */
  const double lor = (G5 / 2.0) / (pi * (d * d + G5 * G5 / 4.0));
  /* Gauss of full width G5: sqrt(4 ln 2 / pi) / G5 exp(-4 ln 2 d^2 / G5^2) */
  const double gau = sqrt(4.0 * log(2.0) / pi) / G5 * exp(-4.0 * log(2.0) * d * d / (G5 * G5));
  return eta * lor + (1.0 - eta) * gau;
}
#endif

#endif
