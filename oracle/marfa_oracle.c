/*
 * marfa_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load this code.  It shares nothing with the HIP library.
 *
 * Paper: MARFA, "An Effective Line-by-line Tool for Calculating Molecular
 * Absorption in Planetary Atmospheres" (arXiv 2411.03418).
 *   Eq.(2),(3)   absorption coefficient and cross-section, Section 2.1
 *   Eq.(4),(5)   Lorentz and Gauss profiles, Section 2.2
 *   Eq.(7),(8)   Voigt profile through K(x,y), Section 2.2
 *   Eq.(10)      Tonkov chi-factor, Section 2.3
 *   Section 2.4  eleven-grid interpolation technique, 10 cm^-1 intervals,
 *                finest step 10/20480 cm^-1, 3-point interpolation
 * Where the paper is silent, each function states the reading it takes.
 */
#include "marfa_oracle.h"
#include "orc_user.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* constants (CODATA 2018)                                             */
/* ------------------------------------------------------------------ */
static const double kPi = 3.14159265358979323846;
static const double kSqrtPi = 1.77245385090551602730;
static const double kLn2 = 0.69314718055994530942;
static const double kC2 = 1.438776877;          /* hc/k_B [cm K] */
static const double kTref = 296.0;              /* HITRAN reference temperature */
static const double kBoltz = 1.380649e-23;      /* [J/K] */
static const double kAvogadro = 6.02214076e23;  /* [1/mol] */
static const double kLight = 299792458.0;       /* [m/s] */
static const double kAtm = 101325.0;            /* [Pa] */
static const double kH0 = 1.0 / 2048.0;         /* finest step, 10/20480 cm^-1 */

/* ------------------------------------------------------------------ */
/* Dawson's integral D(x) = exp(-x^2) * int_0^x exp(t^2) dt            */
/* Small |x|: its Maclaurin series.  Otherwise Rybicki's sampling      */
/* formula D(x) = lim_{h->0} pi^{-1/2} sum_{n odd} exp(-(x-nh)^2)/n,    */
/* whose error for step h is of order exp(-(pi/(2h))^2); h = 0.2.      */
/* ------------------------------------------------------------------ */
double orc_dawson(double x) {
  double ax = fabs(x), r;
  if (ax < 0.5) {
    double term = ax, sum = ax, x2 = ax * ax;
    for (int k = 1; k < 60; ++k) {
      term *= -2.0 * x2 / (2.0 * k + 1.0);
      sum += term;
      if (fabs(term) < 1e-18 * fabs(sum)) break;
    }
    r = sum;
  } else {
    const double h = 0.2;
    long n0 = (long)floor((ax - 7.5) / h), n1 = (long)ceil((ax + 7.5) / h);
    double sum = 0.0;
    for (long n = n0; n <= n1; ++n) {
      if ((n & 1L) == 0) continue;
      double u = ax - (double)n * h;
      sum += exp(-u * u) / (double)n;
    }
    r = sum / kSqrtPi;
  }
  return x < 0 ? -r : r;
}

/* ------------------------------------------------------------------ */
/* Voigt function K(x,y) of Eq.(8), K = Re w(x+iy), w the Faddeeva     */
/* function.  Three regions, each an exact representation of w:        */
/*  (a) |z| >= 7: asymptotic series w ~ i/(sqrt(pi) z) sum_k            */
/*      (2k-1)!!/(2z^2)^k, truncated at its smallest term;              */
/*  (b) y >= 0.5, |z| < 7: Laplace continued fraction for               */
/*      pi^{-1/2} int exp(-t^2)/(z-t) dt with partial numerators k/2,   */
/*      depth ~200/y^2 (the Gauss-Hermite convergents);                 */
/*  (c) y < 0.5, |z| < 7: Taylor series in y about the real axis, with  */
/*      w(x) = exp(-x^2) + 2i D(x)/sqrt(pi), w' = -2zw + 2i/sqrt(pi),   */
/*      w^(n+1) = -2x w^(n) - 2n w^(n-1).                               */
/* ------------------------------------------------------------------ */
static double voigt_series(double x, double y) {
  /* z = x + iy; 1/(2 z^2) */
  double zr = x, zi = y;
  double z2r = zr * zr - zi * zi, z2i = 2.0 * zr * zi;
  double den = 2.0 * (z2r * z2r + z2i * z2i);
  double qr = z2r / den, qi = -z2i / den;          /* 1/(2 z^2) */
  double sr = 1.0, si = 0.0, tr = 1.0, ti = 0.0, prev = 1.0;
  for (int k = 1; k < 400; ++k) {
    double f = 2.0 * k - 1.0;
    double nr = f * (tr * qr - ti * qi), ni = f * (tr * qi + ti * qr);
    double mag = hypot(nr, ni);
    if (mag >= prev) break;                          /* smallest term reached */
    tr = nr; ti = ni; prev = mag;
    sr += tr; si += ti;
    if (mag < 1e-19 * hypot(sr, si)) break;
  }
  /* i/(sqrt(pi) z) * s, real part */
  double zz = zr * zr + zi * zi;
  double ir = zi / zz, ii = zr / zz;               /* i/z = (y + i x)/|z|^2 */
  return (ir * sr - ii * si) / kSqrtPi;
}

static double voigt_cfrac(double x, double y) {
  int n = (int)(200.0 / (y * y)) + 30;
  if (n > 200000) n = 200000;
  double tr = x, ti = y;
  for (int k = n; k >= 1; --k) {
    double a = 0.5 * k;
    double d = tr * tr + ti * ti;
    /* t = z - a / t */
    double ur = a * tr / d, ui = -a * ti / d;
    tr = x - ur; ti = y - ui;
  }
  double d = tr * tr + ti * ti;
  double gi = -ti / d;                             /* Im of G = 1/t */
  return -gi / kSqrtPi;                            /* Re(i G)/sqrt(pi) */
}

static double voigt_taylor(double x, double y) {
  double D = orc_dawson(x);
  double wr0 = exp(-x * x), wi0 = 2.0 / kSqrtPi * D;
  double wr1 = -2.0 * x * wr0, wi1 = -2.0 * x * wi0 + 2.0 / kSqrtPi;
  double K = wr0, fact = 1.0, yn = 1.0;
  double wrm = wr0, wim = wi0, wrn = wr1, win = wi1;
  for (int n = 1; n < 120; ++n) {
    fact *= n;
    yn *= y;
    double t;
    switch (n & 3) {
      case 0: t = wrn; break;
      case 1: t = -win; break;
      case 2: t = -wrn; break;
      default: t = win; break;
    }
    double term = t * yn / fact;
    K += term;
    if (n > 4 && fabs(term) < 1e-19 * fabs(K)) break;
    double wr2 = -2.0 * x * wrn - 2.0 * n * wrm, wi2 = -2.0 * x * win - 2.0 * n * wim;
    wrm = wrn; wim = win; wrn = wr2; win = wi2;
  }
  return K;
}

double orc_voigt_K(double x, double y) {
  x = fabs(x);
  if (y < 0) return NAN;
  if (x * x + y * y >= 49.0) return voigt_series(x, y);
  if (y >= 0.5) return voigt_cfrac(x, y);
  return voigt_taylor(x, y);
}

int orc_voigt_K_vec(int64_t n, const double* x, const double* y, double* out) {
  if (n < 0 || (n > 0 && (!x || !y || !out))) return -1;
  for (int64_t i = 0; i < n; ++i) out[i] = orc_voigt_K(x[i], y[i]);
  return 0;
}

/* Tonkov chi-factor, Eq.(10), with the printed inequalities; or the user chi. */
double orc_chi(int32_t chi, double a) {
  if (chi == ORC_CHI_USER) return orc_user_chi(a);
  if (chi != ORC_CHI_TONKOV) return 1.0;
  if (a >= 3.0 && a <= 150.0) return 1.084 * exp(-0.027 * a);
  if (a > 150.0 && a <= 300.0) return 0.208 * exp(-0.016 * a);
  if (a > 300.0) return 0.025 * exp(-0.009 * a);
  return 1.0;
}

/* The user chi's break points (ascending, cm^-1); returns their number. */
int orc_user_chi_breaks(double* out, int cap) {
  if (cap < ORC_USER_CHI_NBREAK || (ORC_USER_CHI_NBREAK > 0 && !out)) return -1;
  for (int i = 0; i < ORC_USER_CHI_NBREAK; ++i) out[i] = orc_user_chi_break[i];
  return ORC_USER_CHI_NBREAK;
}

/* Normalised line shapes of Eq.(4), Eq.(5) and Eq.(7), or the user shape, all
 * centred at the shifted centre; d = nu - nu~0. */
double orc_shape(int32_t shape, double d, double gL, double aD) {
  if (shape == ORC_SHAPE_USER) return orc_user_shape(d, gL, aD);
  if (shape == ORC_SHAPE_LORENTZ || (shape == ORC_SHAPE_VOIGT && aD <= 0.0))
    return gL / (kPi * (gL * gL + d * d));
  if (shape == ORC_SHAPE_DOPPLER) {
    if (aD <= 0.0) return 0.0;
    return sqrt(kLn2 / (kPi * aD * aD)) * exp(-d * d * kLn2 / (aD * aD));
  }
  double s = sqrt(kLn2) / aD;
  return sqrt(kLn2 / kPi) / aD * orc_voigt_K(s * d, s * gL);
}

/* HITRAN-form temperature/pressure dependences (the paper cites them without
 * printing them): S(T) with partition ratio, Boltzmann and stimulated-emission
 * factors; gamma_L = (296/T)^n_air (gamma_air (p - p_self) + gamma_self p_self);
 * alpha_D = nu0/c sqrt(2 ln2 k_B T N_A / M); nu~0 = nu0 + delta_air p. */
int orc_line_state_of(const orc_lines* L, const orc_layer* lay, int64_t j, orc_line_state* o) {
  double T = lay->T_K, p = lay->p_atm, ps = lay->p_self_atm;
  double nu = L->nu0[j];
  double q = lay->q_ratio > 0.0 ? lay->q_ratio : kTref / T;
  double boltz = exp(-kC2 * (double)L->E_lower[j] * (1.0 / T - 1.0 / kTref));
  double stim;
  if (nu > 0.0)
    stim = expm1(-kC2 * nu / T) / expm1(-kC2 * nu / kTref);
  else
    stim = kTref / T;
  o->S = (double)L->S296[j] * q * boltz * stim;
  o->gamma_L = pow(kTref / T, (double)L->n_air[j]) *
               ((double)L->gamma_air[j] * (p - ps) + (double)L->gamma_self[j] * ps);
  o->alpha_D = nu / kLight * sqrt(2.0 * kLn2 * kBoltz * kAvogadro * T / (L->molar_mass * 1e-3));
  o->nu_t = nu + (double)L->delta_air[j] * p;
  return 0;
}

/* the line states of every line of the list (arrays of L->n values) */
int orc_line_states(const orc_lines* L, const orc_layer* lay, double* S, double* gamma_L, double* alpha_D,
                    double* nu_t) {
  if (!L || !lay || !S || !gamma_L || !alpha_D || !nu_t) return -1;
  for (int64_t j = 0; j < L->n; ++j) {
    orc_line_state st;
    orc_line_state_of(L, lay, j, &st);
    S[j] = st.S;
    gamma_L[j] = st.gamma_L;
    alpha_D[j] = st.alpha_D;
    nu_t[j] = st.nu_t;
  }
  return 0;
}

double orc_number_density(const orc_layer* lay) {
  return lay->p_self_atm * kAtm / (kBoltz * lay->T_K) * 1e-6;
}

/* ------------------------------------------------------------------ */
/* validation and per-line preparation shared by both summations       */
/* ------------------------------------------------------------------ */
static int finite_d(double v) { return isfinite(v); }

static int validate(const orc_lines* L, const orc_layer* lay, const orc_request* rq) {
  if (!L || !lay || !rq || L->n < 0) return -1;
  if (!finite_d(rq->nu_begin) || !finite_d(rq->nu_end) || rq->nu_end <= rq->nu_begin) return -1;
  if (rq->nu_begin < 0.0) return -1;
  if (floor(rq->nu_begin * 2048.0) != rq->nu_begin * 2048.0) return -1;
  if (floor(rq->nu_end * 2048.0) != rq->nu_end * 2048.0) return -1;
  if (!(rq->cutoff > 0.0) || !finite_d(rq->cutoff)) return -1;
  if (!(rq->R >= 4.0) || !finite_d(rq->R)) return -1;
  if (rq->stencil != 0 && rq->stencil != 3 && rq->stencil != 4 && rq->stencil != 5) return -1;
  if (!(lay->T_K > 0.0) || !(lay->p_atm >= 0.0) || !(lay->p_self_atm >= 0.0) ||
      lay->p_self_atm > lay->p_atm || !finite_d(lay->T_K) || !finite_d(lay->p_atm))
    return -1;
  if (!(L->molar_mass > 0.0)) return -1;
  for (int64_t j = 0; j < L->n; ++j)
    if (!finite_d(L->nu0[j]) || !isfinite(L->S296[j]) || !isfinite(L->gamma_air[j]) ||
        !isfinite(L->gamma_self[j]) || !isfinite(L->E_lower[j]) || !isfinite(L->n_air[j]) ||
        !isfinite(L->delta_air[j]) || L->S296[j] < 0.0f || L->gamma_air[j] < 0.0f ||
        L->gamma_self[j] < 0.0f || L->nu0[j] < 0.0)
      return -1;
  return 0;
}

typedef struct {
  int64_t n;
  double* S;
  double* gL;
  double* aD;
  double* nu;   /* shifted centre */
} kept_lines;

/* Per-layer line states; lines below prune_rel * max S are dropped (max over the
 * whole supplied list).  Kept lines are sorted by shifted centre. */
static int cmp_pair(const void* a, const void* b) {
  double x = ((const double*)a)[0], y = ((const double*)b)[0];
  return (x > y) - (x < y);
}

static int prepare(const orc_lines* L, const orc_layer* lay, const orc_request* rq, kept_lines* K) {
  int64_t n = L->n;
  orc_line_state* st = (orc_line_state*)malloc(sizeof(orc_line_state) * (size_t)(n > 0 ? n : 1));
  if (!st) return -2;
  double smax = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    orc_line_state_of(L, lay, j, &st[j]);
    if (st[j].S > smax) smax = st[j].S;
  }
  double thr = rq->prune_rel > 0.0 ? rq->prune_rel * smax : -1.0;
  int64_t m = 0;
  double* key = (double*)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
  for (int64_t j = 0; j < n; ++j)
    if (st[j].S >= thr) {
      key[2 * m] = st[j].nu_t;
      key[2 * m + 1] = (double)j;
      ++m;
    }
  qsort(key, (size_t)m, 2 * sizeof(double), cmp_pair);
  K->n = m;
  K->S = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  K->gL = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  K->aD = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  K->nu = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  for (int64_t i = 0; i < m; ++i) {
    int64_t j = (int64_t)key[2 * i + 1];
    K->S[i] = st[j].S;
    K->gL[i] = st[j].gamma_L;
    K->aD[i] = st[j].alpha_D;
    K->nu[i] = st[j].nu_t;
  }
  free(key);
  free(st);
  return 0;
}

static void free_kept(kept_lines* K) {
  free(K->S); free(K->gL); free(K->aD); free(K->nu);
}

static double out_scale(const orc_layer* lay, const orc_request* rq) {
  return rq->out_kind == ORC_OUT_K_KM ? orc_number_density(lay) * 1e5 : 1.0;
}

/* ------------------------------------------------------------------ */
/* the definition: Eq.(3) at each requested node, every kept line with */
/* |nu - nu~0| <= cutoff                                                */
/* ------------------------------------------------------------------ */
typedef struct {
  const kept_lines* K;
  const orc_request* rq;
  const int64_t* nodes;
  double* out;
  int64_t i0, i1;
  double scale;
} direct_job;

static int64_t lower_bound(const double* a, int64_t n, double v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

static void* direct_worker(void* arg) {
  direct_job* jb = (direct_job*)arg;
  const kept_lines* K = jb->K;
  double c = jb->rq->cutoff;
  for (int64_t i = jb->i0; i < jb->i1; ++i) {
    double nu = (double)jb->nodes[i] * kH0;
    int64_t a = lower_bound(K->nu, K->n, nu - c - 1e-9);
    double s = 0.0;
    for (int64_t j = a; j < K->n && K->nu[j] <= nu + c + 1e-9; ++j) {
      double d = nu - K->nu[j];
      if (fabs(d) > c) continue;
      s += K->S[j] * orc_shape(jb->rq->shape, d, K->gL[j], K->aD[j]) * orc_chi(jb->rq->chi, fabs(d));
    }
    jb->out[i] = s * jb->scale;
  }
  return NULL;
}

int orc_direct(const orc_lines* L, const orc_layer* lay, const orc_request* rq,
               const int64_t* nodes, int64_t n_nodes, double* out, int32_t n_threads) {
  if (validate(L, lay, rq)) return -1;
  if (n_nodes < 0 || (n_nodes > 0 && (!nodes || !out))) return -1;
  kept_lines K;
  if (prepare(L, lay, rq, &K)) return -2;
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  direct_job jobs[256];
  double scale = out_scale(lay, rq);
  for (int t = 0; t < n_threads; ++t) {
    jobs[t].K = &K; jobs[t].rq = rq; jobs[t].nodes = nodes; jobs[t].out = out;
    jobs[t].i0 = n_nodes * t / n_threads; jobs[t].i1 = n_nodes * (t + 1) / n_threads;
    jobs[t].scale = scale;
    pthread_create(&th[t], NULL, direct_worker, &jobs[t]);
  }
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  free_kept(&K);
  return 0;
}

/* ------------------------------------------------------------------ */
/* the eleven-grid method, step by step (Section 2.4, our reading)     */
/*                                                                      */
/* Lattices: level 0 has step 2^-11 cm^-1 (N = 20481 per 10 cm^-1);     */
/* levels 1..10 have steps 2^-9 .. 1 cm^-1 (N_i = 10*2^(i-1)+1 points   */
/* per 10 cm^-1, i = 10..1), nodes at nu = m*h.  Region boundaries      */
/* b_l = R*h_(l+1).  A line whose half-width bound w = max(gamma_L,     */
/* alpha_D) satisfies R*h_s <= w starts at level s (largest such s, 0   */
/* if none): level s holds |d| < b_s, level l > s holds b_(l-1) <= |d|  */
/* < b_l, level 10 holds up to the cut-off.  T_l(d) is the part of the  */
/* line that level l and all coarser levels together represent.  Level  */
/* l receives D_l(m) = T_l(d_m) - sum_i w_i T_(l+1)(d_(m_i)) on its      */
/* region and on the nodes whose stencil straddles a jump of T_(l+1)     */
/* (its inner edge, the cut-off, chi breakpoints); elsewhere D_l is the  */
/* interpolation error of a smooth function and is dropped.              */
/* Cascade: A_10 = sum D_10, A_l = sum D_l + P(A_(l+1)), sigma = A_0.   */
/* P is the 3-point (or 5-point) Lagrange interpolation centred on the  */
/* nearest coarse node (ties to the lower one), injection at coinciding  */
/* nodes; Section 2.4 names both orders.                                 */
/* ------------------------------------------------------------------ */
#define NLEV 11

typedef struct {
  int ns;                   /* stencil points, 3, 4 or 5 */
  int64_t r[NLEV];          /* level step in finest steps */
  double h[NLEV];           /* level step [cm^-1] */
  double b[NLEV];           /* b_l = R h_(l+1), l = 0..9 */
  double B[NLEV];           /* band half-width (ns+1)/2 h_(l+1): hull reach from a node */
  int64_t lo[NLEV], hi[NLEV];
  double* A[NLEV];
  double c;
  int32_t shape, chi;
} grid_geom;

static int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

static void make_geom(const orc_request* rq, grid_geom* G) {
  G->ns = rq->stencil == 0 ? 3 : rq->stencil;
  const int half = G->ns == 3 ? 1 : 2;   /* coarse nodes a stencil reaches beyond its interval */
  for (int l = 0; l < NLEV; ++l) {
    if (rq->level_table == 1) G->r[l] = (int64_t)1 << l;
    else G->r[l] = l == 0 ? 1 : ((int64_t)1 << (l + 1));
    G->h[l] = (double)G->r[l] * kH0;
  }
  for (int l = 0; l < NLEV - 1; ++l) {
    G->b[l] = rq->R * G->h[l + 1];
    G->B[l] = (double)(half + 1) * G->h[l + 1];
  }
  G->b[NLEV - 1] = INFINITY;
  G->B[NLEV - 1] = 0.0;
  G->lo[0] = (int64_t)llround(rq->nu_begin * 2048.0);
  G->hi[0] = (int64_t)llround(rq->nu_end * 2048.0);
  for (int l = 0; l < NLEV - 1; ++l) {
    int64_t rho = G->r[l + 1] / G->r[l];
    G->lo[l + 1] = floor_div(G->lo[l], rho) - half;
    G->hi[l + 1] = -floor_div(-G->hi[l], rho) + half;
  }
  G->c = rq->cutoff;
  G->shape = rq->shape;
  G->chi = rq->chi;
}

static int start_level(const grid_geom* G, double R, double w) {
  int s = 0;
  for (int l = 0; l < NLEV; ++l)
    if (R * G->h[l] <= w) s = l;
  return s;
}

/* one kept line */
typedef struct {
  double S, gL, aD, nu;
  int s;
} gline;

static double g_of(const grid_geom* G, const gline* ln, double d) {
  double a = fabs(d);
  if (a > G->c) return 0.0;
  return ln->S * orc_shape(G->shape, d, ln->gL, ln->aD) * orc_chi(G->chi, a);
}

/* T_l(d): the line restricted to what levels >= l represent */
static double T_of(const grid_geom* G, const gline* ln, int l, double d) {
  if (l > ln->s && fabs(d) < G->b[l - 1]) return 0.0;
  return g_of(G, ln, d);
}

static int in_region(const grid_geom* G, const gline* ln, int l, double a) {
  if (a > G->c || l < ln->s) return 0;
  if (l > ln->s && a < G->b[l - 1]) return 0;
  if (l < NLEV - 1 && a >= G->b[l]) return 0;
  return 1;
}

/* jump points of T_(l+1) in |d| */
static int jumps_of(const grid_geom* G, const gline* ln, int l, double* q) {
  int n = 0;
  double lo = 0.0;
  if (l + 1 > ln->s) {
    lo = G->b[l];
    if (lo > G->c) return 0;
    q[n++] = lo;
  }
  q[n++] = G->c;
  if (G->chi == ORC_CHI_TONKOV) {
    const double br[3] = {3.0, 150.0, 300.0};
    for (int i = 0; i < 3; ++i)
      if (br[i] >= lo && br[i] <= G->c) q[n++] = br[i];
  }
  _Static_assert(ORC_USER_CHI_NBREAK <= 6, "q holds 8 jumps");
  if (G->chi == ORC_CHI_USER)
    for (int i = 0; i < ORC_USER_CHI_NBREAK; ++i)
      if (orc_user_chi_break[i] >= lo && orc_user_chi_break[i] <= G->c) q[n++] = orc_user_chi_break[i];
  return n;
}

/* Stencil of level-l node m on level l+1, u = m r_l / r_(l+1) in coarse
 * steps: one node with weight 1 where m coincides with a coarse node;
 * otherwise Lagrange weights w_i(t) = prod_{j != i} (t - j') / (i' - j') over
 * the stencil's offsets i', j'.
 *  3 or 5 points: the ns coarse nodes centred on the nearest one kc (a tie
 *    goes to the lower), k[i] = kc - ns/2 + i, offsets -ns/2 .. ns/2, t = u - kc;
 *  4 points: the two coarse nodes on each side of u, k[i] = q - 1 + i with
 *    q = floor(u), offsets -1 .. 2, t = u - q (at a midpoint the weights are
 *    (-1, 9, 9, -1)/16). */
static int stencil(const grid_geom* G, int l, int64_t m, int64_t* k, double* w) {
  int64_t rho = G->r[l + 1] / G->r[l];
  int64_t q = floor_div(m, rho);
  int64_t rem = m - q * rho;
  if (rem == 0) {
    k[0] = q; w[0] = 1.0;
    return 1;
  }
  double f = (double)rem / (double)rho, t;
  if (G->ns == 4) {
    for (int i = -1; i <= 2; ++i) {
      double v = 1.0;
      for (int j = -1; j <= 2; ++j)
        if (j != i) v *= (f - j) / (double)(i - j);
      k[i + 1] = q + i;
      w[i + 1] = v;
    }
    return 4;
  }
  int64_t kc;
  if (f <= 0.5) { kc = q; t = f; } else { kc = q + 1; t = f - 1.0; }
  const int half = G->ns / 2;
  for (int i = -half; i <= half; ++i) {
    double v = 1.0;
    for (int j = -half; j <= half; ++j)
      if (j != i) v *= (t - j) / (double)(i - j);
    k[i + half] = kc + i;
    w[i + half] = v;
  }
  return G->ns;
}

int orc_stencil_of(const orc_request* rq, int32_t l, int64_t m, int64_t* k, double* w) {
  if (!rq || !k || !w || l < 0 || l >= NLEV - 1) return -1;
  if (rq->stencil != 0 && rq->stencil != 3 && rq->stencil != 4 && rq->stencil != 5) return -1;
  grid_geom G;
  memset(&G, 0, sizeof G);
  make_geom(rq, &G);
  return stencil(&G, l, m, k, w);
}

/* Does the stencil of node m (level l) straddle a jump of T_(l+1)?
 * True when some jump point q lies in the closed |d| hull of the stencil's
 * coarse nodes; only there does interpolating T_(l+1) smear a jump. */
static int straddles(const grid_geom* G, const gline* ln, int l, int64_t m, const double* q, int nq) {
  int64_t k[5];
  double w[5];
  if (stencil(G, l, m, k, w) == 1) return 0;
  double d0 = (double)k[0] * G->h[l + 1] - ln->nu;
  double d2 = (double)k[G->ns - 1] * G->h[l + 1] - ln->nu;
  double lo = (d0 * d2 <= 0.0) ? 0.0 : fmin(fabs(d0), fabs(d2));
  double hi = fmax(fabs(d0), fabs(d2));
  for (int i = 0; i < nq; ++i)
    if (q[i] >= lo && q[i] <= hi) return 1;
  return 0;
}

/* the line's D_l at node m (level l) */
static double D_at(const grid_geom* G, const gline* ln, int l, int64_t m) {
  double d = (double)m * G->h[l] - ln->nu;
  double v = T_of(G, ln, l, d);
  if (l < NLEV - 1) {
    int64_t k[5];
    double w[5];
    int ns = stencil(G, l, m, k, w);
    for (int i = 0; i < ns; ++i)
      v -= w[i] * T_of(G, ln, l + 1, (double)k[i] * G->h[l + 1] - ln->nu);
  }
  return v;
}

typedef struct { int64_t a, b; } ival;

static int cmp_ival(const void* x, const void* y) {
  int64_t a = ((const ival*)x)->a, b = ((const ival*)y)->a;
  return (a > b) - (a < b);
}

static void add_line(const grid_geom* G, const gline* ln, double* const* A) {
  for (int l = 0; l < NLEV; ++l) {
    double h = G->h[l];
    ival iv[16];
    int ni = 0;
    /* region */
    if (l >= ln->s) {
      double inner = (l == ln->s) ? 0.0 : G->b[l - 1];
      double outer = fmin(G->b[l], G->c);
      if (inner <= outer) {
        iv[ni].a = (int64_t)floor((ln->nu - outer) / h) - 1;
        iv[ni].b = (int64_t)ceil((ln->nu + outer) / h) + 1;
        ++ni;
      }
    }
    /* bands around the jumps of T_(l+1) */
    double q[8];
    int nq = (l < NLEV - 1) ? jumps_of(G, ln, l, q) : 0;
    for (int i = 0; i < nq; ++i) {
      double B = G->B[l];
      iv[ni].a = (int64_t)floor((ln->nu + q[i] - B) / h) - 1;
      iv[ni].b = (int64_t)ceil((ln->nu + q[i] + B) / h) + 1;
      ++ni;
      iv[ni].a = (int64_t)floor((ln->nu - q[i] - B) / h) - 1;
      iv[ni].b = (int64_t)ceil((ln->nu - q[i] + B) / h) + 1;
      ++ni;
    }
    if (ni == 0) continue;
    qsort(iv, (size_t)ni, sizeof(ival), cmp_ival);
    int64_t cur = INT64_MIN;
    for (int i = 0; i < ni; ++i) {
      int64_t a = iv[i].a > cur ? iv[i].a : cur;
      int64_t b = iv[i].b;
      if (a < G->lo[l]) a = G->lo[l];
      if (b > G->hi[l]) b = G->hi[l];
      for (int64_t m = a; m <= b; ++m) {
        double d = (double)m * h - ln->nu;
        double ad = fabs(d);
        int use = in_region(G, ln, l, ad);
        if (!use && nq > 0) use = straddles(G, ln, l, m, q, nq);
        if (use) A[l][m - G->lo[l]] += D_at(G, ln, l, m);
      }
      if (iv[i].b + 1 > cur) cur = iv[i].b + 1;
    }
  }
}

typedef struct {
  const grid_geom* G;
  const kept_lines* K;
  double R;
  int64_t j0, j1;
  double* A[NLEV];
} grid_job;

static void* grid_worker(void* arg) {
  grid_job* jb = (grid_job*)arg;
  const grid_geom* G = jb->G;
  double numin = (double)G->lo[NLEV - 1] * G->h[NLEV - 1] - G->c - 4.0;
  double numax = (double)G->hi[NLEV - 1] * G->h[NLEV - 1] + G->c + 4.0;
  for (int64_t j = jb->j0; j < jb->j1; ++j) {
    gline ln;
    ln.S = jb->K->S[j]; ln.gL = jb->K->gL[j]; ln.aD = jb->K->aD[j]; ln.nu = jb->K->nu[j];
    if (ln.nu < numin || ln.nu > numax) continue;
    ln.s = start_level(G, jb->R, fmax(ln.gL, ln.aD));
    add_line(G, &ln, jb->A);
  }
  return NULL;
}

int orc_grid(const orc_lines* L, const orc_layer* lay, const orc_request* rq,
             double* out, int32_t n_threads) {
  if (validate(L, lay, rq)) return -1;
  if (rq->level_table != 0 && rq->level_table != 1) return -1;
  if (!out) return -1;
  kept_lines K;
  if (prepare(L, lay, rq, &K)) return -2;
  grid_geom G;
  make_geom(rq, &G);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 64) n_threads = 64;
  pthread_t th[64];
  grid_job* jobs = (grid_job*)calloc((size_t)n_threads, sizeof(grid_job));
  int err = 0;
  for (int t = 0; t < n_threads; ++t) {
    jobs[t].G = &G; jobs[t].K = &K; jobs[t].R = rq->R;
    jobs[t].j0 = K.n * t / n_threads; jobs[t].j1 = K.n * (t + 1) / n_threads;
    for (int l = 0; l < NLEV; ++l) {
      jobs[t].A[l] = (double*)calloc((size_t)(G.hi[l] - G.lo[l] + 1), sizeof(double));
      if (!jobs[t].A[l]) err = 1;
    }
  }
  if (!err) {
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, grid_worker, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    /* reduce the per-thread level arrays in thread order */
    for (int l = 0; l < NLEV; ++l) {
      G.A[l] = jobs[0].A[l];
      int64_t n = G.hi[l] - G.lo[l] + 1;
      for (int t = 1; t < n_threads; ++t)
        for (int64_t i = 0; i < n; ++i) G.A[l][i] += jobs[t].A[l][i];
    }
    /* cascade, coarse to fine */
    for (int l = NLEV - 2; l >= 0; --l) {
      for (int64_t m = G.lo[l]; m <= G.hi[l]; ++m) {
        int64_t k[5];
        double w[5];
        int ns = stencil(&G, l, m, k, w);
        double v = 0.0;
        for (int i = 0; i < ns; ++i) v += w[i] * G.A[l + 1][k[i] - G.lo[l + 1]];
        G.A[l][m - G.lo[l]] += v;
      }
    }
    double scale = out_scale(lay, rq);
    int64_t n0 = G.hi[0] - G.lo[0] + 1;
    for (int64_t i = 0; i < n0; ++i) out[i] = G.A[0][i] * scale;
  }
  for (int t = 0; t < n_threads; ++t)
    for (int l = 0; l < NLEV; ++l) free(jobs[t].A[l]);
  free(jobs);
  free_kept(&K);
  return err ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* FP64 reference for the small fully connected network                */
/* ------------------------------------------------------------------ */
static double silu(double v) { return v / (1.0 + exp(-v)); }
static double dsilu(double v) {
  double s = 1.0 / (1.0 + exp(-v));
  return s * (1.0 + v * (1.0 - s));
}

static int64_t param_count(int32_t nl, const int32_t* wd) {
  int64_t n = 0;
  for (int l = 0; l < nl; ++l) n += (int64_t)wd[l + 1] * wd[l] + wd[l + 1];
  return n;
}

int orc_mlp_forward(int32_t nl, const int32_t* wd, const double* P, const double* X,
                    int64_t batch, double* Y) {
  if (nl < 1 || nl > 16 || !wd || !P || !X || !Y || batch < 0) return -1;
  int maxw = 0;
  for (int l = 0; l <= nl; ++l) {
    if (wd[l] < 1 || wd[l] > 4096) return -1;
    if (wd[l] > maxw) maxw = wd[l];
  }
  double* a = (double*)malloc(sizeof(double) * (size_t)maxw);
  double* z = (double*)malloc(sizeof(double) * (size_t)maxw);
  for (int64_t bi = 0; bi < batch; ++bi) {
    for (int i = 0; i < wd[0]; ++i) a[i] = X[bi * wd[0] + i];
    const double* p = P;
    for (int l = 0; l < nl; ++l) {
      const double* W = p;
      const double* bb = p + (size_t)wd[l + 1] * wd[l];
      for (int o = 0; o < wd[l + 1]; ++o) {
        double s = bb[o];
        for (int i = 0; i < wd[l]; ++i) s += W[(size_t)o * wd[l] + i] * a[i];
        z[o] = (l < nl - 1) ? silu(s) : s;
      }
      for (int o = 0; o < wd[l + 1]; ++o) a[o] = z[o];
      p += (size_t)wd[l + 1] * wd[l] + wd[l + 1];
    }
    for (int o = 0; o < wd[nl]; ++o) Y[bi * wd[nl] + o] = a[o];
  }
  free(a);
  free(z);
  return 0;
}

int orc_mlp_loss_grad(int32_t nl, const int32_t* wd, const double* P, const double* X,
                      const double* target, int64_t batch, double* loss, double* grad) {
  if (nl < 1 || nl > 16 || !wd || !P || !X || !target || !loss || !grad || batch < 1) return -1;
  if (wd[nl] != 1) return -1;
  int64_t np = param_count(nl, wd);
  memset(grad, 0, sizeof(double) * (size_t)np);
  int maxw = 0;
  for (int l = 0; l <= nl; ++l) if (wd[l] > maxw) maxw = wd[l];
  /* activations a_l (post) and pre-activations z_l per layer for one sample */
  double* acts = (double*)malloc(sizeof(double) * (size_t)(nl + 1) * maxw);
  double* pre = (double*)malloc(sizeof(double) * (size_t)(nl + 1) * maxw);
  double* delta = (double*)malloc(sizeof(double) * (size_t)maxw);
  double* dprev = (double*)malloc(sizeof(double) * (size_t)maxw);
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)nl);
  int64_t o0 = 0;
  for (int l = 0; l < nl; ++l) { off[l] = o0; o0 += (int64_t)wd[l + 1] * wd[l] + wd[l + 1]; }
  double L = 0.0;
  for (int64_t bi = 0; bi < batch; ++bi) {
    for (int i = 0; i < wd[0]; ++i) acts[i] = X[bi * wd[0] + i];
    for (int l = 0; l < nl; ++l) {
      const double* W = P + off[l];
      const double* bb = W + (size_t)wd[l + 1] * wd[l];
      for (int o = 0; o < wd[l + 1]; ++o) {
        double s = bb[o];
        for (int i = 0; i < wd[l]; ++i) s += W[(size_t)o * wd[l] + i] * acts[(size_t)l * maxw + i];
        pre[(size_t)(l + 1) * maxw + o] = s;
        acts[(size_t)(l + 1) * maxw + o] = (l < nl - 1) ? silu(s) : s;
      }
    }
    double e = acts[(size_t)nl * maxw] - target[bi];
    L += e * e;
    delta[0] = 2.0 * e / (double)batch;     /* dL/dz at the output */
    for (int l = nl - 1; l >= 0; --l) {
      double* gW = grad + off[l];
      double* gb = gW + (size_t)wd[l + 1] * wd[l];
      const double* W = P + off[l];
      for (int o = 0; o < wd[l + 1]; ++o) {
        gb[o] += delta[o];
        for (int i = 0; i < wd[l]; ++i) gW[(size_t)o * wd[l] + i] += delta[o] * acts[(size_t)l * maxw + i];
      }
      if (l > 0) {
        for (int i = 0; i < wd[l]; ++i) {
          double s = 0.0;
          for (int o = 0; o < wd[l + 1]; ++o) s += W[(size_t)o * wd[l] + i] * delta[o];
          dprev[i] = s * dsilu(pre[(size_t)l * maxw + i]);
        }
        for (int i = 0; i < wd[l]; ++i) delta[i] = dprev[i];
      }
    }
  }
  *loss = L / (double)batch;
  free(acts); free(pre); free(delta); free(dprev); free(off);
  return 0;
}
