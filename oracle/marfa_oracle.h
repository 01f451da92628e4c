/*
 * marfa_oracle.h -- plain FP64 CPU oracle for eleven-grid line-by-line absorption.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its Python binding) never links, loads or calls it, and
 * the oracle shares no code, header, table or constant generator with it.
 *
 * Everything is computed in double precision, slowly and plainly:
 *   orc_voigt_K   -- the Voigt function K(x,y) of Eq.(8) (Section 2.2)
 *   orc_line_state-- S(T), gamma_L(p,T), alpha_D(T), shifted centre (Section 2.2,
 *                    "Spectroscopy" module; HITRAN forms, our reading)
 *   orc_direct    -- the definition: Eq.(3) summed over every kept line within the
 *                    cut-off at the requested nodes (Section 2.4, cut-off)
 *   orc_grid      -- the eleven-grid method of Section 2.4 step by step (our
 *                    reading of the lattices, regions, residual bands and the
 *                    3-point interpolation cascade)
 * Every function returns 0 on success and a negative value on invalid input.
 */
#ifndef MARFA_ORACLE_H
#define MARFA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Line list, structure-of-arrays, one entry per line; fields of the 36-byte
 * database record of Appendix B (nu in FP64, the rest FP32). */
typedef struct {
  int64_t n;
  const double* nu0;        /* transition wavenumber [cm^-1] */
  const float* S296;        /* intensity at 296 K [cm/molecule] */
  const float* gamma_air;   /* air-broadened HWHM at 296 K [cm^-1/atm] */
  const float* gamma_self;  /* self-broadened HWHM at 296 K [cm^-1/atm] */
  const float* E_lower;     /* lower-state energy [cm^-1] */
  const float* n_air;       /* temperature exponent of gamma */
  const float* delta_air;   /* pressure shift [cm^-1/atm] */
  double molar_mass;        /* [g/mol] */
} orc_lines;

typedef struct {
  double p_atm;             /* total pressure [atm] */
  double T_K;               /* temperature [K] */
  double p_self_atm;        /* partial pressure of the absorber [atm] */
  double q_ratio;           /* Q(296)/Q(T); <= 0 selects 296/T */
} orc_layer;

/* USER: the compiled-in orc_user_shape / orc_user_chi of orc_user.h */
enum { ORC_SHAPE_VOIGT = 0, ORC_SHAPE_LORENTZ = 1, ORC_SHAPE_DOPPLER = 2, ORC_SHAPE_USER = 3 };
enum { ORC_CHI_NONE = 0, ORC_CHI_TONKOV = 1, ORC_CHI_USER = 2 };
enum { ORC_OUT_SIGMA = 0, ORC_OUT_K_KM = 1 };

typedef struct {
  double nu_begin, nu_end;  /* output interval, multiples of 2^-11 cm^-1 */
  double cutoff;            /* line cut-off [cm^-1], |nu - nu~0| <= cutoff */
  int32_t shape, chi, out_kind;
  int32_t level_table;      /* 0: steps 2^-11, 2^-9 .. 1; 1: 2^-11 .. 2^-1 */
  double prune_rel;         /* keep S >= prune_rel * max S; 0 keeps all */
  double R;                 /* region multiple of the level step */
  int32_t stencil;          /* interpolation points between levels: 3 (default, 0 = 3), 4 or 5 */
} orc_request;

typedef struct {
  double S;                 /* S(T) [cm/molecule] */
  double gamma_L;           /* Lorentz HWHM [cm^-1] */
  double alpha_D;           /* Doppler HWHM [cm^-1] */
  double nu_t;              /* pressure-shifted centre [cm^-1] */
} orc_line_state;

double orc_dawson(double x);
double orc_voigt_K(double x, double y);
/* element-wise K over n points */
int orc_voigt_K_vec(int64_t n, const double* x, const double* y, double* out);
double orc_chi(int32_t chi, double absd);
/* coarse nodes k[] and weights w[] (up to 5 each) of the interpolation of
 * level-l node m from level l + 1 under rq's level table and stencil;
 * returns their number, or -1 */
int orc_stencil_of(const orc_request* rq, int32_t l, int64_t m, int64_t* k, double* w);
/* break points of the user chi (ascending, cm^-1) into out[cap]; their number, or -1 */
int orc_user_chi_breaks(double* out, int cap);
/* normalised line shape F(d) [cm], d = nu - nu~0 */
double orc_shape(int32_t shape, double d, double gamma_L, double alpha_D);
int orc_line_state_of(const orc_lines* L, const orc_layer* lay, int64_t j, orc_line_state* out);
/* number density of the absorber [cm^-3] */
/* orc_line_state_of for every line: S, gamma_L, alpha_D, nu_t arrays of L->n values. */
int orc_line_states(const orc_lines* L, const orc_layer* lay, double* S, double* gamma_L, double* alpha_D,
                    double* nu_t);
double orc_number_density(const orc_layer* lay);

/* Definition (direct sum) at nodes nu = nodes[i] * 2^-11. */
int orc_direct(const orc_lines* L, const orc_layer* lay, const orc_request* rq,
               const int64_t* nodes, int64_t n_nodes, double* out, int32_t n_threads);
/* Eleven-grid method over [nu_begin, nu_end]; out has (nu_end-nu_begin)*2048+1 entries. */
int orc_grid(const orc_lines* L, const orc_layer* lay, const orc_request* rq,
             double* out, int32_t n_threads);

/* Small fully connected network, FP64 (reference for the learned line shape):
 * widths[0] inputs -> ... -> widths[n_layers] outputs, SiLU on hidden layers,
 * identity on the output.  Weights W_l are row-major [out][in], biases b_l [out],
 * packed layer after layer as W_0, b_0, W_1, b_1, ...  X is [batch][widths[0]]. */
int orc_mlp_forward(int32_t n_layers, const int32_t* widths, const double* params,
                    const double* X, int64_t batch, double* Y);
/* Mean-squared-error loss L = mean_b (Y_b - target_b)^2 for a single output,
 * and its gradient with respect to every parameter (same packing). */
int orc_mlp_loss_grad(int32_t n_layers, const int32_t* widths, const double* params,
                      const double* X, const double* target, int64_t batch,
                      double* loss, double* grad);

#ifdef __cplusplus
}
#endif
#endif
