/*
 * marfa.h -- C ABI of the MI355X (gfx950) eleven-grid line-by-line absorption
 * library.
 *
 * What it computes (MARFA, arXiv 2411.03418):
 *   sigma(nu; p, T) = sum_j S_j(T) f_j(nu - nu~0_j; gamma_L, alpha_D) chi(|nu - nu~0_j|)
 *   over every line j with |nu - nu~0_j| <= cutoff                 -- Eq.(3), Section 2.1
 *   k(nu; p, T)     = n(p_self, T) * sigma                          -- Eq.(2), Section 2.1
 * on the lattice nu = m * 2^-11 cm^-1 (10/20480, Appendix A), one spectrum per
 * pressure-temperature layer, evaluated with the eleven-grid interpolation
 * technique of Section 2.4 (line centres on the finest grid, wings on ten
 * coarser grids, 3-point interpolation back to the finest grid).  Line shapes:
 * Voigt (default, Eq.(7)-(8)), Lorentz (Eq.(4)), Doppler (Eq.(5)) or a user
 * shape; wing factor: none, Tonkov (Eq.(10), Section 2.3) or a user chi.  The
 * user shape and chi are compile-time plug-ins (the user-selectable shape and
 * chi functions of Sections 2.2-2.3): structs MarfaUserShape / MarfaUserChi in
 * a header built into the kernels (the shipped example: the Thompson-Cox-
 * Hastings pseudo-Voigt and a stepped stretched-exponential chi).  Line parameters follow the database
 * record of Appendix B; their temperature/pressure dependences are the HITRAN
 * forms the paper cites (Section 2.2).
 *
 * Conventions
 *  - Every function returns a marfa_status; nothing throws across the ABI.
 *    marfa_last_error() gives a thread-local text for the last failure.
 *  - Host inputs are borrowed for the duration of the call and copied.
 *  - Device outputs are caller-owned device memory on the plan's device.
 *  - A plan is not thread-safe; distinct plans are independent.
 *  - Execution is asynchronous on the caller's HIP stream.
 */
#ifndef MARFA_H
#define MARFA_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MARFA_OK = 0,
  MARFA_E_INVALID = -1,      /* an argument violates the rules stated below */
  MARFA_E_NOMEM = -2,        /* host or device allocation failed */
  MARFA_E_DEVICE = -3,       /* HIP error, or no usable gfx950 device */
  MARFA_E_UNSUPPORTED = -4,  /* valid but not available (e.g. untrained surrogate) */
  MARFA_E_STATE = -5,        /* call out of order */
  MARFA_E_IO = -6            /* a file could not be opened or written */
} marfa_status;

typedef enum {
  MARFA_SHAPE_VOIGT = 0,
  MARFA_SHAPE_LORENTZ = 1,
  MARFA_SHAPE_DOPPLER = 2,
  MARFA_SHAPE_USER = 3        /* the compiled-in MarfaUserShape */
} marfa_shape;
typedef enum {
  MARFA_CHI_NONE = 0,
  MARFA_CHI_TONKOV = 1,
  MARFA_CHI_USER = 2          /* the compiled-in MarfaUserChi, with its declared breaks */
} marfa_chi;
typedef enum { MARFA_OUT_SIGMA_CM2 = 0, MARFA_OUT_K_PER_KM = 1 } marfa_output;
typedef enum { MARFA_EVAL_PLAIN = 0, MARFA_EVAL_SURROGATE = 1 } marfa_eval;

/* Line list, structure of arrays in HOST memory, n entries each (fields of the
 * 36-byte record of Appendix B).  Any order; the plan sorts by nu0.
 * Rules: 0 <= n <= 2^26 - 1; every value finite; nu0 >= 0; S296, gamma_* >= 0;
 * molar_mass_g > 0.  mol_iso may be NULL (it is carried, not used). */
typedef struct {
  int64_t n;
  const double* nu0;          /* transition wavenumber [cm^-1] */
  const float* S296;          /* intensity at 296 K [cm/molecule] */
  const float* gamma_air;     /* air-broadened HWHM at 296 K, 1 atm [cm^-1/atm] */
  const float* gamma_self;    /* self-broadened HWHM at 296 K, 1 atm [cm^-1/atm] */
  const float* E_lower;       /* lower-state energy E'' [cm^-1] */
  const float* n_air;         /* temperature exponent of the half-width */
  const int32_t* mol_iso;     /* joint molecule/isotopologue id */
  const float* delta_air;     /* pressure shift at 296 K [cm^-1/atm] */
  double molar_mass_g;        /* [g/mol] */
} marfa_lines;

/* One pressure-temperature layer.  Rules: T_K > 0, 0 <= p_self_atm <= p_atm.
 * q_ratio = Q(296)/Q(T); a value <= 0 selects 296/T. */
typedef struct {
  double p_atm, T_K, p_self_atm, q_ratio;
} marfa_layer;

/* Request.  Rules: nu_begin >= 0, nu_end > nu_begin, both multiples of 2^-11;
 * cutoff > 0 (cm^-1, inclusive, measured from the shifted centre);
 * R an integer in [4, 4096] (region multiple of the level step, default 48);
 * level_table 0 (steps 2^-11, 2^-9, ..., 1 cm^-1) or 1 (2^-11, ..., 2^-1);
 * prune_rel in [0, 1): lines with S(T) < prune_rel * max_j S_j(T) are dropped
 * per layer (max over the whole list); fp64 = 1 runs the device path in double
 * precision (output then FP64); stencil 0, 3, 4 or 5.  Zero-initialise reserved
 * fields. */
typedef struct {
  double nu_begin, nu_end;
  double cutoff;
  int32_t shape;              /* marfa_shape */
  int32_t chi;                /* marfa_chi */
  int32_t out_kind;           /* marfa_output */
  int32_t eval;               /* marfa_eval: MARFA_EVAL_PLAIN evaluates the line shapes
                                 directly; MARFA_EVAL_SURROGATE through the learned line
                                 shape attached with marfa_plan_set_surrogate (the execute
                                 calls return MARFA_E_UNSUPPORTED while none is attached).
                                 marfa_plan_set_eval switches it later. */
  double prune_rel;
  double R;
  int32_t level_table;
  int32_t fp64;
  int32_t stencil;            /* interpolation points between levels: 3 (0 = 3) or 5,
                                 centred on the nearest coarse node (Section 2.4
                                 names both; 5 points lower the interpolation error
                                 tens of times at equal R), or 4, the symmetric rule
                                 on the two coarse nodes on each side ((-1, 9, 9, -1)/16
                                 at a midpoint), between them in error and cost.  The
                                 learned shape runs with 3 points. */
  int32_t reserved[3];
} marfa_request;

typedef struct marfa_plan marfa_plan;

/* Per-plan counters from the last marfa_plan_count(): exact (node, line) pairs
 * evaluated, split by level and by line-shape branch, and the work they stand
 * for.  Counted flops are a static count of the single-precision kernel
 * source per unit of work (fused multiply-add = 2, add / multiply = 1,
 * reciprocal / exp2 = 1; compares, selects and integer address arithmetic not
 * counted): flops_per_eval for one line-shape evaluation of the wing form with
 * its distance, chi factor and accumulation (every evaluation, core ones
 * included, computes it), flops_per_core for the Taylor core added on top,
 * flops_per_term per further term of the wing series, flops_per_band per
 * residual-band correction (the stencil interpolation and the difference),
 * flops_per_cascade per interpolated node of the cascade.  Algorithmic bytes
 * count each line record read once per layer and every level and output node
 * written once. */
typedef struct {
  int64_t points_per_layer;       /* output nodes per layer */
  int32_t n_layers;
  int64_t lines_total;            /* lines in the plan */
  int64_t lines_kept;             /* sum over layers of lines kept after pruning */
  int64_t pairs_level[11];        /* pairs with a non-zero contribution, per level */
  int64_t pairs_core;             /* Voigt evaluations in the core branch (|z| < 6) */
  int64_t pairs_wing;             /* evaluations in the wing series branch */
  int64_t pairs_band;             /* pairs carrying a residual-band correction */
  int64_t wing_terms;             /* sum over wing evaluations of series terms beyond the first */
  int64_t level_nodes;            /* nodes of levels 1..10 over all layers */
  int64_t iters_level[11];        /* wavefront iterations over line windows, per level */
  int64_t band_iters_level[11];   /* of which ran a residual-band correction */
  double flops_per_eval, flops_per_core, flops_per_term, flops_per_band, flops_per_cascade;
  double flops_level;             /* counted flops of the level kernel, all layers */
  double flops_cascade;           /* counted flops of the cascade, all layers */
  double bytes_level;             /* algorithmic bytes of the level kernel: records read, level and output nodes written */
  double bytes_cascade;           /* algorithmic bytes of the cascade: 3 (4, 5) coarse reads and 1 read-modify-write per node */
} marfa_stats;

/* Create a plan: validates and copies the inputs, sorts lines by nu0, uploads
 * them to `device`, sizes the workspace.  n_layers >= 1.  On success *out
 * receives the plan (destroy with marfa_plan_destroy).
 * Errors: MARFA_E_INVALID for any rule above; MARFA_E_DEVICE if the device is
 * missing or not gfx950; MARFA_E_NOMEM on allocation failure. */
marfa_status marfa_plan_create(marfa_plan** out, const marfa_lines* lines,
                               const marfa_layer* layers, int32_t n_layers,
                               const marfa_request* req, int32_t device);

/* Output nodes per layer: (nu_end - nu_begin) * 2048 + 1. */
marfa_status marfa_plan_points(const marfa_plan* plan, int64_t* points_per_layer);

/* Compute every layer into out_dev (device memory, FP32, or FP64 if fp64),
 * layout [n_layers][layer_stride], node m of layer L at out[L*stride + m],
 * m = 0 .. points-1 <-> nu = nu_begin + m 2^-11.  layer_stride >= points.
 * hip_stream is a hipStream_t (NULL = legacy default stream).  Asynchronous.
 * The first call on a plan captures the work into a HIP graph; later calls
 * with the same (out_dev, layer_stride, stream) replay it. */
marfa_status marfa_execute(marfa_plan* plan, void* out_dev, int64_t layer_stride, void* hip_stream);

/* As marfa_execute for layers [first, first+count) only; out_dev points at
 * the slot of layer `first`.  Never graph-captured. */
marfa_status marfa_execute_layers(marfa_plan* plan, int32_t first, int32_t count,
                                  void* out_dev, int64_t layer_stride, void* hip_stream);

/* Count pairs exactly (runs the same loops without evaluating shapes) and
 * fill *stats.  Synchronous. */
marfa_status marfa_plan_count(marfa_plan* plan, marfa_stats* stats);

/* Tile parameters of the level kernel, as chosen at plan creation from the
 * line density or by marfa_plan_tune.
 *  item_nodes     nodes per work item on levels with step >= 16 fine units;
 *                 finer levels take 16/step times as many
 *  blocks_per_cu  persistent workgroups per compute unit
 *  tuned          1 once marfa_plan_tune has run on the plan
 *  wave_nodes[l]  region tile of level l: nodes per wavefront (the other
 *                 64 / wave_nodes lanes split the line window)
 *  tune_ms        wall time of the last marfa_plan_tune */
typedef struct {
  int32_t item_nodes;
  int32_t blocks_per_cu;
  int32_t tuned;
  int32_t wave_nodes[11];
  float tune_ms;
} marfa_tiles;
marfa_status marfa_plan_tiles(const marfa_plan* plan, marfa_tiles* tiles);
/* Use given tile parameters (e.g. from an earlier marfa_plan_tune of a plan
 * of the same shape) instead of tuning: item_nodes a multiple of 64 in
 * [64, 8192], blocks_per_cu in [1, 32], wave_nodes[l] a power of two in
 * [1, 64]; tuned and tune_ms are ignored.  Graphs are rebuilt on the next
 * execute.  Errors: MARFA_E_INVALID, MARFA_E_NOMEM. */
marfa_status marfa_plan_set_tiles(marfa_plan* plan, const marfa_tiles* tiles);

/* Autotuner: runs line preparation, then times the level kernel on the
 * device for candidate tile parameters with the plan's own lines and layers
 * and keeps the fastest -- per level the region tile (wave_nodes 1, 2, 4,
 * ..., 64), then the work-item size (128, 256, 512) and the persistent
 * grid (4, 8, 16 workgroups per CU), then one pass over the levels trying
 * each tile's two neighbouring widths with the whole stage timed.
 * scratch_out_dev is an output buffer as for marfa_execute (overwritten).
 * Synchronous on hip_stream; captured graphs are rebuilt on the next
 * execute.  Tile shapes change the summation order, so results may change
 * in the last bits, not in accuracy.  Errors as marfa_execute. */
marfa_status marfa_plan_tune(marfa_plan* plan, void* scratch_out_dev, int64_t layer_stride,
                             void* hip_stream);

/* As marfa_execute, but the three stages (line preparation, level
 * accumulation, cascade) are launched as three graphs on hip_stream with HIP
 * events recorded on that stream between them; waits for completion and
 * returns each stage's duration in *t.  Same kernels and arguments as
 * marfa_execute (used to time the dominant kernel). */
typedef struct {
  float prep_ms, level_ms, cascade_ms, total_ms;
} marfa_timing;
marfa_status marfa_execute_timed(marfa_plan* plan, void* out_dev, int64_t layer_stride, void* hip_stream,
                                 marfa_timing* t);

void marfa_plan_destroy(marfa_plan* plan);

/* ------------------------------------------------------------------
 * Learned line shape (the surrogate of the Voigt x chi line shape).
 *
 * A 3-64-64-64-64-1 SiLU network, weights rounded to BF16, evaluated and
 * trained with BF16-in / FP32-accumulate matrix-core instructions.  For a
 * line with Voigt parameters x = sqrt(ln2) d / alpha_D, y = sqrt(ln2)
 * gamma_L / alpha_D (Eq.(7)-(8)) it predicts t = log(K chi) - log(Kb), the
 * residual of K(x, y) chi(|d|) (Eq.(10)) against the analytic base
 *   Kb = y (1 + (3x^2 - y^2) / (2 rho^2 + 1)) / (sqrt(pi) (rho + exp(-rho) / 2))
 *        + exp(-x^2) / (1 + sqrt(pi) y)^2,   rho = x^2 + y^2,
 * from the inputs f = (asinh|x| / 8, log10(y) / 2, max(|d| - 3, 0) / c)
 * (|d|, c in cm^-1).  A network serves one (chi, cut-off) pair.  Parameters
 * are 12801 FP32 values packed as W0[64][3], b0[64], W1[64][64], b1[64],
 * W2, b2, W3, b3, W4[1][64], b4[1] (row-major [out][in]).
 * ------------------------------------------------------------------ */
typedef struct marfa_surrogate marfa_surrogate;

/* Lines and layers a surrogate is trained for: line centres in
 * [nu_lo, nu_hi] cm^-1 and temperatures in [T_lo, T_hi] K (the Doppler widths
 * of the samples), molar mass in g/mol.  All > 0, lo <= hi. */
typedef struct {
  double nu_lo, nu_hi;
  double T_lo, T_hi;
  double molar_mass_g;
} marfa_sample_cfg;

/* Training run: n_train samples drawn once (n_val more for validation),
 * `epochs` passes in mini-batches of `batch` (a multiple of 32), Adam (state
 * reset at the start of the run) with a cosine learning-rate schedule from
 * lr_max to lr_min after a 2 % warm-up, samples from a counter-based
 * generator seeded by `seed`.  loss_power 2 minimises the mean squared error
 * of t, 4 the mean fourth power (a fine-tuning stage that weights the
 * largest errors).  A run continues from the current parameters. */
typedef struct {
  int64_t n_train, n_val;
  int32_t epochs, batch;
  float lr_max, lr_min;
  uint64_t seed;
  int32_t loss_power;
  int32_t reserved;
} marfa_train_cfg;

/* Outcome: final mini-batch loss, validation mean-squared and mean/max
 * absolute error of t, wall time, optimizer steps, and the largest |x| of
 * the training distribution (pairs beyond it use the plain line shape). */
typedef struct {
  float train_loss, val_loss, val_max_abs, val_mean_abs;
  float ms;
  int64_t steps;
  double x_max;
} marfa_train_report;

/* New network for (chi, cutoff) on `device`: Glorot-uniform weights from a
 * counter-based generator seeded by `seed`, zero biases.  Errors:
 * MARFA_E_INVALID (unknown chi, cutoff <= 0), MARFA_E_UNSUPPORTED (the user chi:
 * the network's distance feature starts at the Tonkov chi's first break),
 * MARFA_E_DEVICE, MARFA_E_NOMEM. */
marfa_status marfa_surrogate_create(marfa_surrogate** out, int32_t chi, double cutoff, uint64_t seed,
                                    int32_t device);
/* Replace / read the FP32 parameters (host arrays of n = 12801 values);
 * setting them resets the optimizer state.  Synchronous: set_params first
 * waits for all work already enqueued on the surrogate's device (plans that
 * evaluate with the old weights finish with them), then returns once the new
 * weights are in place. */
marfa_status marfa_surrogate_set_params(marfa_surrogate* s, const float* params, int64_t n);
marfa_status marfa_surrogate_get_params(const marfa_surrogate* s, float* params, int64_t n);
/* Save and restore a trained network: its 12801 FP32 parameters and the
 * largest |x| of its training distribution (x_max of the train report), the
 * two things a plan reads from it besides the chi and cut-off it was created
 * with.  load sets the parameters as set_params does (synchronous, optimizer
 * state reset) and marks the network trained, so plans can attach it; a plan
 * attached before the call keeps the x_max it read when it attached (attach
 * it again).  Errors: MARFA_E_INVALID (null, n != 12801, a non-finite
 * parameter, x_max not finite and > 0); save: MARFA_E_UNSUPPORTED for a
 * network never trained or loaded. */
marfa_status marfa_surrogate_load(marfa_surrogate* s, const float* params, int64_t n, double x_max);
marfa_status marfa_surrogate_save(const marfa_surrogate* s, float* params, int64_t n, double* x_max);
/* Network output t for n samples: X_dev [n][3] features, out_dev [n], both
 * device memory on the surrogate's device.  Asynchronous on hip_stream. */
marfa_status marfa_surrogate_forward(marfa_surrogate* s, const float* X_dev, int64_t n, float* out_dev,
                                     void* hip_stream);
/* Mean-squared error over n samples (targets T_dev [n]) and its gradient
 * with respect to the 12801 parameters, evaluated with the BF16-rounded
 * weights the forward pass uses; loss and grad are host outputs.  Synchronous. */
marfa_status marfa_surrogate_loss_grad(marfa_surrogate* s, const float* X_dev, const float* T_dev, int64_t n,
                                       float* loss, float* grad);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, allocation-free training or serving loops): the computation of
 * marfa_surrogate_loss_grad with no allocation at all.  Its partial
 * gradients live in a fixed array of the library, one per device, 128
 * workgroups x 12802 floats (6.6 MB), held until the process ends.
 * n: 1 <= n <= 4096 samples (MARFA_E_INVALID beyond).  X_dev [n][3], T_dev [n]
 * as for marfa_surrogate_loss_grad; out_dev: caller-owned device float[12802]
 * on the surrogate's device, receiving the gradient of the mean squared
 * error in [0, 12801) and that error in [12801] -- the same values, bit for
 * bit, that marfa_surrogate_loss_grad returns.  Asynchronous on hip_stream.
 * Every call on one device shares that device's array: calls that overlap
 * on one device race (issue them on one stream). */
marfa_status marfa_surrogate_loss_grad_noalloc(marfa_surrogate* s, const float* X_dev, const float* T_dev, int64_t n,
                                               float* out_dev, void* hip_stream);
/* n training samples on the device (features X_dev [n][3], targets T_dev
 * [n]) with targets from the double-precision device line shape.
 * Asynchronous on hip_stream. */
marfa_status marfa_surrogate_make_samples(marfa_surrogate* s, const marfa_sample_cfg* c, uint64_t seed, int64_t n,
                                          float* X_dev, float* T_dev, void* hip_stream);
/* Draw samples and train on the device (forward, backward and Adam kernels);
 * synchronous (like set_params it first waits for all work enqueued on the
 * device); fills *report and marks the network trained. */
marfa_status marfa_surrogate_train(marfa_surrogate* s, const marfa_sample_cfg* c, const marfa_train_cfg* cfg,
                                   marfa_train_report* report);
void marfa_surrogate_destroy(marfa_surrogate* s);

/* Attach a trained surrogate to a plan (NULL detaches it).  A plan whose
 * eval is MARFA_EVAL_SURROGATE evaluates its line shapes with it; pairs
 * outside the trained domain (y outside [1e-4, 1e3] or |x| above the
 * report's x_max) take the plain line shape.  Requires a single-precision
 * Voigt plan with the 3-point stencil and the surrogate's chi and cut-off.
 * The learned-shape kernel runs on work items of its own (128 nodes, 1024
 * on level 0, allocated here on first attach); marfa_plan_tune always tunes
 * the plain kernel.  The surrogate must outlive its use by the plan.  Waits
 * for the device's queued work before rebuilding the plan's graphs.
 * Errors: MARFA_E_INVALID (mismatch), MARFA_E_UNSUPPORTED (untrained
 * network, another stencil, a cut-off under two coarsest steps),
 * MARFA_E_NOMEM. */
marfa_status marfa_plan_set_surrogate(marfa_plan* plan, const marfa_surrogate* s);

/* Switch the plan's line-shape evaluation (marfa_eval, as the request's
 * eval field).  Waits for the device's queued work before rebuilding the
 * plan's graphs.  Errors: MARFA_E_INVALID for an unknown value. */
marfa_status marfa_plan_set_eval(marfa_plan* plan, int32_t eval);

/* Spectral line database file (Appendix B): packed little-endian records of
 * 36 bytes, one per line, in this order: nu0 (float64), S296, gamma_air,
 * gamma_self, E_lower, n_air (float32 each), mol_iso (int32), delta_air
 * (float32).  No header and no record markers.
 *
 * marfa_linedb_count: *n = file size / 36.  MARFA_E_INVALID for NULL
 * arguments or a size that is not a multiple of 36; MARFA_E_IO if the file
 * cannot be opened.
 * marfa_linedb_read: copies records [first, first + count) into the caller's
 * host arrays (each of count elements; mol_iso may be NULL).  MARFA_E_INVALID
 * for NULL arrays, negative first/count or a range past the end; MARFA_E_IO on
 * a read failure.
 * marfa_linedb_write: writes lines->n records (creating or truncating path);
 * mol_iso NULL writes zeros.  MARFA_E_INVALID for NULL arguments or n < 0,
 * MARFA_E_IO on failure. */
#define MARFA_LINEDB_RECORD 36
marfa_status marfa_linedb_count(const char* path, int64_t* n);
marfa_status marfa_linedb_read(const char* path, int64_t first, int64_t count, double* nu0, float* S296,
                               float* gamma_air, float* gamma_self, float* E_lower, float* n_air,
                               int32_t* mol_iso, float* delta_air);
marfa_status marfa_linedb_write(const char* path, const marfa_lines* lines);

/* PT-table record file (Appendix A).  One binary direct-access file per layer
 * holds records of MARFA_PTBIN_NT = 20481 single-precision values: record r
 * (r >= 1; r = int(nu / 10) for a wavenumber nu inside it) holds the spectrum
 * at nu = 10 r + i / 2048 cm^-1, i = 0 .. 20480 (both interval ends; the last
 * value of record r is the first of record r + 1), at byte offset
 * (r - 1) * 20481 * 4, little-endian.
 *
 * marfa_ptbin_write writes every record whose whole interval [10 r, 10 r + 10]
 * lies inside the n_points lattice values starting at nu_begin (values[i] is the
 * spectrum at nu_begin + i / 2048); other records of the file are left as they
 * are (zero-filled where the file grows past them).  values may be host memory
 * (values_on_device = 0) or device memory on the current device, e.g. a row of
 * marfa_execute's output (values_on_device = 1: copied to the host on
 * hip_stream, which the call then synchronizes).  flags: MARFA_PTBIN_TRUNCATE
 * empties an existing file first.  *records_written (may be NULL) receives the
 * number of records written; zero when no whole interval is covered.
 * Errors: MARFA_E_INVALID (NULL path or values with n_points > 0, n_points < 0,
 * nu_begin negative or not on the 2^-11 cm^-1 lattice, unknown flags),
 * MARFA_E_IO (open or write failed), MARFA_E_DEVICE (copy failed). */
#define MARFA_PTBIN_NT 20481
#define MARFA_PTBIN_TRUNCATE 1
marfa_status marfa_ptbin_write(const char* path, const float* values, int64_t n_points, double nu_begin,
                               int32_t values_on_device, void* hip_stream, int32_t flags,
                               int32_t* records_written);

const char* marfa_status_string(int32_t status);
/* Copy the calling thread's last error text into buf (NUL-terminated). */
marfa_status marfa_last_error(char* buf, size_t n);

/* Device Voigt function for tests: K(x_i, y_i) for n points in HOST arrays,
 * evaluated by the same device code as the hot path (fp64 selects the double
 * instantiation).  Synchronous. */
marfa_status marfa_voigt_eval(int32_t device, int64_t n, const double* x, const double* y,
                              double* out, int32_t fp64);

#ifdef __cplusplus
}
#endif
#endif
