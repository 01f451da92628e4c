// marfa_internal.h -- shared between the host runtime and the HIP kernels of
// the eleven-grid library (not installed; the public ABI is include/marfa.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "marfa.h"
#include "marfa_mlp.h"

namespace marfa {

constexpr int kLevels = 11;      // Section 2.4: eleven grids
constexpr int kGroups = 11;      // lines grouped by start level 0..10
constexpr int kMaxIntervals = 8; // disjoint |d| windows per (level, start-level classes)
constexpr int kMaxJumps = 5;     // jump points of T_(l+1) per (level, start level)
constexpr int kWave = 64;        // CDNA wavefront
constexpr int kWeidemanN64 = 48; // rational-series length of the double-precision Voigt core
constexpr int kBucketPerCm = 256; // line-index buckets per cm^-1 (8 finest steps)
// Single-precision Voigt core: Taylor expansions of the Faddeeva function about
// the centres (i + j sqrt(-1)) / kTaylorPerUnit, 0 <= i, j < kTaylorSide, with
// kTaylorTerms coefficients each (packed as re/im pairs in kTaylorQuads float4)
constexpr int kTaylorPerUnit = 4;
constexpr int kTaylorSide = 25;
constexpr int kTaylorTerms = 9;
constexpr int kTaylorQuads = 5;

// Counted flops per unit of work of the single-precision level kernel, from a
// static count of its source (marfa_level.h; FMA = 2, add / mul = 1,
// rcp / exp2 = 1, compares, selects and integer arithmetic not counted):
//  eval  one wing-form evaluation in the region scan (scan_fast step): distance
//        (1) and its scale to cm (1); shape_wing: gamma^2 (1), d^2 + gamma^2
//        (2), 1/. (1), e (1), -4 gamma^2 (1), U_2 (2), 1 + e U_2 (2), A Q sum
//        (2); chi by its recurrence (1); the product and the sum into the node
//        (2) -- 17
//  core  voigt_core32 on top: x, y (2), their lattice offsets (2 + 4), seven
//        complex Horner steps (56), the last real step (4), the scale (1) -- 69
//  term  one more series term: the coefficient (2), U's recurrence (2), the
//        sum (2) -- 6
//  band  one residual-band correction: the 3-point (4-, 5-point) interpolation
//        (6, 8, 10), the difference (1), the sum into the node (1) -- 8 (10, 12)
//  cascade  one interpolated node: 3 (4, 5) weights times values (6, 8, 10),
//        the sum into the finer level (1) -- 7 (9, 11)
constexpr int kFlopsEval = 17, kFlopsCore = 69, kFlopsTerm = 6;
constexpr int kFlopsBand3 = 8, kFlopsBand4 = 10, kFlopsBand5 = 12;
constexpr int kFlopsCascade3 = 7, kFlopsCascade4 = 9, kFlopsCascade5 = 11;

// Coefficient tables of a device, computed on the host at first use of the
// device and kept until the process ends.
struct DeviceTables {
  double weid[kWeidemanN64 + 2];   // Weideman a_0 .. a_N, then the scale L
  float taylor[kTaylorSide * kTaylorSide * kTaylorQuads * 4];
};

// Lattice geometry, identical for every layer.  Positions are in units of the
// finest step h0 = 2^-11 cm^-1 ("fine units"); node m of level l sits at
// X = m * r[l].
struct Geometry {
  int32_t r[kLevels];        // level step in fine units
  int32_t lnw[kLevels];      // log2 of nodes per wavefront tile (lanes = nodes x line slices)
  int64_t lo[kLevels];       // first node index of each level (incl. halo)
  int64_t n[kLevels];        // nodes per level
  int64_t aoff[kLevels];     // offset of level l >= 1 in a layer's level array
  int64_t a_total;           // level-array length per layer (levels 1..10)
  double b[kLevels];         // region boundary b_l = R r_(l+1), fine units (l < 10)
  double hb[kLevels];        // band reach (ns/2 + 1/2) r_(l+1) + 1, fine units (l < 10)
  double c_fine;             // cut-off in fine units
  // jump points of T_(l+1) for lines starting at or below l (q1) and above l (q2)
  double q1[kLevels][kMaxJumps], q2[kLevels][kMaxJumps];
  int32_t nq1[kLevels], nq2[kLevels];
  int32_t shape, chi, out_kind, fp64;
  int32_t ns, pad_ns;        // stencil points between levels (3 or 5)
  int32_t nbucket;           // buckets of the per-layer line index (kBucketPerCm per cm^-1)
  int32_t pad;
  double bucket_origin;      // wavenumber of bucket 0 [cm^-1] (below every shifted centre)
  int32_t pad2;
  // Tonkov chi pieces as exp2(chi_c0[i] + chi_c1[i] |d|), |d| in cm (host-computed)
  double chi_c0[3], chi_c1[3];
  const double* weid;        // the device's Weideman coefficients (double-precision core)
  const float4* ktab;        // the device's Taylor table (single-precision core)
};

// Region windows (|d| in fine units, closed, disjoint) scanned at one level
// for one combination of start-level classes present in a layer (bit 0: lines
// with s < l, bit 1: s == l, bit 2: s > l), and the jumps of T_(l+1) that the
// residual-band pass corrects.
struct IntervalSet {
  int32_t n_iv;
  int32_t n_jump;
  double a[kMaxIntervals], b[kMaxIntervals];
  // chi over the whole window: exp2(c0 + c1 |d|) (fine units), or chi_mixed = 1
  double chi_c0[kMaxIntervals], chi_c1[kMaxIntervals];
  int32_t chi_mixed[kMaxIntervals];
  // fast region test, one window: fast_ok = 1 when the lines of the level all
  // start below it (annulus |d| in [ra, rbx), two sides), 2 when none starts
  // below it (own region |d| < rbx, ra = 0, one side); rbx is exclusive:
  // min(b_l, next value above the cut-off).  fast_need_s: lines starting
  // above the level are present and are skipped by their start level.  chi
  // over the window is exp2(fc0 + fc1 |d|) unless fchi_mixed.
  double ra64, rbx64;
  float ra32, rbx32;
  double fc0, fc1;
  int32_t fchi_mixed, fast_ok;
  int32_t fast_need_s, fast_pad;
  // jumps of T_(l+1), ascending, with the classes of lines they apply to
  // (bit 0: start level <= l, bit 1: start level > l)
  double jq[kMaxJumps];
  int32_t jmask[kMaxJumps];
  // line-major band pass: usable when every jump exceeds (ns - 1) r_(l+1) + 2 (no
  // stencil hull around a line centre can hold one) and rho is 2 or 4;
  // lc_eps widens the centre estimate past single-precision rounding of d
  int32_t lc_ok, pad_lc;
  double lc_eps;
  // jumps farther apart than two stencil hulls: a hull holds at most one,
  // so the smallest straddled jump is the one straddled
  int32_t jumps_isolated, pad_ji;
  // chi over the evaluation points around jump k (|d| within q +- (3 r1 + 4)):
  // jchi_mode 0 = 1, 1 = exp2(jchi_c0 + jchi_c1 |d|) (fine units), 2 = any piece
  int32_t jchi_mode[kMaxJumps];
  int32_t pad_jc;
  double jchi_c0[kMaxJumps], jchi_c1[kMaxJumps];
};

// One work item of the level kernel: `count` consecutive nodes of one level,
// processed by one workgroup in wavefront tiles.
struct Tile {
  int32_t level;
  int32_t count;
  int64_t first;   // first node, relative to lo[level]
};

// Compacted line record of one layer (single precision path).
struct LineRec32 {
  int32_t k0;     // floor(nu~0 * 2048)
  float frac;     // nu~0 * 2048 - k0, in [0, 1)
  float A;        // S'/pi gamma_L with S' = S(T)/max S(T) (Voigt, Lorentz); S' (Doppler)
  float gam;      // gamma_L [cm^-1]
  float amp;      // S' sqrt(ln 2) / (sqrt(pi) alpha_D): scale of K(x, y) in the core (0 without Doppler width)
  float ae;       // alpha_D^2 / (2 ln 2); the core branch holds for d^2 + gamma_L^2 < 72 ae
  float xs;       // sqrt(ln 2) / alpha_D, 0 when alpha_D = 0
  int32_t s;      // start level
};

struct LineRec64 {
  int32_t k0;
  int32_t s;
  double frac, A, gam, gam2, ae, xs;
  double amp;     // as LineRec32 (64-byte records)
};
static_assert(sizeof(LineRec32) == 32, "LineRec32 is two 16-byte words");
static_assert(sizeof(LineRec64) == 64, "LineRec64 is four 16-byte words");

// Device-side workspace of a plan.
struct DeviceBuffers {
  // line list sorted by nu0
  double* nu0 = nullptr;
  float* S296 = nullptr;
  float* gair = nullptr;
  float* gself = nullptr;
  float* El = nullptr;
  float* nair = nullptr;
  float* dair = nullptr;
  double* layers = nullptr;        // [n_layers][4] p, T, p_self, q_ratio
  double* lconst = nullptr;        // [n_layers][8] per-layer constants of the line preparation
  unsigned long long* smax = nullptr;  // [n_layers] bits of max S(T) (FP64)
  int32_t* bcount = nullptr;       // [n_layers][n_blocks] kept lines per block -> offsets
  int32_t* scount = nullptr;       // [n_layers][n_blocks][12] lines per start level (12 = dropped)
  int32_t* kept = nullptr;         // [n_layers] kept lines
  int32_t* gcount = nullptr;       // [n_layers][12] lines per start level
  void* rec = nullptr;             // [n_layers][n_lines] LineRec32/64, kept lines in nu0 order
  double* cnu = nullptr;           // [n_layers][n_lines] shifted centre of the kept lines
  void* csp = nullptr;             // [n_layers][n_lines] S(T)/max S(T) of the kept lines (FP32/FP64)
  int32_t* bucket = nullptr;       // [n_layers][nbucket+1] first kept line with nu~0 >= origin + b/kBucketPerCm
  void* A = nullptr;               // [n_layers][a_total] level arrays 1..10
  IntervalSet* ivs = nullptr;      // [11][8]
  Tile* tiles = nullptr;           // [n_tiles] heaviest first
  Tile* stiles = nullptr;          // the learned shape's work items (smaller, so two workgroups fit a CU's LDS)
  unsigned int* counter = nullptr; // work-queue counter
  double* scale = nullptr;         // [n_layers] output scale
  double* span = nullptr;          // [n_layers] max |(delta_i - delta_j) p| [cm^-1]
  int32_t* perm = nullptr;         // [n_layers][n_lines] line indices in order of shifted centre
  unsigned long long* stats = nullptr;  // counters for marfa_plan_count
};

// Raw (sorted) line list as seen by the preparation kernels.
struct LineIn {
  const double* nu0;
  const float *S296, *gair, *gself, *El, *nair, *dair;
  double molar_mass;
  int64_t n;
};

// Arguments of the level-accumulation kernel.
struct LevelArgs {
  const Tile* tiles;
  int64_t n_tiles;       // work items per layer
  int32_t n_layers;
  unsigned int* counter; // work-queue counter (cleared before each launch)
  const void* rec;       // [layer][line] LineRec32/64
  const void* csp;       // [layer][line] S(T)/max S(T)
  const int32_t* bucket; // [layer][nbucket+1]
  const int32_t* gcount; // [layer][12]
  const IntervalSet* ivs;
  int64_t n_lines;
  void* A;               // [layer][a_total]
  void* out;             // [layer][stride]
  int64_t stride;
  unsigned long long* stats;  // counting mode only
  int32_t max_item;      // largest work item (nodes), sizes the LDS accumulator
  // learned line shape (single-precision Voigt plans with a surrogate)
  int32_t surr;
  float mlp_xmax;        // pairs with |x| above it use the plain shape
  float mlp_inv_c;       // 1 / cut-off [cm]
  MlpDev mlp;
  float* sq;             // the wavefront's queue of learned-shape pairs (LDS; set inside the kernel)
};

// the coefficient tables of a device prepared by marfa_use_device (device memory)
const DeviceTables* device_tables(int device);
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
void launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s);
struct PrepArgs {
  const int32_t* perm;   // [layer][line] order of shifted centres
  unsigned long long* smax;
  int32_t *bcount, *scount, *kept, *gcount, *bucket;
  void* rec;
  double* cnu;
  void* csp;
  double* scale;
  double* lc;   // [layer][8] per-layer constants, written by the preparation's first kernel
  double prune, R;
  int32_t out_kind, fp64;
};
void launch_prep(const LineIn& in, const double* layers, int nL, const Geometry& G, const PrepArgs& pa,
                 hipStream_t s);
void launch_level(const Geometry& G, const LevelArgs& a, int grid, bool fp64, bool count, hipStream_t s);
// training samples of the learned line shape (ranges of the lines and layers it serves)
struct MlpSampleCfg {
  double nu_lo, nu_hi;     // line centres [cm^-1]
  double T_lo, T_hi;       // temperatures [K]
  double molar_mass;       // [g/mol]
  double y_lo, y_hi;       // Voigt y range
  double cutoff;           // [cm^-1]
  int32_t chi, pad;
};
void launch_mlp_samples(const MlpSampleCfg& c, uint64_t seed, int64_t n, float* X, float* T,
                        const DeviceTables* tabs, hipStream_t s);
// error text of the calling thread, and device set-up (Weideman tables)
marfa_status marfa_set_error(marfa_status st, const char* msg);
marfa_status marfa_use_device(int device);
void launch_rank(const LineIn& in, const double* layers, int nL, const double* span, int32_t* perm, hipStream_t s);
void launch_cascade(const Geometry& G, int nL, void* A, void* out, int64_t stride, const double* scale, bool fp64,
                    hipStream_t s);
void launch_voigt_eval(int64_t n, const double* x, const double* y, double* out, bool fp64,
                       const DeviceTables* tabs, hipStream_t s);

}  // namespace marfa
