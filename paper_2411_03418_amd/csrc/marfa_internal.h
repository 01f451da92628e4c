// marfa_internal.h -- shared between the host runtime and the HIP kernels of
// the eleven-grid library (not installed; the public ABI is include/marfa.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "marfa.h"

namespace marfa {

constexpr int kLevels = 11;      // Section 2.4: eleven grids
constexpr int kGroups = 11;      // lines grouped by start level 0..10
constexpr int kMaxIntervals = 6; // disjoint |d| intervals per (level, start level)
constexpr int kMaxJumps = 5;     // jump points of T_(l+1) per (level, start level)
constexpr int kWave = 64;        // CDNA wavefront
constexpr int kWeidemanN32 = 32; // rational-series length, single-precision path
constexpr int kWeidemanN64 = 48; // rational-series length, double-precision path

// Lattice geometry, identical for every layer.  Positions are in units of the
// finest step h0 = 2^-11 cm^-1 ("fine units"); node m of level l sits at
// X = m * r[l].
struct Geometry {
  int32_t r[kLevels];        // level step in fine units
  int64_t lo[kLevels];       // first node index of each level (incl. halo)
  int64_t n[kLevels];        // nodes per level
  int64_t aoff[kLevels];     // offset of level l >= 1 in a layer's level array
  int64_t a_total;           // level-array length per layer (levels 1..10)
  double b[kLevels];         // region boundary b_l = R r_(l+1), fine units (l < 10)
  double B[kLevels];         // band half-width 2 r_(l+1), fine units (l < 10)
  double c_fine;             // cut-off in fine units
  int32_t shape, chi, out_kind, fp64;
};

// For one (level l, start level s): the |d| intervals (fine units, closed)
// that can hold a non-zero contribution, and the jump points of T_(l+1).
struct IntervalSet {
  int32_t n_iv;
  int32_t n_q;
  double a[kMaxIntervals], b[kMaxIntervals];
  double q[kMaxJumps];
};

// One work item of the level kernel: `count` consecutive nodes of one level,
// processed by one workgroup in wavefront-sized sub-tiles.
struct Tile {
  int32_t level;
  int32_t count;
  int64_t first;   // first node, relative to lo[level]
};

// Compacted line record of one layer (single precision path).
struct LineRec32 {
  int32_t k0;     // floor(nu~0 * 2048)
  float frac;     // nu~0 * 2048 - k0, in [0, 1)
  float Sp;       // S(T) / max S(T) of the layer
  float gam;      // gamma_L [cm^-1]
  float gam2;     // gamma_L^2
  float ae;       // alpha_D^2 / (2 ln 2)
  float xs;       // sqrt(ln 2) / alpha_D, 0 when alpha_D = 0
  float aD;       // alpha_D [cm^-1]
};

struct LineRec64 {
  int32_t k0;
  int32_t pad;
  double frac, Sp, gam, gam2, ae, xs, aD;
};

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
  unsigned long long* smax = nullptr;  // [n_layers] bits of max S(T) (FP64)
  int32_t* bcount = nullptr;       // [n_layers][n_blocks][12]
  int32_t* gcount = nullptr;       // [n_layers][12]
  int32_t* gstart = nullptr;       // [n_layers][12]
  void* rec = nullptr;             // [n_layers][n_lines] LineRec32/64
  double* cnu = nullptr;           // [n_layers][n_lines] nu0 of compacted lines
  void* A = nullptr;               // [n_layers][a_total] level arrays 1..10
  IntervalSet* ivs = nullptr;      // [11][11]
  Tile* tiles = nullptr;           // [n_tiles] sorted heaviest first
  unsigned int* counter = nullptr; // work-queue counter
  double* scale = nullptr;         // [n_layers] output scale
  double* shift = nullptr;         // [n_layers][2] nu0 - nu~0 range [cm^-1]
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
  const double* cnu;     // [layer][line] nu0 of the compacted lines
  const int32_t* gcount; // [layer][12]
  const int32_t* gstart; // [layer][12]
  const IntervalSet* ivs;
  const double* shift;   // [layer][2] range of nu~0 - nu0 [cm^-1]
  int64_t n_lines;
  void* A;               // [layer][a_total]
  void* out;             // [layer][stride]
  int64_t stride;
  unsigned long long* stats;  // counting mode only
};

hipError_t upload_weideman(const double* a32, const double* a64, const double* L2);
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
void launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s);
void launch_prep(const LineIn& in, const double* layers, int nL, unsigned long long* smax, double prune, double R,
                 const Geometry& G, int32_t* bcount, int32_t* gcount, int32_t* gstart, void* rec, double* cnu,
                 double* scale, int out_kind, bool fp64, hipStream_t s);
void launch_level(const Geometry& G, const LevelArgs& a, int grid, bool fp64, bool count, hipStream_t s);
void launch_cascade(const Geometry& G, int nL, void* A, void* out, int64_t stride, const double* scale, bool fp64,
                    hipStream_t s);
void launch_voigt_eval(int64_t n, const double* x, const double* y, double* out, bool fp64, hipStream_t s);

}  // namespace marfa
