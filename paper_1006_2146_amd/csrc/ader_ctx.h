// Host-side context shared by the library's translation units: the device
// buffers, the problem table of a batch, the launch configuration and the
// stage functions of each (system, precision, order, form) variant.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/ader.h"
#include "recon_tile.h"
#include "zone_ops.h"

namespace ader {

// One periodic mesh of a batch, as the kernels see it.  Its zones sit at
// indices base .. base+N-1 of every batch array (stride S = all zones).
struct Problem {
  int nx, ny, nz, pad;
  long long N, base;
  double dx, dy, dz;
  // non-periodic faces: ghost layers before the interior along each axis
  // (0 on periodic axes; nx, ny, nz then count them), the interior size,
  // and the kinds of the faces x-, x+, y-, y+, z-, z+ (ADER_BC_*)
  int gx, gy, gz, ux, uy, uz;
  int bc[6];
};

// ghost layers on each non-periodic face (enough for order 4)
constexpr int kGhost = 4;

// the states of the six faces' inflow (conserved, [face][v]; faces x-, x+,
// y-, y+, z-, z+), passed to the ghost fill by value
struct InflowStates {
  double v[6][5];
};

// the fused face-flux+update kernel: x-y tiles of kFuTX x kFuTY zones, a
// work item walks kFuSeg planes of one tile in z
constexpr int kFuTX = 32, kFuTY = 8, kFuSeg = 16;

// zone (i, j, k) of a padded problem is a ghost zone (diagnostics sum the
// interior only)
__host__ __device__ inline bool ghost_zone(const Problem& pr, int i, int j, int k) {
  return (pr.gx && (i < pr.gx || i >= pr.gx + pr.ux)) ||
         (pr.gy && (j < pr.gy || j >= pr.gy + pr.uy)) ||
         (pr.gz && (k < pr.gz || k >= pr.gz + pr.uz));
}

// Kernel argument: the device problem table and the array stride.
struct Batch {
  const Problem* P;
  int np;
  long long S;
};

// Launch shape of one kernel class: threads per block and the number of
// persistent blocks per compute unit.
struct LaunchShape {
  int block;
  int blocks_per_cu;
};

enum { kClassDt = 0, kClassRecon = 1, kClassPredict = 2, kClassFlux = 3, kClassUpdate = 4,
       kNumClasses = 5 };

// Diagnostics: zones per reduction tile, and values per partial row (five
// hydro sums, three face-field sums, the largest |div B|).
constexpr long long kDiagTile = 8192;
constexpr int kDiagVals = 9;

}  // namespace ader

struct ader_ctx;

namespace ader {

// The stages of one step for one variant, each one persistent launch over
// every problem of the context (reconstruction: one per sweep).
struct StageFns {
  int (*recon)(ader_ctx*);
  int (*predict)(ader_ctx*);
  int (*predict_split)(ader_ctx*);    // lane-split layout, nullptr if not built
  int (*predict_split2)(ader_ctx*);   // the same, registers capped for 2 waves/SIMD
  int (*predict_zone2)(ader_ctx*);    // one lane per zone, facial check in its own pass
  int (*predict_zone_2w)(ader_ctx*);  // one lane per zone, registers capped for 2 waves/SIMD
  int (*predict_pair)(ader_ctx*);     // MHD: two lanes per zone
  int (*predict_pair2)(ader_ctx*);    // the same, registers capped for 2 waves/SIMD
  int (*predict_pair_split)(ader_ctx*);  // the same in two kernels (predictor, sides)
  int (*predict_fused)(ader_ctx*);  // reconstruction and predictor in one kernel (Euler, order 3)
  int (*rk_sides)(ader_ctx*);         // SSP-RK stage: side packets (Euler, modal tables)
  int (*flux)(ader_ctx*);     // face (and, MHD, edge) fluxes
  int (*update)(ader_ctx*);   // eq. (6), and eq. (8) for MHD
  int (*predict_src)(ader_ctx*);   // Euler with the affine source (one lane per zone)
  int (*update_src)(ader_ctx*);    // eq. (6) with the source term
};

}  // namespace ader

struct ader_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 256;
  // problems: host copy and device table
  std::vector<ader::Problem> probs;
  ader::Problem* d_probs = nullptr;
  long long S = 0;                 // total zones (array stride)
  // non-periodic faces (ader_set_boundary): some problem has ghost zones;
  // the caller's arrays hold the interiors only, S_user zones in all
  bool bounded = false;
  // inflow faces' states (ader_set_inflow); bit f of inflow_set: face f given
  ader::InflowStates inflow{};
  unsigned inflow_set = 0;
  unsigned long long inflow_version = 0;   // bumped on every ader_set_inflow
  long long S_user = 0;
  double gamma = 1.4;
  int system = ADER_EULER;
  int order = 3, form = ADER_MODAL, riemann = ADER_HLL, precision = ADER_FP64;
  double* U = nullptr;
  bool owns_U = true;
  void* W = nullptr;
  void* PK = nullptr;
  double* F = nullptr;
  // MHD: face fields, zone field b_0, its modes, the Sec. III normal moments,
  // face-edge fluxes and edge fields
  double* B = nullptr;
  bool owns_B = true;
  double* B0 = nullptr;
  void* WB = nullptr;
  void* BN = nullptr;
  double* FE = nullptr;
  double* E = nullptr;
  // per problem: dt, the CFL rate as the bit pattern of a non-negative
  // double (atomic max), and the status flag of the dt evaluations
  double* d_dt = nullptr;
  unsigned long long* d_rate = nullptr;
  int* d_bad = nullptr;
  bool have_state = false;
  std::vector<char> set_flags;     // problems given a state by ader_batch_set_state
  bool have_dt = false;
  size_t bytes = 0;          // device bytes held: fixed part plus work arrays
  size_t fixed_bytes = 0;
  size_t work_bytes[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // W, PK, WB, BN, RK, EM, TH, SB as allocated
  // MHD pair layout in two kernels: evolutionary modes [NE][8][S] in the
  // bulk type and the two positivity scaling factors [2][S]
  void* EM = nullptr;
  double* TH = nullptr;
  // time stepping (ADER_SCHEME_*); SSP-RK keeps four extra states in RK:
  // the step's starting state, the stage states 2 and 3 and dt L(U^(3))
  int scheme = ADER_SCHEME_ADER;
  double* RK = nullptr;
  ader::LaunchShape shape[ader::kNumClasses] = {{256, 8}, {256, 8}, {128, 4}, {256, 8}, {256, 8}};
  // predictor layout: -1 the variant's default, else an ADER_LAYOUT_*
  int layout = -1;
  // reconstruction: -1 default, else an ADER_RECON_*; tiles of kTile^3
  // zones, problem p's tiles at tile_base[p] .. tile_base[p+1]-1
  int recon_mode = -1;
  long long* d_tile_base = nullptr;
  long long ntiles = 0;
  // tiles of kTile x kTile x kFusedTZ zones of the fused reconstruction+predictor
  long long* d_ftile_base = nullptr;
  long long nftiles = 0;
  // column segments (kMarchTile^2 zones x kMarchSeg planes) of the z-marching
  // reconstruction
  long long* d_xytile_base = nullptr;
  long long nxytiles = 0;
  // face fluxes and update in one kernel (ADER_FLUX_*; -1 the default, the
  // two kernels); its work items, kFuTX x kFuTY columns of kFuSeg planes
  int flux_mode = -1;
  long long* d_fu_base = nullptr;
  long long nfutiles = 0;
  // z-column segments of the column mode: problem p's at seg_base[p] ..
  long long* d_seg_base = nullptr;
  long long nsegs = 0;
  // stage timing: events recorded around each stage while enabled
  bool timing = false;
  std::vector<hipEvent_t> events;
  std::vector<int> marks;  // stage of each (start, stop) event pair
  // hipGraph of one CFL step, rebuilt when the configuration changes
  bool use_graph = false;
  hipGraphExec_t graph_exec = nullptr;
  double graph_cfl = 0.0;
  unsigned long long graph_key = 0;

  // positivity (ADER_POSITIVITY_*): the check of the paper's scheme or the
  // scaling; per problem the count of scaled zone polynomials
  int positivity = ADER_POSITIVITY_CHECK;
  unsigned int* d_limited = nullptr;
  // velocity of the linear-advection test system
  double adv[3] = {1.0, 0.0, 0.0};
  // affine source term (Euler): S(u) = A u + b, and dt S-bar per zone [5][S]
  bool has_source = false;
  ader::SourceAffine source{};
  unsigned long long source_version = 0;   // bumped on every ader_set_source
  double* SB = nullptr;
  // diagnostics: problem p's reduction tiles at diag_base[p] ..
  // diag_base[p+1]-1, and the partial rows and results (allocated on first
  // use)
  long long* d_diag_base = nullptr;
  long long ndiag_tiles = 0;
  double* d_diag = nullptr;

  ader::Batch batch() const { return ader::Batch{d_probs, (int)probs.size(), S}; }
  // flags and counts of problem p at [p], sink slots of its deep ghost
  // zones at [np + p]
  ader::PosCtl pos() const {
    return ader::PosCtl{positivity == ADER_POSITIVITY_LIMIT ? 1 : 0, d_bad, d_limited, np()};
  }
  int np() const { return (int)probs.size(); }
  // the fused face-flux+update kernel runs the ADER step of Euler without a
  // source term when set; elsewhere the two kernels do
  bool flux_fused() const {
    return flux_mode == ADER_FLUX_FUSED && system == ADER_EULER && !has_source &&
           scheme == ADER_SCHEME_ADER;
  }
  // where the predictor keeps the zone averages for that kernel (the first
  // five rows of F, which it does not use), nullptr when not needed: only
  // the deviation-form packets (mixed precision) need them
  double* keep_avg() const {
    return flux_fused() && precision == ADER_MIXED ? F : nullptr;
  }
};

namespace ader {

inline int check(hipError_t e) { return e == hipSuccess ? ADER_OK : ADER_EDEVICE; }
inline int launched() { return check(hipGetLastError()); }

#define ADER_TRY(expr)              \
  do {                              \
    int _rc = (expr);               \
    if (_rc != ADER_OK) return _rc; \
  } while (0)

// Persistent grid of a kernel class: blocks_per_cu blocks per compute unit,
// and never more blocks than the zones need (zones_per_wave zones per 64
// lanes: 64 for one zone per lane, 64 / NV in the lane-split layout).
inline unsigned grid_for(const ader_ctx* c, int cls, int zones_per_wave = 64) {
  const LaunchShape& s = c->shape[cls];
  const long long per_block = (long long)zones_per_wave * (s.block / 64);
  const long long need = (c->S + per_block - 1) / per_block;
  const long long cap = (long long)s.blocks_per_cu * c->num_cus;
  const long long g = need < cap ? need : cap;
  return (unsigned)(g < 1 ? 1 : g);
}

// Stage tables of the variants, one translation unit each.
#define ADER_VARIANTS(X)                                                                  \
  X(euler, fp64, 2, 0) X(euler, fp64, 2, 1) X(euler, fp64, 3, 0) X(euler, fp64, 3, 1)     \
  X(euler, fp64, 4, 0) X(euler, fp64, 4, 1)                                              \
  X(euler, mixed, 2, 0) X(euler, mixed, 2, 1) X(euler, mixed, 3, 0) X(euler, mixed, 3, 1) \
  X(euler, mixed, 4, 0) X(euler, mixed, 4, 1)                                             \
  X(mhd, fp64, 2, 0) X(mhd, fp64, 2, 1) X(mhd, fp64, 3, 0) X(mhd, fp64, 3, 1)             \
  X(mhd, fp64, 4, 0) X(mhd, fp64, 4, 1)                                                   \
  X(mhd, mixed, 2, 0) X(mhd, mixed, 2, 1) X(mhd, mixed, 3, 0) X(mhd, mixed, 3, 1)         \
  X(mhd, mixed, 4, 0) X(mhd, mixed, 4, 1)                                                 \
  X(linadv, fp64, 2, 0) X(linadv, fp64, 2, 1) X(linadv, fp64, 3, 0) X(linadv, fp64, 3, 1) \
  X(linadv, fp64, 4, 0) X(linadv, fp64, 4, 1)
#define ADER_STAGES_NAME(sys, prec, order, form) stages_##sys##_##prec##_o##order##_f##form
#define ADER_DECLARE_STAGES(sys, prec, order, form) \
  const StageFns* ADER_STAGES_NAME(sys, prec, order, form)();
ADER_VARIANTS(ADER_DECLARE_STAGES)
#undef ADER_DECLARE_STAGES

}  // namespace ader
