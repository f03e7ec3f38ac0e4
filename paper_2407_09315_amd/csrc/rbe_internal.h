// Internal types shared by the host plan code and the gfx950 kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <hip/hip_runtime.h>

#include "rbe.h"

namespace rbe {

// Per-system metadata, one 64-byte row per system in the workspace.
struct SysDesc {
  int64_t n_off;      // first particle of the system in the concatenated arrays
  int64_t k_off;      // first wave vector
  int64_t part_off;   // first partial-sum slot (complex) of the system's [p][ntiles] block
  int64_t cache_off;  // first (cos, sin) slot of the system's [p][n] phase cache
  int32_t n;          // particles
  int32_t p;          // wave vectors
  int32_t ntiles;     // rho-pass particle tiles
  int32_t cdf_len;    // 2M+1 entries of the sampler's prefix-sum table (0: no table)
  double L;
  double alpha;       // Ewald splitting parameter (virial)
};
static_assert(sizeof(SysDesc) == 64, "SysDesc layout");

// Reduction descriptor of one wave vector: its tile partials are slots
// slot .. slot + ntiles - 1 (complex) of the partial-sum region; sys is its system.
struct KRed {
  int64_t slot;
  int32_t ntiles;
  int32_t sys;
};

// Force-pass row of one wave vector in the FP32 forms (64 bytes, four 16-byte quarters),
// written once per evaluation from the reduced rho; every force block copies the two
// quarters its form reads into LDS.  With rho'_l = C'_l + i S'_l the structure factor rotated
// onto the form's phases, R_l = c_l |rho'_l| and delta_l = 1/4 - arg(rho'_l) / (2 pi) turns,
//   c_l (S'_l cos theta - C'_l sin theta) = R_l cos(theta + 2 pi delta_l),
// so a recomputed term needs one cosine of the phase shifted by delta_l.
struct ForceRowF32 {
  uint32_t d;           // quarter 0: delta_l as a 32-bit fixed-point fraction of a turn and
  int32_t mx, my, mz;   //   m_l; quarter 1: R_l m_l (fixed-point phases, 28 bytes read)
  float gx, gy, gz;
  float pad0;
  float fx, fy, fz;     // quarter 2: m_l as float, delta_l in turns in [0, 1); quarter 3: R_l m_l
  float dt;             //   and R_l (FP32 phases; the phase-cache pass forms c_l S'_l and
  float hx, hy, hz;     //   c_l C'_l from them)
  float r;
};
static_assert(sizeof(ForceRowF32) == 64, "ForceRowF32 layout");

// Sampler table of system b: cdf[b * stride ...] = S, 2M+1, p, k_off, then the Metropolis
// chain's proposal half-width D and beta = pi^2 / (alpha L^2) (as doubles), then the 2M+1
// prefix sums (zero-padded to the stride), so a table's address needs no other lookup.
constexpr int kCdfHeader = 6;

// rho-pass work item: one particle tile x one range of wave vectors.
struct RhoItem {
  int32_t sys;
  int32_t tile;
  int32_t k0;   // first local wave vector
  int32_t nk;   // number of wave vectors
};

// force-pass work item: a contiguous particle range of one system.
struct ForceItem {
  int32_t sys;
  int32_t p0;     // first local particle
  int32_t np;     // particles
  int32_t flags;  // bit 0: this block writes the system's energy
};

// Kernel variant tables (the autotuner picks one entry of each).
// rho: particles per lane, wave vectors per chunk, at most krange wave vectors per work item
// (a system's wave vectors are cut into ranges of whole chunks whose counts differ by <= 1),
// waves per block: 4 (one item per wave), 16 (one block per CU sharing single-chunk
// items through LDS; krange is then one chunk) or 1 for the k-lane layout (one item per
// 256-thread block, wave vectors across the lanes; "wave vectors per chunk" is then the
// wave vectors per lane)
// tile: particles per tile; comp: compensated FP32 sums in the forward k-lane pass
struct RhoVariant { int npl; int kc; int krange; int wpb; int tile; int comp; };
struct ForceVariant { int nplf; };                       // particles per lane (256-thread blocks)

constexpr int kNumRhoVariantsF32 = 13;
constexpr int kNumRhoVariantsF64 = 10;
constexpr int kNumForceVariants = 3;
extern const RhoVariant kRhoVariantsF32[kNumRhoVariantsF32];
extern const RhoVariant kRhoVariantsF64[kNumRhoVariantsF64];
extern const ForceVariant kForceVariants[kNumForceVariants];

constexpr int kForceBlock = 256;
constexpr int kReduceBlock = 256;
constexpr int kMaxAttempts = 1024;

// Device-side views of the workspace regions.
struct WsView {
  const SysDesc* sys;
  const RhoItem* rho_items;
  const ForceItem* force_items;
  const KRed* kred;      // reduction descriptor of each wave vector
  const double* cdf;     // sampler tables, one per system at a fixed stride
  double* partials;      // complex partial sums (rho pass, then VJP pass B1)
  double* xy;            // P_total complex values (VJP X + iY)
  float* cache;          // (cos, sin) phase cache, FP32_MIXED + CACHED only
  ForceRowF32* frows;    // P_total force-pass rows (FP32 forms)
};

struct LaunchShape {
  int32_t B;
  int64_t n_total;
  int64_t p_total;
  int32_t n_rho_items;
  int32_t n_force_items;
  int precision;
  int cached;
  RhoVariant rv;
  int rho_variant;
  ForceVariant fv;
  int force_variant;
  int32_t cdf_stride;    // doubles per system in the sampler-table region
  int32_t sampler;       // RBE_SAMPLER_EXACT or RBE_SAMPLER_METROPOLIS
  int32_t burn_in;       // Metropolis steps per chain
  int32_t rho_grid_cap;  // persistent-grid caps (0: one block per work item)
  int32_t rho_clamp;     // 1: cap the rho-pass blocks per CU at their even share
  int32_t force_grid_cap;
  SysDesc sys0;          // the system when B == 1 (then work items follow from the block index)
  // optional events recorded right before / after the rho-pass and force-pass kernels
  hipEvent_t ev_rho_begin, ev_rho_end, ev_force_begin, ev_force_end;
};

// Error reporting shared by the library's entry points (rbe_host.cpp): fail() records the
// message returned by rbe_last_error() and returns st; hip_fail() wraps a HIP error;
// device_ok() reports RBE_ENODEV when no device is present.
rbe_status fail(rbe_status st, const char* fmt, ...);
rbe_status hip_fail(hipError_t e, const char* what);
rbe_status device_ok();

// Kernel launchers (rbe_kernels.hip).  Each returns hipSuccess or the launch error.
// launch_rho with rows != 0 (FP32 forms) also writes the force rows from the reduced rho (wk:
// the weights); launch_force with rows_ready != 0 uses them, otherwise it writes them from
// rho first.
hipError_t launch_rho(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const double* wk, double* rho,
                      int rows, hipStream_t st);
hipError_t launch_force(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                        const double* z, const double* q, const int32_t* m, const double* wk,
                        const double* rho, void* F, double* U, uint64_t* counter, int rows_ready,
                        hipStream_t st);
hipError_t launch_vjp(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const double* wk,
                      const double* rho, const double* gU, const void* gF, double* gr, double* gq,
                      hipStream_t st);
hipError_t launch_sample(const LaunchShape& s, const WsView& w, uint64_t seed, uint64_t stream_id,
                         const uint64_t* counter, int32_t* m, double* wk, hipStream_t st);
hipError_t launch_virial(const LaunchShape& s, const WsView& w, const int32_t* m, const double* wk,
                         const double* rho, double* W, hipStream_t st);

}  // namespace rbe
