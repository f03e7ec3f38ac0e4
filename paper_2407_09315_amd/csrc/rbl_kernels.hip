// Random batch list (RBL) short-range force on gfx950 (Sec. 2.3; Algorithm 2): a cell list
// built on the device, the exact core sum and the systematic shell batch per particle, and
// the momentum correction.  FP64 throughout.
//
// One evaluation:
//   cells   : cell of every particle, per-cell counts (atomic adds), exclusive scan into
//             cell starts, scatter into cell order (at the ranks the count atomics gave),
//             then every cell's short segment sorted by particle index, so the order is
//             deterministic;
//   gather  : positions, charges and LJ parameters read in particle order and written into
//             cell order, and every particle's batch offset u_i drawn;
//   select  : one wave per cell classifies the cell's stencil against its particles (FP32
//             distances from fixed-point coordinates, FP64 inside a band around the
//             cutoffs) and writes every particle's pairs -- the core and the batch -- into
//             a slot of Q entries;
//   pairs   : one lane per particle adds its slot's pair forces in order;
//   fallback: particles whose stencil or pair count exceeds what the selection holds are
//             done one wave each, classifying the stencil window by window;
//   correct : two fixed-order summations of the forces; every force gets -(1/N) of the
//             total.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "philox.h"
#include "rbe_internal.h"
#include "rbl.h"

namespace rbe {
namespace {

constexpr int kRblBlock = 256;
constexpr int kScanChunk = kRblBlock * 8;   // cells per block of the scan
constexpr size_t kRblAlign = 256;
constexpr double kRblPi = 3.14159265358979323846264338327950288;

size_t rbl_align(size_t v) { return (v + kRblAlign - 1) / kRblAlign * kRblAlign; }

struct RblGrid {
  int32_t nc;     // cells per axis
  int32_t R;      // stencil reach in cells
  int32_t span;   // stencil cells per axis: 2R + 1, or nc when that would wrap
  int32_t wrap;   // 1 when the stencil covers every cell of an axis
  float inv_span;       // 1 / span
  double inv_nc, inv_nc2;   // 1 / nc, 1 / nc^2
};

// One particle in cell order: position and charge, sqrt(eps) and sigma, and its batch offset
// u_i; 56 bytes padded to 64, so that a pair's data is one cache-line half.
struct alignas(64) RblRec {
  double4 pq;
  double2 lj;
  double u;
};
static_assert(sizeof(RblRec) == 64, "RblRec is 64 bytes");

struct RblWs {
  int32_t* count;
  int32_t* rank;     // N, by particle index: its arrival in its cell's count (counting atomics)
  int32_t* start;    // ncell + 1
  int32_t* bsum;     // scan block sums
  int32_t* cell;     // N, by particle index: the cell, then (after the sort) the cell-order position
  int32_t* idx;      // N: particle index at each cell-order position
  RblRec* rec;       // N, in cell order
  uint4* fxa;        // N, in cell order: the position in 32-bit fixed point, frac(x / L) 2^32 (a
                     // wrapping difference is the minimum image), read by the selection
  int2* range;       // ncell: first and one-past-last cell-order position of each cell
  uint32_t* slot;    // Q pair entries per particle, interleaved (slot_index)
  int32_t* cnt;      // N, in cell order: pairs in the slot, -1 for the fallback
  int32_t* tns;      // N, in cell order: N_s
  int32_t* fb;       // N: cell-order positions left to the fallback
  int32_t* nfb;      // 1: their count
  double* partial;   // 3 per block of the first summation
  double* corr;      // 3
  double* etab;      // erfcx table: kErfcCoef Taylor coefficients per interval (erfcx_table)
};

// Cell coordinate of a position along one axis: min(floor(frac(x / L) nc), nc - 1).  A
// non-finite coordinate gets cell 0 (its forces come out NaN and spread to every particle
// through the momentum correction).
__device__ inline int32_t cell_coord(double x, double L, int32_t nc) {
  const double s = x / L;
  double f = s - floor(s);
  if (!(f >= 0.0 && f < 1.0)) f = 0.0;
  const int32_t c = (int32_t)floor(f * (double)nc);
  return c < nc - 1 ? c : nc - 1;
}

// erfc(x) = exp(-x^2) erfcx(x), with erfcx tabulated on [0, x_tab] as degree-9 Taylor
// polynomials around the centres of intervals of width x_tab / eni <= 0.1
constexpr int kErfcDeg = 9;
constexpr int kErfcCoef = kErfcDeg + 1;
constexpr int kErfcMaxIntervals = 256;
constexpr double kErfcMaxX = 25.6;          // erfc(25.6) = 2e-287: zero beyond, to the force

// Interval k of the erfcx table: erfcx(x_k + t h / 2) = sum_j c_j t^j, t in [-1, 1], around the
// centre x_k = (k + 1/2) h, with c_j = erfcx^(j)(x_k) (h / 2)^j / j!.  The derivatives follow
// from erfcx' = 2 x erfcx - 2 / sqrt(pi), differentiated n times:
// erfcx^(n+1) = 2 x erfcx^(n) + 2 n erfcx^(n-1).  (An error in erfcx(x_k) grows along the
// recurrence as (2 x_k)^n and reaches c_n times (x_k h)^n / n!: at most e^(x_k h) < 13 in all
// for x_k <= 25.6 and h <= 0.1, and near 1 for the x_k h < 0.3 of typical cutoffs.)
__device__ inline void erfcx_interval(double* __restrict__ c, int32_t k, double h) {
  const double xc = ((double)k + 0.5) * h, hw = 0.5 * h;
  double d0 = erfc(xc) * exp(xc * xc);
  double d1 = 2.0 * xc * d0 - 1.1283791670955125739;   // 2 / sqrt(pi)
  c[0] = d0;
  double f = hw;
  c[1] = d1 * f;
  for (int j = 1; j < kErfcDeg; ++j) {
    const double d2 = 2.0 * xc * d1 + 2.0 * (double)j * d0;
    f *= hw / (double)(j + 1);
    c[j + 1] = d2 * f;
    d0 = d1;
    d1 = d2;
  }
}

// erfcx(x) for 0 <= x from the table: the last interval also takes x a rounding past its end,
// and x >= kErfcMaxX gives 0 (exp(-x^2) erfcx(x) < 1e-286 there).  A NaN x gives NaN.
__device__ inline double erfcx_table(const double* __restrict__ tab, int32_t ni, double inv, double x) {
  if (x >= kErfcMaxX) return 0.0;
  const double u = x * inv;
  const int32_t k = min(max((int32_t)u, 0), ni - 1);
  const double t = 2.0 * (u - (double)k) - 1.0;
  const double* c = tab + k * kErfcCoef;
  double p = c[kErfcDeg];
#pragma unroll
  for (int j = kErfcDeg - 1; j >= 0; --j) p = fma(p, t, c[j]);
  return p;
}

// Memory order of the cells: z runs are contiguous, and the nc^2 runs are laid out in tiles of
// 8 x 8 (x, y) runs, x-major over the tiles and within a tile, so that a contiguous range of
// cells (and of particles in cell order) is compact in space.  The rank of run (x, y):
// slabs of 8 x values before x hold 8 nc runs each, the tiles before y in x's slab hold
// 8 wx runs each (wx: the slab's width, 8 or less at the end), then x-major in the tile.
__host__ __device__ inline int32_t run_rank(int32_t x, int32_t y, int32_t nc) {
  const int32_t tx = x >> 3, ty = y >> 3;
  const int32_t wx = min(8, nc - (tx << 3)), wy = min(8, nc - (ty << 3));
  return (tx << 3) * nc + (ty << 3) * wx + (x & 7) * wy + (y & 7);
}

// The cell counts and the fallback counter to zero; the first eni threads also write the
// erfcx table (erfcx_interval, intervals of width h).
__global__ __launch_bounds__(kRblBlock) void rbl_zero_kernel(int32_t* __restrict__ count, int64_t n,
                                                             int32_t* __restrict__ nfb, double* __restrict__ etab,
                                                             int32_t eni, double h) {
  const int64_t i = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (i < n) count[i] = 0;
  if (i == 0) *nfb = 0;
  if (i < eni) erfcx_interval(etab + i * kErfcCoef, (int32_t)i, h);
}

__global__ __launch_bounds__(kRblBlock) void rbl_cell_kernel(const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             const double* __restrict__ z, int64_t n, double L,
                                                             int32_t nc, int32_t* __restrict__ cell,
                                                             int32_t* __restrict__ count, int32_t* __restrict__ rank) {
  const int64_t i = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t c = run_rank(cell_coord(x[i], L, nc), cell_coord(y[i], L, nc), nc) * nc + cell_coord(z[i], L, nc);
  cell[i] = c;
  rank[i] = atomicAdd(&count[c], 1);
}

// Inclusive scan of v over the 64 lanes (lane i gets the sum over lanes 0 .. i).
// Data-parallel-primitive moves: a scan within each row of 16 lanes (shifts right by 1, 2,
// 4, 8, an empty source giving 0), then lane 15's sum added into rows 1 and 3 and lane 31's
// into rows 2 and 3 (rows the mask leaves out add 0).
__device__ inline int32_t wave_scan(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return v;
}

// The sum of v over the 64 lanes, in every lane's hands.
__device__ inline int32_t wave_sum(int32_t v) { return __builtin_amdgcn_readlane(wave_scan(v), 63); }

// Exclusive scan of the cell counts in three launches: per-chunk totals, an in-order scan
// of the totals (one block), then each chunk rescanned with its offset.  Within a block:
// each wave's scan, then the wave totals through LDS.
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* sh, int32_t* total) {
  constexpr int kWaves = kRblBlock / 64;
  const int32_t lane = (int32_t)(threadIdx.x & 63), wv = (int32_t)(threadIdx.x >> 6);
  const int32_t incl = wave_scan(v);
  if (lane == 63) sh[wv] = incl;
  __syncthreads();
  int32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    const int32_t t = sh[k];
    off += k < wv ? t : 0;
    tot += t;
  }
  __syncthreads();   // sh is written again by the next call
  *total = tot;
  return off + incl - v;
}

__global__ __launch_bounds__(kRblBlock) void rbl_scan_sums_kernel(const int32_t* __restrict__ count, int64_t ncell,
                                                                  int32_t* __restrict__ bsum) {
  __shared__ int32_t sh[kRblBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int32_t s = 0;
  for (int k = 0; k < kScanChunk / kRblBlock; ++k) {
    const int64_t c = base + (int64_t)k * kRblBlock + threadIdx.x;
    if (c < ncell) s += count[c];
  }
  int32_t tot;
  (void)block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kRblBlock) void rbl_scan_offsets_kernel(int32_t* __restrict__ bsum, int32_t nb) {
  // one block: thread t scans a contiguous run of block totals, then the run totals
  __shared__ int32_t sh[kRblBlock];
  const int per = (nb + kRblBlock - 1) / kRblBlock;
  const int b0 = threadIdx.x * per;
  int32_t s = 0;
  for (int b = b0; b < min(b0 + per, nb); ++b) s += bsum[b];
  int32_t tot;
  int32_t off = block_exclusive_scan(s, sh, &tot);
  for (int b = b0; b < min(b0 + per, nb); ++b) {
    const int32_t v = bsum[b];
    bsum[b] = off;
    off += v;
  }
}

__global__ __launch_bounds__(kRblBlock) void rbl_scan_apply_kernel(const int32_t* __restrict__ count, int64_t ncell,
                                                                   const int32_t* __restrict__ bsum,
                                                                   int32_t* __restrict__ start, int2* __restrict__ range,
                                                                   int64_t n) {
  __shared__ int32_t sh[kRblBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int32_t off = bsum[blockIdx.x];
  for (int k = 0; k < kScanChunk / kRblBlock; ++k) {
    const int64_t c = base + (int64_t)k * kRblBlock + threadIdx.x;
    const int32_t v = c < ncell ? count[c] : 0;
    int32_t tot;
    const int32_t ex = block_exclusive_scan(v, sh, &tot);
    if (c < ncell) {
      start[c] = off + ex;
      range[c] = make_int2(off + ex, off + ex + v);
    }
    off += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) start[ncell] = (int32_t)n;
}

// Every particle to its cell's segment, at the place its count atomic gave it (an order the
// segment sort then makes deterministic).
__global__ __launch_bounds__(kRblBlock) void rbl_scatter_kernel(const int32_t* __restrict__ cell, int64_t n,
                                                                const int32_t* __restrict__ start,
                                                                const int32_t* __restrict__ rank,
                                                                int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (i >= n) return;
  idx[start[cell[i]] + rank[i]] = (int32_t)i;
}

// Each cell's segment in ascending particle index (insertion sort: cells hold a few to a
// few dozen particles), then every particle's cell-order position written by particle index
// into pos.
__global__ __launch_bounds__(kRblBlock) void rbl_segment_sort_kernel(const int32_t* __restrict__ start, int64_t ncell,
                                                                     int32_t* __restrict__ idx, int32_t* __restrict__ pos) {
  const int64_t c = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (c >= ncell) return;
  const int32_t b = start[c], e = start[c + 1];
  for (int32_t k = b + 1; k < e; ++k) {
    const int32_t v = idx[k];
    int32_t j = k - 1;
    while (j >= b && idx[j] > v) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = v;
  }
  for (int32_t k = b; k < e; ++k) pos[idx[k]] = k;
}

// floor(frac(x / L) 2^32), below 2^32 (0 for a non-finite coordinate).
__device__ inline uint32_t fixed_coord(double x, double L) {
  const double s = x / L;
  const double v = (s - floor(s)) * 4294967296.0;
  if (!(v >= 0.0)) return 0u;
  return v < 4294967295.0 ? (uint32_t)v : 0xffffffffu;
}

__global__ __launch_bounds__(kRblBlock) void rbl_gather_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                               const double* __restrict__ z, const double* __restrict__ q,
                                                               const double* __restrict__ eps,
                                                               const double* __restrict__ sig, int64_t n, double L,
                                                               uint64_t seed, uint64_t step, RblWs w) {
  // in particle order: the inputs are read in order and each record written to its
  // cell-order position
  const int64_t i = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t t = w.cell[i];
  RblRec r;
  r.pq = make_double4(x[i], y[i], z[i], q[i]);
  r.lj = make_double2(sqrt(eps[i]), sig[i]);
  U64x4 ctr = {{(uint64_t)i, 0ull, 3ull, 0ull}};
  r.u = u01_53(philox4x64_10(ctr, seed, step).v[0]);
  w.rec[t] = r;
  w.fxa[t] = make_uint4(fixed_coord(x[i], L), fixed_coord(y[i], L), fixed_coord(z[i], L), 0u);
}

// Minimum-image difference a - b of one coordinate: d - L rint(d / L), with d / L taken as
// d (1 / L).  The two can differ by one rounding, which changes rint only when |d| is
// within a rounding of L / 2, beyond every cutoff (r_s < L / 2); the result is then the
// other image of the same magnitude.  Evaluated without contraction into FMAs, so the
// squared distance that decides core, shell or neither is the same IEEE expression on
// every side.
__device__ inline double min_image_diff(double a, double b, double L, double invL) {
#pragma clang fp contract(off)
  const double d = a - b;
  return d - L * rint(d * invL);
}

__device__ inline double dist2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return dx * dx + dy * dy + dz * dz;
}

// Force on i from j given d = r_i - r_j and r2 = |d|^2, added into f (Eqs. lj and fshort),
// with the mixed LJ well depth as sqrt(eps_i) sqrt(eps_j) and one division, 1 / r^2.
// The pair force of Eq. (lj) and (fshort) on i from j, added to (fx, fy, fz); erfc(sqrt(alpha) r)
// as exp(-alpha r^2) erfcx(sqrt(alpha) r), the exponential shared with the Gaussian term.
__device__ inline void pair_force_add(double qi, double qj, double rei, double rej, double si, double sj,
                                      double alpha, double sqa, double tsap, const double* __restrict__ etab,
                                      int32_t eni, double einv, double dx, double dy, double dz,
                                      double r2, double& fx, double& fy, double& fz) {
  const double ir2 = 1.0 / r2;
  const double r = sqrt(r2);
  const double ir = r * ir2;
  double g = 0.0;
  const double e = rei * rej;
  if (e != 0.0) {
    const double s = 0.5 * (si + sj);
    const double s2 = s * s * ir2;
    const double s6 = s2 * s2 * s2;
    g += 24.0 * e * (2.0 * s6 * s6 - s6) * ir2;
  }
  if (qi != 0.0 && qj != 0.0) {
    const double ex = exp(-alpha * r2);
    const double kern = ex * (erfcx_table(etab, eni, einv, sqa * r) * ir2 + tsap * ir);
    g += qi * qj * kern * ir;
  }
  fx += g * dx;
  fy += g * dy;
  fz += g * dz;
}

// Position of pair entry j of the particle at cell-order position t.  The slots of 64
// consecutive particles are interleaved in groups of 4 entries, so the pair pass reads its
// 64 lanes' next 4 entries as one contiguous kilobyte, 16 B per lane (Q is a multiple of 4).
__device__ inline int64_t slot_index(int64_t t, int32_t Q, int32_t j) {
  return (t >> 6) * 64 * (int64_t)Q + (t & 63) * 4 + (int64_t)(j >> 2) * 256 + (j & 3);
}

// c mod nc for c in [-nc, 2 nc): stencil offsets stay within one period.
__device__ inline int32_t wrap_cell(int32_t c, int32_t nc) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); }

// Coordinates of the cell with x-major ordinal c = (cx nc + cy) nc + cz, through products with 1 / nc^2
// and 1 / nc in FP64: the quotients' fractional parts are at least 0.5 / nc^2 away from an
// integer, far beyond the rounding.
__device__ inline void cell_coords(int32_t c, const RblGrid& g, int32_t& cx, int32_t& cy, int32_t& cz) {
  cx = (int32_t)(((double)c + 0.5) * g.inv_nc2);
  const int32_t r = c - cx * g.nc * g.nc;
  cy = (int32_t)(((double)r + 0.5) * g.inv_nc);
  cz = r - cy * g.nc;
}

constexpr int kRblWaves = kRblBlock / 64;   // waves per block
constexpr int kListCap = 512;               // stencil positions held in LDS per wave
constexpr int kBatchCap = 256;              // batch positions held in LDS per wave (fallback)
static_assert(kListCap / 64 <= 32, "one bit per chunk in a 32-bit word");
constexpr int kTgtGroup = 3;                // targets classified together (2.2 per cell on average)
constexpr int kFallbackBlocks = 512;
constexpr int kCorrBlocks = 256;
constexpr int kMaxPairSlots = 4096;         // pair slots per particle at most

struct RblArgs {
  int64_t n, ncell;
  int32_t nblk, nblk8;   // blocks of the select kernel and that count over the 8 XCDs, rounded up
  int32_t p, Q;          // batch size, pair slots per particle
  int32_t eni;           // intervals of the erfcx table
  double einv;           // intervals per unit of x = sqrt(alpha) r
  double L, invL, alpha, sqa, tsap, rc2, rs2;
  // r_c^2 and r_s^2 in fixed-point units^2, each widened to a band [lo, hi] that holds every
  // squared distance the fixed-point FP32 estimate cannot place on one side
  float rc2lo, rc2hi, rs2lo, rs2hi;
};

// The lanes of the wave whose p is true (a comparison straight into a lane mask).
__device__ inline uint64_t wave_mask(bool p) { return __builtin_amdgcn_ballot_w64(p); }


__device__ inline int32_t lanes_below(uint64_t m) {
  return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// LDS written by some lanes of a wave and read by others: keep the accesses in order.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The stencil of cell (cx, cy, cz) in traversal order is span^2 rows (x outer, y inner);
// along z a row is the cells z0, z0 + 1, ... (mod nc), which in cell order is one run of
// particles, or two when it wraps.  Writes the positions [W0, W0 + kListCap) of the
// flattened traversal (cell-order indices) into list and returns its length T.
__device__ int32_t fill_stencil_window(const RblWs& w, const RblGrid& g, int32_t cx, int32_t cy, int32_t cz,
                                       int32_t W0, int32_t* list, int32_t lane) {
  const int32_t nc = g.nc, span = g.span, o0 = g.wrap ? 0 : -g.R;
  const int32_t z0 = wrap_cell(cz + o0, nc);
  const int32_t nsr = z0 + span > nc ? 2 : 1;
  const int32_t nseg = span * span * nsr;
  int32_t T = 0;
  for (int32_t s0 = 0; s0 < nseg; s0 += 64) {
    const int32_t sidx = s0 + lane;
    int32_t sb = 0, sl = 0;
    if (sidx < nseg) {
      const int32_t row = nsr == 2 ? sidx >> 1 : sidx, piece = sidx - row * nsr;
      // row / span through 1 / span in FP32: (row + 1/2) / span is at least 1 / (2 span)
      // from an integer, and span^2 < 2^19
      const int32_t a = (int32_t)(((float)row + 0.5f) * g.inv_span), b = row - a * span;
      const int32_t base = run_rank(wrap_cell(cx + o0 + a, nc), wrap_cell(cy + o0 + b, nc), nc) * nc;
      const int32_t c0 = piece == 0 ? z0 : 0;
      const int32_t c1 = piece == 0 ? min(z0 + span, nc) : z0 + span - nc;
      sb = w.range[base + c0].x;
      sl = w.range[base + c1 - 1].y - sb;
    }
    const int32_t incl = wave_scan(sl);
    const int32_t ex = T + incl - sl;
    const int32_t lo = max(ex, W0), hi = min(ex + sl, W0 + kListCap);
    // the run's positions: single entries up to a multiple of 4 (W0 is one), then 16 B at a time
    int32_t f = lo;
    for (; f < hi && (f & 3) != 0; ++f) list[f - W0] = sb + (f - ex);
    for (; f + 4 <= hi; f += 4) {
      const int32_t v = sb + (f - ex);
      *reinterpret_cast<int4*>(list + (f - W0)) = make_int4(v, v + 1, v + 2, v + 3);
    }
    for (; f < hi; ++f) list[f - W0] = sb + (f - ex);
    T += __builtin_amdgcn_readlane(incl, 63);
  }
  return T;
}

// Shell rank of draw b: floor((b + u) N_s / p), the expression and rounding of the
// definition, at most N_s - 1 (the exact value when the rounding of b + u reaches p).
__device__ inline int32_t batch_pos(int32_t b, double u, int32_t ns, int32_t p) {
  return min((int32_t)floor(((double)b + u) * (double)ns / (double)p), ns - 1);
}

__device__ inline double separation(double xi, double yi, double zi, const double4& o, double L, double invL,
                                   double& dx, double& dy, double& dz) {
  dx = min_image_diff(xi, o.x, L, invL);
  dy = min_image_diff(yi, o.y, L, invL);
  dz = min_image_diff(zi, o.z, L, invL);
  return dist2(dx, dy, dz);
}

// Selection: one wave per cell.  The cell's stencil -- its cell-order positions in traversal
// order, held in LDS -- is at most kListCap positions, streamed 64 at a time with the next
// chunk's fixed-point coordinates in flight.  Pass 1, per group of up to kTgtGroup particles
// of the cell, classifies every candidate against every target from the fixed-point
// differences in FP32; each lane keeps one core bit and one shell bit per chunk and target;
// where the estimate falls in a band around r_c^2 or r_s^2 the lane is classified afterwards
// with the FP64 distance of the definition.  The batch draws mark their shell ranks
// floor((b + u) N_s / p) in an LDS byte array, and each lane writes the pair entries it holds
// -- cell-order index, top bit set for shell members -- into the target's slot of Q entries
// from a wave prefix sum of the lanes' counts: every core member, and every shell member
// whose rank is marked (all of them when N_s <= p).  A cell whose stencil exceeds kListCap
// positions, or a target with more than Q
// pairs, is left to the fallback.  The pass waits on LDS and L2 at every chunk, so it keeps
// 8 waves per SIMD (64 VGPRs with groups of 3 targets).
__global__ __launch_bounds__(kRblBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void rbl_select_kernel(
    RblWs w, RblArgs a, RblGrid g) {
  __shared__ __align__(16) int32_t list_[kRblWaves][kListCap];
  __shared__ uint64_t mark_[kRblWaves][kListCap / 8];   // one byte per shell rank
  // blocks are dealt to the XCDs in turn: give each XCD a contiguous run of cells
  const int32_t blk = (int32_t)(blockIdx.x & 7) * a.nblk8 + (int32_t)(blockIdx.x >> 3);
  if (blk >= a.nblk) return;
  const int32_t lane = (int32_t)(threadIdx.x & 63);
  const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  // waves take the cells in x-major order of their coordinates
  const int32_t ord = blk * kRblWaves + wv;
  if (ord >= a.ncell) return;
  int32_t cx, cy, cz;
  cell_coords(ord, g, cx, cy, cz);
  const int2 own = w.range[run_rank(cx, cy, g.nc) * g.nc + cz];   // in flight with the stencil's ranges
  int32_t* list = list_[wv];
  uint8_t* mark = reinterpret_cast<uint8_t*>(mark_[wv]);
  mark_[wv][lane] = 0;
  const int32_t T = fill_stencil_window(w, g, cx, cy, cz, 0, list, lane);
  const int32_t t0 = __builtin_amdgcn_readfirstlane(own.x), t1 = __builtin_amdgcn_readfirstlane(own.y);
  if (t1 <= t0) return;
  if (T > kListCap) {
    for (int32_t t = t0 + lane; t < t1; t += 64) {
      w.cnt[t] = -1;
      w.fb[atomicAdd(w.nfb, 1)] = t;
    }
    return;
  }
  const int32_t C = (T + 63) / 64;
  wave_sync();
  for (int32_t g0 = t0; g0 < t1; g0 += kTgtGroup) {
    const int32_t mg = min(kTgtGroup, t1 - g0);
    uint4 tf[kTgtGroup];
    // bit c of cb[k] / sb[k] / ab[k]: this lane's candidate of chunk c is a core / shell /
    // ambiguous member of target g0 + k (the counts come from these bits afterwards)
    uint32_t cb[kTgtGroup], sb[kTgtGroup], ab[kTgtGroup];
    // every load of the group is issued here: a wait for a load also waits for the stores
    // before it, and the slot writes below are many
    double ug[kTgtGroup];
#pragma unroll
    for (int k = 0; k < kTgtGroup; ++k) {
      tf[k] = w.fxa[g0 + min(k, mg - 1)];
      ug[k] = w.rec[g0 + min(k, mg - 1)].u;
      cb[k] = sb[k] = ab[k] = 0;
    }
    int32_t un = lane < T ? list[lane] : -1;
    uint4 fn = un >= 0 ? w.fxa[un] : make_uint4(0u, 0u, 0u, 0u);
    for (int32_t c = 0; c < C; ++c) {
      const int32_t u = un;
      const uint4 fo = fn;
      if (c + 1 < C) {
        const int32_t f = (c + 1) * 64 + lane;
        un = f < T ? list[f] : -1;
        if (un >= 0) fn = w.fxa[un];
      }
      const uint32_t bit = 1u << c;
#pragma unroll
      for (int k = 0; k < kTgtGroup; ++k) {
        if (k < mg) {
          const float fdx = (float)(int32_t)(tf[k].x - fo.x);
          const float fdy = (float)(int32_t)(tf[k].y - fo.y);
          const float fdz = (float)(int32_t)(tf[k].z - fo.z);
          const float f2 = fdx * fdx + fdy * fdy + fdz * fdz;
          // bitwise, not short-circuit: straight-line lane masks
          const bool v = u >= 0;
          const bool near = f2 < a.rc2lo;
          const bool mid = (f2 > a.rc2hi) & (f2 < a.rs2lo);
          const bool shell = v & mid;
          const bool core = v & near & (u != g0 + k);
          const bool amb = v & !near & !mid & !(f2 > a.rs2hi);
          cb[k] |= core ? bit : 0u;
          sb[k] |= shell ? bit : 0u;
          ab[k] |= amb ? bit : 0u;
        }
      }
    }
    for (int32_t k = 0; k < mg; ++k) {
      const int32_t t = g0 + k;
      uint32_t cbits = 0, sbits = 0, abits = 0;
      double uoff = 0.0;
#pragma unroll
      for (int kk = 0; kk < kTgtGroup; ++kk) {
        if (kk == k) {
          cbits = cb[kk];
          sbits = sb[kk];
          abits = ab[kk];
          uoff = ug[kk];
        }
      }
      if (wave_mask(abits != 0) != 0) {
        // the ambiguous lanes (rare), with the FP64 distance of the definition
        const double4 me = w.rec[t].pq;
        for (int32_t c = 0; c < C; ++c) {
          if ((abits >> c) & 1) {
            const int32_t u = list[c * 64 + lane];
            double dx, dy, dz;
            const double r2 = separation(me.x, me.y, me.z, w.rec[u].pq, a.L, a.invL, dx, dy, dz);
            cbits |= (r2 < a.rc2 && u != t) ? (1u << c) : 0u;
            sbits |= (r2 >= a.rc2 && r2 <= a.rs2) ? (1u << c) : 0u;
          }
        }
      }
      const int32_t ns = wave_sum(__popc(sbits)), ncore = wave_sum(__popc(cbits));
      const bool sub = ns > a.p;
      const int32_t total = ncore + (sub ? a.p : ns);
      if (total > a.Q) {
        if (lane == 0) {
          w.cnt[t] = -1;
          w.fb[atomicAdd(w.nfb, 1)] = t;
        }
        continue;
      }
      if (sub) {
        for (int32_t b = lane; b < a.p; b += 64) mark[batch_pos(b, uoff, ns, a.p)] = 1;
        wave_sync();
      }
      // the lane's candidates the target uses: every core member, and every shell member
      // whose rank (in traversal order: chunks, then lanes) is marked -- all of them when
      // N_s <= p
      uint32_t ubits = cbits;
      if (sub) {
        int32_t rank0 = 0;
        for (int32_t c = 0; c < C; ++c) {
          const bool shell = (sbits >> c) & 1;
          const uint64_t sm = wave_mask(shell);
          if (shell && mark[rank0 + lanes_below(sm)] != 0) ubits |= 1u << c;
          rank0 += __popcll(sm);
        }
      } else {
        ubits |= sbits;
      }
      // every lane writes its entries in chunk order from its prefix offset (the slot holds
      // them by lane, then by chunk); entry j of the target sits at out[(j / 4) 256 + j mod 4]
      // (slot_index)
      uint32_t* const out = w.slot + slot_index(t, a.Q, 0);
      const int32_t mine = __popc(ubits);
      const int32_t incl = wave_scan(mine);
      const int32_t pos0 = __builtin_amdgcn_readlane(incl, 63);
      uint32_t j = (uint32_t)(incl - mine);
      while (ubits != 0) {
        const int32_t c = __builtin_ctz(ubits);
        ubits &= ubits - 1;
        out[((j >> 2) << 8) | (j & 3u)] = (uint32_t)list[c * 64 + lane] | (((sbits >> c) & 1) ? 0x80000000u : 0u);
        ++j;
      }
      if (sub) {
        wave_sync();
        mark_[wv][lane] = 0;
      }
      if (lane == 0) {
        w.cnt[t] = pos0;
        w.tns[t] = ns;
      }
    }
  }
}

// Pair forces: one lane per target (cell order), its slot's pairs added in slot order, shell
// pairs times N_s / p.
__global__ __launch_bounds__(kRblBlock) void rbl_pair_kernel(RblWs w, RblArgs a, double* __restrict__ F,
                                                             int32_t* __restrict__ ns_out) {
  __shared__ double etab[kErfcMaxIntervals * kErfcCoef];   // the erfcx table
  for (int i = threadIdx.x; i < a.eni * kErfcCoef; i += kRblBlock) etab[i] = w.etab[i];
  __syncthreads();
  const int32_t nb = (int32_t)((a.n + kRblBlock - 1) / kRblBlock), nb8 = (nb + 7) / 8;
  const int32_t blk = (int32_t)(blockIdx.x & 7) * nb8 + (int32_t)(blockIdx.x >> 3);
  const int64_t t = (int64_t)blk * kRblBlock + threadIdx.x;
  if (blk >= nb || t >= a.n) return;
  const int32_t cnt = w.cnt[t];
  if (cnt < 0) return;
  const double4 me = w.rec[t].pq;
  const double2 mlj = w.rec[t].lj;
  const int32_t i = w.idx[t];
  const int32_t ns = w.tns[t];
  const double wgt = ns > a.p ? (double)ns / (double)a.p : 1.0;
  // this particle's groups of 4 entries, 64 groups (1 KB) apart
  const uint4* e = reinterpret_cast<const uint4*>(w.slot + slot_index(t, a.Q, 0));
  double ax = 0.0, ay = 0.0, az = 0.0;
  // software pipeline: pair j + 1's data and the next group of entries are in flight while
  // pair j is evaluated
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  uint4 cur = cnt > 0 ? e[0] : z4;
  uint4 nxt = cnt > 4 ? e[64] : z4;
  uint32_t en = cur.x;
  double4 on = make_double4(0.0, 0.0, 0.0, 0.0);
  double2 ljn = make_double2(0.0, 0.0);
  if (cnt > 0) {
    on = w.rec[en & 0x7fffffffu].pq;
    ljn = w.rec[en & 0x7fffffffu].lj;
  }
  for (int32_t j = 0; j < cnt; ++j) {
    const uint32_t ej = en;
    const double4 o = on;
    const double2 olj = ljn;
    if (j + 1 < cnt) {
      const int32_t k = (j + 1) & 3;   // the same on every lane
      if (k == 0) {
        cur = nxt;
        if (j + 5 < cnt) nxt = e[((j + 5) >> 2) * 64];
      }
      en = k == 0 ? cur.x : k == 1 ? cur.y : k == 2 ? cur.z : cur.w;
      on = w.rec[en & 0x7fffffffu].pq;
      ljn = w.rec[en & 0x7fffffffu].lj;
    }
    double dx, dy, dz;
    const double r2 = separation(me.x, me.y, me.z, o, a.L, a.invL, dx, dy, dz);
    double px = 0.0, py = 0.0, pz = 0.0;
    pair_force_add(me.w, o.w, mlj.x, olj.x, mlj.y, olj.y, a.alpha, a.sqa, a.tsap, etab, a.eni, a.einv, dx, dy, dz, r2,
                   px, py, pz);
    const double wt = (ej >> 31) ? wgt : 1.0;
    ax += wt * px;
    ay += wt * py;
    az += wt * pz;
  }
  if (!isfinite(me.x + me.y + me.z)) ax = ay = az = __builtin_nan("");
  F[i] = ax;
  F[a.n + i] = ay;
  F[2 * a.n + i] = az;
  if (ns_out != nullptr) ns_out[i] = ns;
}

// Fallback for the targets the selection left (a stencil longer than kListCap, or more than
// Q pairs): one wave per target, the stencil streamed in windows of kListCap positions and
// classified twice (N_s, then ranks); each shell member's rank is tested against the draws
// near floor(r p / N_s - u); the pairs go through an LDS queue evaluated 64 at a time, each
// lane summing its pairs, and a fixed butterfly sums the lanes.
__global__ __launch_bounds__(kRblBlock) void rbl_fallback_kernel(RblWs w, RblArgs a, RblGrid g, double* __restrict__ F,
                                                                 int32_t* __restrict__ ns_out) {
  __shared__ __align__(16) int32_t list_[kRblWaves][kListCap];
  __shared__ uint32_t queue_[kRblWaves][64];
  __shared__ int32_t batch_[kRblWaves][kBatchCap];
  const int32_t nfb = __builtin_amdgcn_readfirstlane(*w.nfb);
  const int32_t lane = (int32_t)(threadIdx.x & 63);
  const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  int32_t* list = list_[wv];
  uint32_t* queue = queue_[wv];
  int32_t* batch = batch_[wv];
  for (int32_t s = (int32_t)blockIdx.x * kRblWaves + wv; s < nfb; s += (int32_t)gridDim.x * kRblWaves) {
    const int32_t t = __builtin_amdgcn_readfirstlane(w.fb[s]);
    const int32_t i = w.idx[t];
    const double4 me = w.rec[t].pq;
    const double2 mlj = w.rec[t].lj;
    const int32_t cx = cell_coord(me.x, a.L, g.nc), cy = cell_coord(me.y, a.L, g.nc), cz = cell_coord(me.z, a.L, g.nc);
    wave_sync();
    const int32_t T = fill_stencil_window(w, g, cx, cy, cz, 0, list, lane);
    // fn(u, core, shell) for every stencil position, 64 at a time, window by window
    auto classified = [&](auto&& fn) {
      for (int32_t W0 = 0; W0 < T; W0 += kListCap) {
        wave_sync();
        fill_stencil_window(w, g, cx, cy, cz, W0, list, lane);
        wave_sync();
        const int32_t W1 = min(T, W0 + kListCap);
        for (int32_t f0 = W0; f0 < W1; f0 += 64) {
          const int32_t f = f0 + lane;
          const int32_t u = f < W1 ? list[f - W0] : t;
          double dx, dy, dz;
          const double r2 = separation(me.x, me.y, me.z, w.rec[u].pq, a.L, a.invL, dx, dy, dz);
          fn(u, r2 < a.rc2 && u != t, r2 >= a.rc2 && r2 <= a.rs2);
        }
      }
    };
    int32_t ns = 0;
    classified([&](int32_t, bool, bool shell) { ns += __popcll(wave_mask(shell)); });
    const bool sub = ns > a.p;
    const double uoff = w.rec[t].u;
    const double wgt = sub ? (double)ns / (double)a.p : 1.0;
    const double slope = (double)a.p / (double)ns;
    const bool listed = sub && a.p <= kBatchCap;
    if (listed) {
      wave_sync();
      for (int32_t b = lane; b < a.p; b += 64) batch[b] = batch_pos(b, uoff, ns, a.p);
      wave_sync();
    }
    // whether shell rank r is a draw's: the draw that can land on r is within one of
    // floor(r p / N_s - u)
    auto in_batch = [&](int32_t r) {
      const int32_t bc = (int32_t)floor((double)r * slope - uoff);
      bool hit = false;
      for (int32_t b = bc - 1; b <= bc + 1; ++b)
        if (b >= 0 && b < a.p) hit |= (listed ? batch[b] : batch_pos(b, uoff, ns, a.p)) == r;
      return hit;
    };
    double ax = 0.0, ay = 0.0, az = 0.0;
    auto flush = [&](int32_t nq) {
      if (lane < nq) {
        const uint32_t e = queue[lane];
        const int32_t u = (int32_t)(e & 0x7fffffffu);
        const double4 o = w.rec[u].pq;
        const double2 olj = w.rec[u].lj;
        double dx, dy, dz;
        const double r2 = separation(me.x, me.y, me.z, o, a.L, a.invL, dx, dy, dz);
        double px = 0.0, py = 0.0, pz = 0.0;
        pair_force_add(me.w, o.w, mlj.x, olj.x, mlj.y, olj.y, a.alpha, a.sqa, a.tsap, w.etab, a.eni, a.einv, dx, dy,
                       dz, r2, px, py, pz);
        const double wt = (e >> 31) ? wgt : 1.0;
        ax += wt * px;
        ay += wt * py;
        az += wt * pz;
      }
    };
    int32_t qn = 0, rank0 = 0;
    classified([&](int32_t u, bool core, bool shell) {
      const uint64_t M = wave_mask(shell);
      const bool use = core || (shell && (!sub || in_batch(rank0 + lanes_below(M))));
      rank0 += __popcll(M);
      const uint64_t U = wave_mask(use);
      const int32_t cnt = __popcll(U);
      if (cnt == 0) return;
      const int32_t pos = qn + lanes_below(U);
      const uint32_t e = (uint32_t)u | (shell ? 0x80000000u : 0u);
      if (use && pos < 64) queue[pos] = e;
      if (qn + cnt >= 64) {
        wave_sync();
        flush(64);
        wave_sync();
        if (use && pos >= 64) queue[pos - 64] = e;
        qn += cnt - 64;
      } else {
        qn += cnt;
      }
    });
    wave_sync();
    flush(qn);
    for (int o = 1; o < 64; o <<= 1) {
      ax += __shfl_xor(ax, o, 64);
      ay += __shfl_xor(ay, o, 64);
      az += __shfl_xor(az, o, 64);
    }
    if (!isfinite(me.x + me.y + me.z)) ax = ay = az = __builtin_nan("");
    if (lane == 0) {
      F[i] = ax;
      F[a.n + i] = ay;
      F[2 * a.n + i] = az;
      if (ns_out != nullptr) ns_out[i] = ns;
    }
  }
}

// Fixed-order sums of 3-vectors: block b adds entries [b per, (b + 1) per) of src (thread t
// takes every 256th from t, then a fixed tree) and writes scale times the sum to dst[3 b + d].
// Entry k, component d is src[d * stride + k] (SOA) or src[3 k + d].  Two launches, the first
// over the forces, give F^corr = -(1/N) sum_i F_i.
template <bool SOA>
__global__ __launch_bounds__(kRblBlock) void rbl_sum3_kernel(const double* __restrict__ src, int64_t stride, int64_t nsrc,
                                                             int64_t per, double scale, double* __restrict__ dst) {
  __shared__ double red[3][kRblBlock];
  double s[3] = {0.0, 0.0, 0.0};
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(b0 + per, nsrc);
  for (int64_t b = b0 + threadIdx.x; b < b1; b += kRblBlock)
    for (int d = 0; d < 3; ++d) s[d] += SOA ? src[d * stride + b] : src[3 * b + d];
  for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = s[d];
  __syncthreads();
  for (int k = kRblBlock / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x < 3) dst[3 * (int64_t)blockIdx.x + threadIdx.x] = scale * red[threadIdx.x][0];
}

__global__ __launch_bounds__(kRblBlock) void rbl_apply_kernel(const double* __restrict__ corr, int64_t n,
                                                              double* __restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (i >= n) return;
  F[i] += corr[0];
  F[n + i] += corr[1];
  F[2 * n + i] += corr[2];
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>((n + kRblBlock - 1) / kRblBlock, 1); }

}  // namespace
}  // namespace rbe

using namespace rbe;

struct rbl_plan {
  rbl_params prm;
  RblGrid grid;
  int64_t ncell = 0;
  int32_t nscan = 0;     // scan blocks
  int32_t nsel = 0;      // select blocks (kRblWaves cells each)
  int32_t Q = 0;         // pair slots per particle
  int32_t eni = 1;       // erfcx table: intervals and their width in x = sqrt(alpha) r
  double eh = 0.1;
  size_t off[18] = {};
  size_t bytes = 0;
  hipEvent_t ev[4] = {};  // caller's events around the select and pair kernels (optional)
};

namespace {

// Slots per particle: room for the mean core count and the smaller of p and the mean shell
// count of a uniform system, each with a Poisson allowance m + 6 sqrt(m) + 16; a particle
// with more pairs takes the fallback.
int32_t pair_slots(const rbl_params& q) {
  const double dens = (double)q.N / (q.L * q.L * q.L);
  const double vc = 4.0 / 3.0 * kRblPi * q.r_c * q.r_c * q.r_c;
  const double vs = 4.0 / 3.0 * kRblPi * q.r_s * q.r_s * q.r_s - vc;
  auto allow = [](double m) { return m + 6.0 * std::sqrt(m) + 16.0; };
  const double k = std::ceil(allow(dens * vc) + std::min((double)q.p, allow(dens * vs)));
  return (int32_t)std::min(4.0 * std::ceil(k / 4.0), (double)kMaxPairSlots);
}

// The band around R^2 (fixed-point units u = L / 2^32) outside which the FP32 estimate f2 of
// a squared distance r^2 is on the same side of R^2 as r^2.  The floors of the two fixed
// coordinates put each difference within 2 u of the exact one, so |DX^2 - d^2| <= 4|d| + 4
// per axis and the sum is within 4 sqrt(3) r + 12 (u^2); the conversions to FP32, squares and
// sums add a relative 3e-7.  At r near R that is a relative 6.93 / R + 12 / R^2 + 3e-7, R in
// units; the band takes four times that plus 1e-6.
void fixed_point_band(double R, double L, float& lo, float& hi) {
  const double Ru = R * (4294967296.0 / L);
  const double rel = 4.0 * (6.93 / Ru + 12.0 / (Ru * Ru) + 3e-7) + 1e-6;
  lo = (float)(Ru * Ru * (1.0 - rel));
  hi = (float)(Ru * Ru * (1.0 + rel));
}

void rbl_layout(rbl_plan* p) {
  const size_t n = (size_t)p->prm.N, nc = (size_t)p->ncell;
  const size_t sizes[18] = {
      sizeof(int32_t) * nc,        sizeof(int32_t) * n,            sizeof(int32_t) * (nc + 1),
      sizeof(int32_t) * (size_t)(p->nscan + 1), sizeof(int32_t) * n, sizeof(int32_t) * n,
      sizeof(RblRec) * n,          sizeof(uint4) * n,              sizeof(int2) * nc,
      1 /* unused */,              sizeof(uint32_t) * 64 * ((n + 63) / 64) * (size_t)p->Q, sizeof(int32_t) * n,
      sizeof(int32_t) * n,         sizeof(int32_t) * n,            sizeof(int32_t),
      sizeof(double) * 3 * kCorrBlocks, sizeof(double) * 3, sizeof(double) * kErfcMaxIntervals * kErfcCoef};
  size_t o = 0;
  for (int k = 0; k < 18; ++k) {
    p->off[k] = o;
    o = rbl_align(o + std::max<size_t>(sizes[k], 1));
  }
  p->bytes = o;
}

RblWs rbl_view(const rbl_plan* p, void* ws) {
  char* b = static_cast<char*>(ws);
  RblWs w;
  w.count = reinterpret_cast<int32_t*>(b + p->off[0]);
  w.rank = reinterpret_cast<int32_t*>(b + p->off[1]);
  w.start = reinterpret_cast<int32_t*>(b + p->off[2]);
  w.bsum = reinterpret_cast<int32_t*>(b + p->off[3]);
  w.cell = reinterpret_cast<int32_t*>(b + p->off[4]);
  w.idx = reinterpret_cast<int32_t*>(b + p->off[5]);
  w.rec = reinterpret_cast<RblRec*>(b + p->off[6]);
  w.fxa = reinterpret_cast<uint4*>(b + p->off[7]);
  w.range = reinterpret_cast<int2*>(b + p->off[8]);
  w.slot = reinterpret_cast<uint32_t*>(b + p->off[10]);
  w.cnt = reinterpret_cast<int32_t*>(b + p->off[11]);
  w.tns = reinterpret_cast<int32_t*>(b + p->off[12]);
  w.fb = reinterpret_cast<int32_t*>(b + p->off[13]);
  w.nfb = reinterpret_cast<int32_t*>(b + p->off[14]);
  w.partial = reinterpret_cast<double*>(b + p->off[15]);
  w.corr = reinterpret_cast<double*>(b + p->off[16]);
  w.etab = reinterpret_cast<double*>(b + p->off[17]);
  return w;
}

}  // namespace

extern "C" {

rbe_status rbl_plan_create(const rbl_params* prm, rbl_plan** out) {
  if (out == nullptr) return fail(RBE_EINVAL, "out is NULL");
  *out = nullptr;
  if (prm == nullptr) return fail(RBE_EINVAL, "params is NULL");
  const rbl_params& q = *prm;
  if (q.N < 0 || q.N >= ((int64_t)1 << 31)) return fail(RBE_EINVAL, "N must be in [0, 2^31) (got %lld)", (long long)q.N);
  if (!(std::isfinite(q.L) && q.L > 0.0)) return fail(RBE_EINVAL, "L must be finite and > 0");
  if (!(std::isfinite(q.alpha) && q.alpha >= 0.0)) return fail(RBE_EINVAL, "alpha must be finite and >= 0");
  if (!(q.r_c > 0.0 && q.r_c <= q.r_s && q.r_s < 0.5 * q.L))
    return fail(RBE_EINVAL, "cutoffs must satisfy 0 < r_c <= r_s < L/2 (got r_c = %g, r_s = %g, L = %g)", q.r_c, q.r_s,
                q.L);
  if (q.p < 1) return fail(RBE_EINVAL, "the batch size p must be >= 1 (got %d)", q.p);
  RblGrid g;
  const double ncd = std::floor(q.L / q.r_c);
  if (ncd > 645.0) return fail(RBE_EINVAL, "the cell grid would exceed 2^28 cells (L / r_c = %g)", q.L / q.r_c);
  g.nc = std::max(1, (int32_t)ncd);
  const double h = q.L / (double)g.nc;
  g.R = (int32_t)std::ceil(q.r_s / h);
  g.wrap = (2 * g.R + 1 > g.nc) ? 1 : 0;
  g.span = g.wrap ? g.nc : 2 * g.R + 1;
  g.inv_span = 1.0f / (float)g.span;
  g.inv_nc = 1.0 / (double)g.nc;
  g.inv_nc2 = 1.0 / ((double)g.nc * (double)g.nc);
  rbl_plan* p = new (std::nothrow) rbl_plan();
  if (p == nullptr) return fail(RBE_EINVAL, "out of host memory");
  p->prm = q;
  p->grid = g;
  p->ncell = (int64_t)g.nc * g.nc * g.nc;
  p->nscan = (int32_t)((p->ncell + kScanChunk - 1) / kScanChunk);
  p->nsel = (int32_t)((p->ncell + kRblWaves - 1) / kRblWaves);
  p->Q = pair_slots(q);
  {
    // the table covers x up to sqrt(alpha) r_s (at least 0.1, at most kErfcMaxX) in intervals
    // of width at most 0.1
    const double x_tab = std::min(std::max(std::sqrt(q.alpha) * q.r_s, 0.1), kErfcMaxX);
    p->eni = std::min(std::max((int32_t)std::ceil(x_tab / 0.1), 1), kErfcMaxIntervals);
    p->eh = x_tab / (double)p->eni;
  }
  rbl_layout(p);
  *out = p;
  return RBE_OK;
}

size_t rbl_plan_workspace_bytes(const rbl_plan* p) { return p ? p->bytes : 0; }

rbe_status rbl_plan_grid(const rbl_plan* p, int32_t* cells_per_axis, int32_t* reach, int32_t* stencil_span) {
  if (!p || !cells_per_axis || !reach || !stencil_span) return fail(RBE_EINVAL, "NULL argument");
  *cells_per_axis = p->grid.nc;
  *reach = p->grid.R;
  *stencil_span = p->grid.span;
  return RBE_OK;
}

rbe_status rbl_plan_capacity(const rbl_plan* p, int32_t* pairs_per_particle, int32_t* stencil_positions) {
  if (!p || !pairs_per_particle || !stencil_positions) return fail(RBE_EINVAL, "NULL argument");
  *pairs_per_particle = p->Q;
  *stencil_positions = kListCap;
  return RBE_OK;
}

rbe_status rbl_plan_set_timing_events(rbl_plan* p, void* select_begin, void* select_end, void* pair_begin,
                                      void* pair_end) {
  if (p == nullptr) return fail(RBE_EINVAL, "plan is NULL");
  p->ev[0] = static_cast<hipEvent_t>(select_begin);
  p->ev[1] = static_cast<hipEvent_t>(select_end);
  p->ev[2] = static_cast<hipEvent_t>(pair_begin);
  p->ev[3] = static_cast<hipEvent_t>(pair_end);
  return RBE_OK;
}

void rbl_plan_destroy(rbl_plan* p) { delete p; }

rbe_status rbl_short_force(const rbl_plan* p, const double* x, const double* y, const double* z, const double* q,
                           const double* eps, const double* sig, uint64_t seed, uint64_t step, double* F,
                           int32_t* ns, void* ws, void* stream) {
  if (p == nullptr) return fail(RBE_EINVAL, "plan is NULL");
  if (ws == nullptr) return fail(RBE_EWORKSPACE, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kRblAlign) return fail(RBE_EWORKSPACE, "workspace must be 256-byte aligned");
  const int64_t n = p->prm.N;
  if (n > 0 && (!x || !y || !z || !q || !eps || !sig || !F)) return fail(RBE_EINVAL, "NULL particle or force array");
  rbe_status st = device_ok();
  if (st != RBE_OK) return st;
  if (n == 0) return RBE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const RblWs w = rbl_view(p, ws);
  const RblGrid& g = p->grid;
  const int64_t nc = p->ncell;
  const rbl_params& prm = p->prm;
  hipLaunchKernelGGL(rbl_zero_kernel, dim3(blocks_for(std::max<int64_t>(nc, kErfcMaxIntervals))), dim3(kRblBlock), 0,
                     s, w.count, nc, w.nfb, w.etab, p->eni, p->eh);
  hipLaunchKernelGGL(rbl_cell_kernel, dim3(blocks_for(n)), dim3(kRblBlock), 0, s, x, y, z, n, prm.L, g.nc, w.cell,
                     w.count, w.rank);
  hipLaunchKernelGGL(rbl_scan_sums_kernel, dim3((unsigned)p->nscan), dim3(kRblBlock), 0, s, w.count, nc, w.bsum);
  hipLaunchKernelGGL(rbl_scan_offsets_kernel, dim3(1), dim3(kRblBlock), 0, s, w.bsum, p->nscan);
  hipLaunchKernelGGL(rbl_scan_apply_kernel, dim3((unsigned)p->nscan), dim3(kRblBlock), 0, s, w.count, nc, w.bsum,
                     w.start, w.range, n);
  hipLaunchKernelGGL(rbl_scatter_kernel, dim3(blocks_for(n)), dim3(kRblBlock), 0, s, w.cell, n, w.start, w.rank,
                     w.idx);
  hipLaunchKernelGGL(rbl_segment_sort_kernel, dim3(blocks_for(nc)), dim3(kRblBlock), 0, s, w.start, nc, w.idx, w.cell);
  hipLaunchKernelGGL(rbl_gather_kernel, dim3(blocks_for(n)), dim3(kRblBlock), 0, s, x, y, z, q, eps, sig, n, prm.L,
                     seed, step, w);
  RblArgs a;
  a.n = n;
  a.ncell = nc;
  a.nblk = p->nsel;
  a.nblk8 = (p->nsel + 7) / 8;
  a.p = prm.p;
  a.Q = p->Q;
  a.eni = p->eni;
  a.einv = 1.0 / p->eh;
  a.L = prm.L;
  a.invL = 1.0 / prm.L;
  a.alpha = prm.alpha;
  a.sqa = std::sqrt(prm.alpha);
  a.tsap = 2.0 * std::sqrt(prm.alpha / kRblPi);
  a.rc2 = prm.r_c * prm.r_c;
  a.rs2 = prm.r_s * prm.r_s;
  fixed_point_band(prm.r_c, prm.L, a.rc2lo, a.rc2hi);
  fixed_point_band(prm.r_s, prm.L, a.rs2lo, a.rs2hi);
  if (p->ev[0] != nullptr) (void)hipEventRecord(p->ev[0], s);
  hipLaunchKernelGGL(rbl_select_kernel, dim3((unsigned)(8 * a.nblk8)), dim3(kRblBlock), 0, s, w, a, g);
  if (p->ev[1] != nullptr) (void)hipEventRecord(p->ev[1], s);
  const int64_t nbp = (n + kRblBlock - 1) / kRblBlock;
  if (p->ev[2] != nullptr) (void)hipEventRecord(p->ev[2], s);
  hipLaunchKernelGGL(rbl_pair_kernel, dim3((unsigned)(8 * ((nbp + 7) / 8))), dim3(kRblBlock), 0, s, w, a, F, ns);
  if (p->ev[3] != nullptr) (void)hipEventRecord(p->ev[3], s);
  hipLaunchKernelGGL(rbl_fallback_kernel, dim3(kFallbackBlocks), dim3(kRblBlock), 0, s, w, a, g, F, ns);
  const int64_t per = (n + kCorrBlocks - 1) / kCorrBlocks;
  const int64_t nb1 = (n + per - 1) / per;
  hipLaunchKernelGGL(rbl_sum3_kernel<true>, dim3((unsigned)nb1), dim3(kRblBlock), 0, s, F, n, n, per, 1.0, w.partial);
  hipLaunchKernelGGL(rbl_sum3_kernel<false>, dim3(1), dim3(kRblBlock), 0, s, w.partial, (int64_t)0, nb1, nb1,
                     -1.0 / (double)n, w.corr);
  hipLaunchKernelGGL(rbl_apply_kernel, dim3(blocks_for(n)), dim3(kRblBlock), 0, s, w.corr, n, F);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "rbl_short_force launch");
  return RBE_OK;
}

}  // extern "C"
