// Random batch list (RBL) short-range force on gfx950 (Sec. 2.3; Algorithm 2): a cell list
// built on the device, the exact core sum and the systematic shell batch per particle, and
// the momentum correction.  FP64 throughout.
//
// One evaluation:
//   cells   : cell of every particle, per-cell counts (atomic adds), exclusive scan into
//             cell starts, scatter into cell order (atomic slots), then every cell's short
//             segment sorted by particle index, so the order is deterministic;
//   gather  : positions, charges and LJ parameters copied into cell order;
//   force   : one thread per particle in cell order (neighbouring lanes share most of their
//             stencil cells); pass 1 over the stencil sums the core and counts the shell,
//             pass 2 walks the shell again and adds the batch members, stopping after the
//             last one; the raw forces are written by particle index and summed per block
//             in a fixed order;
//   correct : one block adds the block sums in order; every force gets -(1/N) of the total.
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
};

struct RblWs {
  int32_t* count;
  int32_t* fill;
  int32_t* start;    // ncell + 1
  int32_t* bsum;     // scan block sums
  int32_t* cell;     // N
  int32_t* idx;      // N: particle index at each cell-order position
  double* xs;        // N each, in cell order
  double* ys;
  double* zs;
  double* qs;
  double* es;
  double* ss;
  double* partial;   // 3 per force block
  double* corr;      // 3
};

// Cell coordinate of a position along one axis: min(floor(frac(x / L) nc), nc - 1).
__device__ inline int32_t cell_coord(double x, double L, int32_t nc) {
  const double s = x / L;
  const double f = s - floor(s);
  const int32_t c = (int32_t)floor(f * (double)nc);
  return c < nc - 1 ? c : nc - 1;
}

__global__ __launch_bounds__(kRblBlock) void rbl_zero_kernel(int32_t* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (i < n) a[i] = 0;
}

__global__ __launch_bounds__(kRblBlock) void rbl_cell_kernel(const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             const double* __restrict__ z, int64_t n, double L,
                                                             int32_t nc, int32_t* __restrict__ cell,
                                                             int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t c = (cell_coord(x[i], L, nc) * nc + cell_coord(y[i], L, nc)) * nc + cell_coord(z[i], L, nc);
  cell[i] = c;
  atomicAdd(&count[c], 1);
}

// Exclusive scan of the cell counts in three launches: per-chunk totals, an in-order scan
// of the totals (one block), then each chunk rescanned with its offset.
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* sh, int32_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kRblBlock; o <<= 1) {
    const int32_t a = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const int32_t incl = sh[t];
  *total = sh[kRblBlock - 1];
  __syncthreads();
  return incl - v;
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
                                                                   int32_t* __restrict__ start, int64_t n) {
  __shared__ int32_t sh[kRblBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int32_t off = bsum[blockIdx.x];
  for (int k = 0; k < kScanChunk / kRblBlock; ++k) {
    const int64_t c = base + (int64_t)k * kRblBlock + threadIdx.x;
    const int32_t v = c < ncell ? count[c] : 0;
    int32_t tot;
    const int32_t ex = block_exclusive_scan(v, sh, &tot);
    if (c < ncell) start[c] = off + ex;
    off += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) start[ncell] = (int32_t)n;
}

__global__ __launch_bounds__(kRblBlock) void rbl_scatter_kernel(const int32_t* __restrict__ cell, int64_t n,
                                                                const int32_t* __restrict__ start,
                                                                int32_t* __restrict__ fill, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t c = cell[i];
  idx[start[c] + atomicAdd(&fill[c], 1)] = (int32_t)i;
}

// Each cell's segment in ascending particle index (insertion sort: cells hold a few to a
// few dozen particles).
__global__ __launch_bounds__(kRblBlock) void rbl_segment_sort_kernel(const int32_t* __restrict__ start, int64_t ncell,
                                                                     int32_t* __restrict__ idx) {
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
}

__global__ __launch_bounds__(kRblBlock) void rbl_gather_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                               const double* __restrict__ z, const double* __restrict__ q,
                                                               const double* __restrict__ eps,
                                                               const double* __restrict__ sig, int64_t n, RblWs w) {
  const int64_t t = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  if (t >= n) return;
  const int32_t i = w.idx[t];
  w.xs[t] = x[i];
  w.ys[t] = y[i];
  w.zs[t] = z[i];
  w.qs[t] = q[i];
  w.es[t] = eps[i];
  w.ss[t] = sig[i];
}

// Minimum-image difference a - b of one coordinate: d - L rint(d / L).  Evaluated without
// contraction into FMAs, so the squared distance that decides core, shell or neither is
// the same IEEE expression on every side.
__device__ inline double min_image_diff(double a, double b, double L) {
#pragma clang fp contract(off)
  const double d = a - b;
  return d - L * rint(d / L);
}

__device__ inline double dist2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return dx * dx + dy * dy + dz * dz;
}

// Force on i from j given d = r_i - r_j and r2 = |d|^2, added into f (Eqs. lj and fshort).
__device__ inline void pair_force_add(double qi, double qj, double ei, double ej, double si, double sj,
                                      double alpha, double sqa, double tsap, double dx, double dy, double dz,
                                      double r2, double& fx, double& fy, double& fz) {
  const double r = sqrt(r2);
  double g = 0.0;
  const double e = sqrt(ei * ej);
  if (e != 0.0) {
    const double s = 0.5 * (si + sj);
    const double s2 = s * s / r2;
    const double s6 = s2 * s2 * s2;
    g += 24.0 * e * (2.0 * s6 * s6 - s6) / r2;
  }
  if (qi != 0.0 && qj != 0.0) {
    const double kern = erfc(sqa * r) / r2 + tsap * exp(-alpha * r2) / r;
    g += qi * qj * kern / r;
  }
  fx += g * dx;
  fy += g * dy;
  fz += g * dz;
}

__device__ inline int32_t wrap_cell(int32_t c, int32_t nc) {
  const int32_t m = c % nc;
  return m < 0 ? m + nc : m;
}

__global__ __launch_bounds__(kRblBlock) void rbl_force_kernel(RblWs w, int64_t n, double L, double alpha, double sqa,
                                                              double tsap, double rc2, double rs2, int32_t p,
                                                              RblGrid g, uint64_t seed, uint64_t step,
                                                              double* __restrict__ F, int32_t* __restrict__ ns_out) {
  __shared__ double red[3][kRblBlock];
  const int64_t t = (int64_t)blockIdx.x * kRblBlock + threadIdx.x;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (t < n) {
    const int32_t i = w.idx[t];
    const double xi = w.xs[t], yi = w.ys[t], zi = w.zs[t];
    const double qi = w.qs[t], ei = w.es[t], si = w.ss[t];
    const int32_t nc = g.nc;
    const int32_t cx = cell_coord(xi, L, nc), cy = cell_coord(yi, L, nc), cz = cell_coord(zi, L, nc);
    const int32_t o0 = g.wrap ? 0 : -g.R;
    // pass 1: core sum and shell count
    double cfx = 0.0, cfy = 0.0, cfz = 0.0;
    int32_t ns = 0;
    for (int32_t a = 0; a < g.span; ++a) {
      const int32_t ca = wrap_cell(cx + o0 + a, nc);
      for (int32_t b = 0; b < g.span; ++b) {
        const int32_t cb = wrap_cell(cy + o0 + b, nc);
        for (int32_t c = 0; c < g.span; ++c) {
          const int32_t cell = (ca * nc + cb) * nc + wrap_cell(cz + o0 + c, nc);
          const int32_t e = w.start[cell + 1];
          for (int32_t u = w.start[cell]; u < e; ++u) {
            const double dx = min_image_diff(xi, w.xs[u], L);
            const double dy = min_image_diff(yi, w.ys[u], L);
            const double dz = min_image_diff(zi, w.zs[u], L);
            const double r2 = dist2(dx, dy, dz);
            if (r2 < rc2) {
              if (w.idx[u] != i)
                pair_force_add(qi, w.qs[u], ei, w.es[u], si, w.ss[u], alpha, sqa, tsap, dx, dy, dz, r2, cfx, cfy,
                               cfz);
            } else if (r2 <= rs2) {
              ++ns;
            }
          }
        }
      }
    }
    // pass 2: the shell batch in traversal order
    double sfx = 0.0, sfy = 0.0, sfz = 0.0;
    double wgt = 1.0;
    if (ns > 0) {
      const bool sub = ns > p;
      double uoff = 0.0;
      int64_t target = 0;
      int32_t picked = 0;
      if (sub) {
        U64x4 ctr = {{(uint64_t)i, 0ull, 3ull, 0ull}};
        uoff = u01_53(philox4x64_10(ctr, seed, step).v[0]);
        wgt = (double)ns / (double)p;
        target = (int64_t)floor((0.0 + uoff) * (double)ns / (double)p);
      }
      const int32_t want = sub ? p : ns;
      int64_t k = 0;
      for (int32_t a = 0; a < g.span && picked < want; ++a) {
        const int32_t ca = wrap_cell(cx + o0 + a, nc);
        for (int32_t b = 0; b < g.span && picked < want; ++b) {
          const int32_t cb = wrap_cell(cy + o0 + b, nc);
          for (int32_t c = 0; c < g.span && picked < want; ++c) {
            const int32_t cell = (ca * nc + cb) * nc + wrap_cell(cz + o0 + c, nc);
            const int32_t e = w.start[cell + 1];
            for (int32_t u = w.start[cell]; u < e && picked < want; ++u) {
              const double dx = min_image_diff(xi, w.xs[u], L);
              const double dy = min_image_diff(yi, w.ys[u], L);
              const double dz = min_image_diff(zi, w.zs[u], L);
              const double r2 = dist2(dx, dy, dz);
              if (r2 < rc2 || r2 > rs2) continue;
              if (!sub || k == target) {
                pair_force_add(qi, w.qs[u], ei, w.es[u], si, w.ss[u], alpha, sqa, tsap, dx, dy, dz, r2, sfx, sfy,
                               sfz);
                ++picked;
                if (sub) target = (int64_t)floor(((double)picked + uoff) * (double)ns / (double)p);
              }
              ++k;
            }
          }
        }
      }
    }
    fx = cfx + wgt * sfx;
    fy = cfy + wgt * sfy;
    fz = cfz + wgt * sfz;
    F[i] = fx;
    F[n + i] = fy;
    F[2 * n + i] = fz;
    if (ns_out != nullptr) ns_out[i] = ns;
  }
  // block sums of the raw forces in a fixed order
  red[0][threadIdx.x] = fx;
  red[1][threadIdx.x] = fy;
  red[2][threadIdx.x] = fz;
  __syncthreads();
  for (int s = kRblBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) w.partial[3 * (int64_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// F^corr = -(1/N) sum of the block sums (thread t adds blocks t, t + 256, ... in order, then
// a fixed tree).
__global__ __launch_bounds__(kRblBlock) void rbl_corr_kernel(RblWs w, int32_t nblocks, int64_t n) {
  __shared__ double red[3][kRblBlock];
  double s[3] = {0.0, 0.0, 0.0};
  for (int32_t b = threadIdx.x; b < nblocks; b += kRblBlock)
    for (int d = 0; d < 3; ++d) s[d] += w.partial[3 * (int64_t)b + d];
  for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = s[d];
  __syncthreads();
  for (int k = kRblBlock / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x < 3) w.corr[threadIdx.x] = n > 0 ? -red[threadIdx.x][0] / (double)n : 0.0;
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
  int32_t nforce = 0;    // force blocks
  size_t off[14] = {};
  size_t bytes = 0;
};

namespace {

void rbl_layout(rbl_plan* p) {
  const int64_t n = p->prm.N, nc = p->ncell;
  const size_t sizes[14] = {
      sizeof(int32_t) * (size_t)nc, sizeof(int32_t) * (size_t)nc, sizeof(int32_t) * (size_t)(nc + 1),
      sizeof(int32_t) * (size_t)(p->nscan + 1), sizeof(int32_t) * (size_t)n, sizeof(int32_t) * (size_t)n,
      sizeof(double) * (size_t)n, sizeof(double) * (size_t)n, sizeof(double) * (size_t)n,
      sizeof(double) * (size_t)n, sizeof(double) * (size_t)n, sizeof(double) * (size_t)n,
      sizeof(double) * 3 * (size_t)p->nforce, sizeof(double) * 3};
  size_t o = 0;
  for (int k = 0; k < 14; ++k) {
    p->off[k] = o;
    o = rbl_align(o + std::max<size_t>(sizes[k], 1));
  }
  p->bytes = o;
}

RblWs rbl_view(const rbl_plan* p, void* ws) {
  char* b = static_cast<char*>(ws);
  RblWs w;
  w.count = reinterpret_cast<int32_t*>(b + p->off[0]);
  w.fill = reinterpret_cast<int32_t*>(b + p->off[1]);
  w.start = reinterpret_cast<int32_t*>(b + p->off[2]);
  w.bsum = reinterpret_cast<int32_t*>(b + p->off[3]);
  w.cell = reinterpret_cast<int32_t*>(b + p->off[4]);
  w.idx = reinterpret_cast<int32_t*>(b + p->off[5]);
  w.xs = reinterpret_cast<double*>(b + p->off[6]);
  w.ys = reinterpret_cast<double*>(b + p->off[7]);
  w.zs = reinterpret_cast<double*>(b + p->off[8]);
  w.qs = reinterpret_cast<double*>(b + p->off[9]);
  w.es = reinterpret_cast<double*>(b + p->off[10]);
  w.ss = reinterpret_cast<double*>(b + p->off[11]);
  w.partial = reinterpret_cast<double*>(b + p->off[12]);
  w.corr = reinterpret_cast<double*>(b + p->off[13]);
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
  rbl_plan* p = new (std::nothrow) rbl_plan();
  if (p == nullptr) return fail(RBE_EINVAL, "out of host memory");
  p->prm = q;
  p->grid = g;
  p->ncell = (int64_t)g.nc * g.nc * g.nc;
  p->nscan = (int32_t)((p->ncell + kScanChunk - 1) / kScanChunk);
  p->nforce = (int32_t)blocks_for(q.N);
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
  hipLaunchKernelGGL(rbl_zero_kernel, dim3(blocks_for(nc)), dim3(kRblBlock), 0, s, w.count, nc);
  hipLaunchKernelGGL(rbl_zero_kernel, dim3(blocks_for(nc)), dim3(kRblBlock), 0, s, w.fill, nc);
  hipLaunchKernelGGL(rbl_cell_kernel, dim3(blocks_for(n)), dim3(kRblBlock), 0, s, x, y, z, n, prm.L, g.nc, w.cell,
                     w.count);
  hipLaunchKernelGGL(rbl_scan_sums_kernel, dim3((unsigned)p->nscan), dim3(kRblBlock), 0, s, w.count, nc, w.bsum);
  hipLaunchKernelGGL(rbl_scan_offsets_kernel, dim3(1), dim3(kRblBlock), 0, s, w.bsum, p->nscan);
  hipLaunchKernelGGL(rbl_scan_apply_kernel, dim3((unsigned)p->nscan), dim3(kRblBlock), 0, s, w.count, nc, w.bsum,
                     w.start, n);
  hipLaunchKernelGGL(rbl_scatter_kernel, dim3(blocks_for(n)), dim3(kRblBlock), 0, s, w.cell, n, w.start, w.fill,
                     w.idx);
  hipLaunchKernelGGL(rbl_segment_sort_kernel, dim3(blocks_for(nc)), dim3(kRblBlock), 0, s, w.start, nc, w.idx);
  hipLaunchKernelGGL(rbl_gather_kernel, dim3(blocks_for(n)), dim3(kRblBlock), 0, s, x, y, z, q, eps, sig, n, w);
  const double sqa = std::sqrt(prm.alpha);
  const double tsap = 2.0 * std::sqrt(prm.alpha / kRblPi);
  hipLaunchKernelGGL(rbl_force_kernel, dim3((unsigned)p->nforce), dim3(kRblBlock), 0, s, w, n, prm.L, prm.alpha, sqa,
                     tsap, prm.r_c * prm.r_c, prm.r_s * prm.r_s, prm.p, g, seed, step, F, ns);
  hipLaunchKernelGGL(rbl_corr_kernel, dim3(1), dim3(kRblBlock), 0, s, w, p->nforce, n);
  hipLaunchKernelGGL(rbl_apply_kernel, dim3(blocks_for(n)), dim3(kRblBlock), 0, s, w.corr, n, F);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "rbl_short_force launch");
  return RBE_OK;
}

}  // extern "C"
