// Host side of the RBE library: argument checks, plans, work lists, workspace
// layout, the host wave-vector sampler and the C entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "metropolis.h"
#include "philox.h"
#include "rbe.h"
#include "rbe_internal.h"

namespace rbe {

namespace {
thread_local std::string g_last_error;
}  // namespace

rbe_status fail(rbe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

rbe_status hip_fail(hipError_t e, const char* what) {
  return fail(RBE_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Device availability, probed once per process.
rbe_status device_ok() {
  static std::once_flag once;
  static int count = 0;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] { err = hipGetDeviceCount(&count); });
  if (err != hipSuccess || count <= 0)
    return fail(RBE_ENODEV, "no HIP device available (%s)", hipGetErrorString(err));
  return RBE_OK;
}

namespace {

constexpr size_t kAlign = 256;
constexpr double kTwoPi = 6.283185307179586476925286766559;
// Largest per-component spread of sampled |m| accepted for RBE_FP32 phases.  At 12 (a
// 1M-atom box at alpha = 0.06) the measured force error is 5e-6 relative RMS; it grows
// about linearly with the spread, so 16 keeps it below 1e-5.
constexpr double kFp32PhaseMaxSigma = 16.0;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------- sampler tables

struct ComponentTable {
  int32_t M = 0;
  std::vector<double> c;   // prefix sums for j = -M..M
};

double beta_of(double L, double alpha) { return (M_PI * M_PI) / (alpha * L * L); }

ComponentTable component_table(double L, double alpha) {
  ComponentTable t;
  const double sigma = L * std::sqrt(alpha / 2.0) / M_PI;
  t.M = (int32_t)std::ceil(9.0 * sigma) + 1;
  const double beta = beta_of(L, alpha);
  t.c.resize(2 * (size_t)t.M + 1);
  double acc = 0.0;
  for (int32_t j = -t.M; j <= t.M; ++j) {
    acc = acc + std::exp(-beta * (double)((int64_t)j * j));
    t.c[(size_t)(j + t.M)] = acc;
  }
  return t;
}

// S = Z^3 - 1 with Z the full one-dimensional sum (window plus margin, in increasing j).
double normalization(double L, double alpha) {
  const ComponentTable t = component_table(L, alpha);
  const double beta = beta_of(L, alpha);
  double z = 0.0;
  for (int32_t j = -t.M - 8; j <= t.M + 8; ++j) z += std::exp(-beta * (double)((int64_t)j * j));
  return z * z * z - 1.0;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace
}  // namespace rbe

using namespace rbe;

// ---------------------------------------------------------------- plan

struct rbe_plan {
  int32_t B = 0;
  std::vector<int64_t> sys_off, k_off;
  std::vector<double> L, alpha;
  int precision = RBE_FP64;
  int phase_mode = RBE_PHASE_AUTO;
  bool cached = false;
  int rho_variant = 0;
  int force_variant = 1;
  int32_t rho_grid_cap = 0;     // waves; 0: one wave per work item
  int32_t rho_clamp = 1;        // occupancy clamp of the rho-shaped passes
  int32_t force_grid_cap = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // optional kernel timing events
  bool sampler_ok = true;
  int32_t sampler = RBE_SAMPLER_EXACT;
  int32_t burn_in = 64;

  // host copies of the device tables
  std::vector<SysDesc> sys;
  std::vector<RhoItem> rho_items;
  std::vector<ForceItem> force_items;
  std::vector<KRed> kred;
  std::vector<double> cdf;
  int64_t cdf_stride = kCdfHeader;   // doubles per system table
  // workspace layout (byte offsets)
  size_t off_sys = 0, off_rho = 0, off_force = 0, off_kred = 0, off_cdf = 0, off_part = 0,
         off_xy = 0, off_cache = 0, off_frows = 0, total = 0;
  size_t ws_bytes = 0;      // workspace size: the largest layout over all variants
  int64_t n_partials = 0;   // complex slots
  int64_t n_cache = 0;      // (cos, sin) pairs
  uint64_t layout_id = 0;   // unique per built layout (process-wide), see rbe_evaluate_static

  int64_t n_total() const { return sys_off[B]; }
  int64_t p_total() const { return k_off[B]; }
  RhoVariant rv() const {
    return precision == RBE_FP64 ? kRhoVariantsF64[rho_variant] : kRhoVariantsF32[rho_variant];
  }
};

struct rbe_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void build_layout(rbe_plan* p) {
  const RhoVariant rv = p->rv();
  const ForceVariant fv = kForceVariants[p->force_variant];
  // particles per rho tile; with the phase cache a k-lane variant runs the per-wave kernel,
  // whose tiles are 64 npl particles
  const int tile = (p->cached && rv.wpb == 1) ? 64 * rv.npl : rv.tile;
  const int fchunk = kForceBlock * fv.nplf;
  p->sys.assign(p->B, SysDesc{});
  p->rho_items.clear();
  p->force_items.clear();
  p->kred.assign((size_t)p->p_total(), KRed{});
  int64_t part = 0, cache = 0;
  for (int32_t b = 0; b < p->B; ++b) {
    SysDesc& s = p->sys[b];
    s.n_off = p->sys_off[b];
    s.k_off = p->k_off[b];
    s.n = (int32_t)(p->sys_off[b + 1] - p->sys_off[b]);
    s.p = (int32_t)(p->k_off[b + 1] - p->k_off[b]);
    s.L = p->L[b];
    s.alpha = p->alpha[b];
    s.ntiles = (s.n + tile - 1) / tile;
    s.part_off = part;
    part += (int64_t)s.ntiles * s.p;
    s.cache_off = cache;
    if (p->cached) cache += (int64_t)s.n * s.p;
    for (int32_t l = 0; l < s.p; ++l) p->kred[(size_t)(s.k_off + l)] = KRed{s.part_off + (int64_t)l * s.ntiles, s.ntiles, b};
    const int nf = std::max(1, (s.n + fchunk - 1) / fchunk);
    for (int f = 0; f < nf; ++f) {
      const int p0 = f * fchunk;
      p->force_items.push_back(ForceItem{b, p0, std::max(0, std::min(fchunk, s.n - p0)), f == 0 ? 1 : 0});
    }
  }
  // rho items.  Cooperative variants (one block per CU sharing work through LDS): one item
  // per (tile, KC-chunk), tile-major, so a wave's consecutive claims reuse its tile.
  // Otherwise a system's wave vectors are cut into ranges of whole KC-chunks whose chunk
  // counts differ by at most one (at most krange vectors each), and items are ordered
  // range-major with the longer ranges first, so the hardware dispatcher starts the
  // longest waves first and the short ones fill the tail.
  if (rv.wpb == 16) {
    for (int32_t b = 0; b < p->B; ++b) {
      const SysDesc& s = p->sys[b];
      for (int32_t t = 0; t < s.ntiles; ++t)
        for (int32_t k0 = 0; k0 < s.p; k0 += rv.kc) p->rho_items.push_back(RhoItem{b, t, k0, std::min(rv.kc, s.p - k0)});
    }
  } else {
    struct Range { int32_t b, k0, nk, chunks; };
    std::vector<Range> ranges;
    for (int32_t b = 0; b < p->B; ++b) {
      const SysDesc& s = p->sys[b];
      if (s.p <= 0 || s.ntiles <= 0) continue;
      const int nr = (s.p + rv.krange - 1) / rv.krange;
      const int nch = (s.p + rv.kc - 1) / rv.kc;
      int c0 = 0;
      for (int r = 0; r < nr; ++r) {
        const int cr = nch / nr + (r < nch % nr ? 1 : 0);
        const int k0 = c0 * rv.kc;
        ranges.push_back(Range{b, k0, std::min(cr * rv.kc, s.p - k0), cr});
        c0 += cr;
      }
    }
    std::stable_sort(ranges.begin(), ranges.end(),
                     [](const Range& a, const Range& c) { return a.chunks > c.chunks; });
    for (const Range& r : ranges)
      for (int32_t t = 0; t < p->sys[r.b].ntiles; ++t) p->rho_items.push_back(RhoItem{r.b, t, r.k0, r.nk});
    if (rv.wpb == 1) {
      // k-lane blocks take one item each, and the dispatcher deals consecutive blocks to
      // the eight XCDs in turn.  The partials of a wave vector lie tile after tile, four
      // tiles to a 64-byte line, so within every aligned group of 32 items of one
      // (system, k-range) block 32g + r takes tile 32g + 4 (r mod 8) + r / 8: the four
      // tiles of a line are written from one XCD's L2.  Results do not depend on the order.
      std::vector<RhoItem>& it = p->rho_items;
      for (size_t g0 = 0; g0 + 32 <= it.size(); g0 += 32) {
        const RhoItem& a = it[g0];
        const RhoItem& z = it[g0 + 31];
        if (a.sys != z.sys || a.k0 != z.k0 || z.tile != a.tile + 31) continue;
        const RhoItem first = a;
        for (int r = 0; r < 32; ++r) it[g0 + (size_t)r] = RhoItem{first.sys, first.tile + 4 * (r % 8) + r / 8, first.k0, first.nk};
      }
    }
  }
  // sampler tables: header (S, 2M+1, p, k_off, D, beta) and c_-M .. c_M per system, fixed stride
  p->sampler_ok = true;
  std::vector<ComponentTable> tabs((size_t)p->B);
  int64_t max_len = 0;
  for (int32_t b = 0; b < p->B; ++b) {
    SysDesc& s = p->sys[b];
    tabs[(size_t)b] = component_table(p->L[b], p->alpha[b]);
    const ComponentTable& t = tabs[(size_t)b];
    const double p0 = t.c[(size_t)t.M] - (t.M > 0 ? t.c[(size_t)t.M - 1] : 0.0);
    const double pz = p0 / t.c.back();
    if (pz * pz * pz > 0.5 || t.c.size() > (1u << 22)) {
      p->sampler_ok = false;
      s.cdf_len = 0;
      continue;
    }
    s.cdf_len = (int32_t)t.c.size();
    max_len = std::max<int64_t>(max_len, s.cdf_len);
  }
  p->cdf_stride = kCdfHeader + max_len;
  if ((int64_t)p->B * p->cdf_stride > ((int64_t)1 << 25)) {
    // tables this large (over 256 MB in all) are not kept on the device
    p->sampler_ok = false;
    for (SysDesc& s : p->sys) s.cdf_len = 0;
    p->cdf_stride = kCdfHeader;
  }
  p->cdf.assign((size_t)(p->B * p->cdf_stride), 0.0);
  for (int32_t b = 0; b < p->B; ++b) {
    const SysDesc& s = p->sys[b];
    double* h = p->cdf.data() + (size_t)b * (size_t)p->cdf_stride;
    h[2] = s.p;
    h[3] = (double)s.k_off;
    h[4] = (double)metropolis_width(p->L[b], p->alpha[b]);
    h[5] = beta_of(p->L[b], p->alpha[b]);
    if (s.cdf_len == 0) continue;
    h[0] = normalization(p->L[b], p->alpha[b]);
    h[1] = s.cdf_len;
    std::copy(tabs[(size_t)b].c.begin(), tabs[(size_t)b].c.end(), h + kCdfHeader);
  }
  p->n_partials = part;
  p->n_cache = cache;
  size_t o = 0;
  p->off_sys = o;   o = align_up(o + sizeof(SysDesc) * p->sys.size());
  p->off_rho = o;   o = align_up(o + sizeof(RhoItem) * p->rho_items.size());
  p->off_force = o; o = align_up(o + sizeof(ForceItem) * p->force_items.size());
  p->off_kred = o;  o = align_up(o + sizeof(KRed) * p->kred.size());
  p->off_cdf = o;   o = align_up(o + sizeof(double) * p->cdf.size());
  p->off_part = o;  o = align_up(o + 2 * sizeof(double) * (size_t)p->n_partials);
  p->off_xy = o;    o = align_up(o + 2 * sizeof(double) * (size_t)p->p_total());
  p->off_cache = o; o = align_up(o + 2 * sizeof(float) * (size_t)p->n_cache);
  p->off_frows = o; o = align_up(o + sizeof(ForceRowF32) * (size_t)p->p_total());
  p->total = std::max<size_t>(o, kAlign);
  static std::atomic<uint64_t> next_layout_id{0};
  p->layout_id = ++next_layout_id;
}

WsView view_of(const rbe_plan* p, void* ws) {
  char* b = static_cast<char*>(ws);
  WsView w;
  w.sys = reinterpret_cast<const SysDesc*>(b + p->off_sys);
  w.rho_items = reinterpret_cast<const RhoItem*>(b + p->off_rho);
  w.force_items = reinterpret_cast<const ForceItem*>(b + p->off_force);
  w.kred = reinterpret_cast<const KRed*>(b + p->off_kred);
  w.cdf = reinterpret_cast<const double*>(b + p->off_cdf);
  w.partials = reinterpret_cast<double*>(b + p->off_part);
  w.xy = reinterpret_cast<double*>(b + p->off_xy);
  w.cache = reinterpret_cast<float*>(b + p->off_cache);
  w.frows = reinterpret_cast<ForceRowF32*>(b + p->off_frows);
  return w;
}

LaunchShape shape_of(const rbe_plan* p) {
  LaunchShape s;
  s.B = p->B;
  s.n_total = p->n_total();
  s.p_total = p->p_total();
  s.n_rho_items = (int32_t)p->rho_items.size();
  s.n_force_items = (int32_t)p->force_items.size();
  s.precision = p->precision;
  s.cached = p->cached ? 1 : 0;
  s.rv = p->rv();
  s.rho_variant = p->rho_variant;
  s.fv = kForceVariants[p->force_variant];
  s.force_variant = p->force_variant;
  s.cdf_stride = (int32_t)p->cdf_stride;
  s.sampler = p->sampler;
  s.burn_in = p->burn_in;
  s.rho_grid_cap = p->rho_grid_cap;
  s.rho_clamp = p->rho_clamp;
  s.force_grid_cap = p->force_grid_cap;
  s.sys0 = p->B == 1 ? p->sys[0] : SysDesc{};
  s.ev_rho_begin = p->ev[0];
  s.ev_rho_end = p->ev[1];
  s.ev_force_begin = p->ev[2];
  s.ev_force_end = p->ev[3];
  return s;
}

rbe_status check_ws(const rbe_plan* p, const void* ws) {
  if (ws == nullptr) return fail(RBE_EWORKSPACE, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(RBE_EWORKSPACE, "workspace must be %zu-byte aligned", kAlign);
  (void)p;
  return RBE_OK;
}

rbe_status check_common(const rbe_plan* p, const void* ws) {
  if (p == nullptr) return fail(RBE_EINVAL, "plan is NULL");
  rbe_status st = check_ws(p, ws);
  if (st != RBE_OK) return st;
  return device_ok();
}

bool need(const void* ptr, int64_t count) { return count == 0 || ptr != nullptr; }

// Copies of the plan's host tables (system rows, work lists, reduction descriptors,
// sampler tables) into ws, enqueued on s.  The source is pageable host memory owned by
// the plan, so each copy has read it by the time hipMemcpyAsync returns.
rbe_status enqueue_upload(const rbe_plan* p, void* ws, hipStream_t s) {
  char* b = static_cast<char*>(ws);
  struct Copy { size_t off; const void* src; size_t bytes; } copies[] = {
      {p->off_sys, p->sys.data(), sizeof(SysDesc) * p->sys.size()},
      {p->off_rho, p->rho_items.data(), sizeof(RhoItem) * p->rho_items.size()},
      {p->off_force, p->force_items.data(), sizeof(ForceItem) * p->force_items.size()},
      {p->off_kred, p->kred.data(), sizeof(KRed) * p->kred.size()},
      {p->off_cdf, p->cdf.data(), sizeof(double) * p->cdf.size()},
  };
  for (const Copy& c : copies) {
    if (c.bytes == 0) continue;
    hipError_t e = hipMemcpyAsync(b + c.off, c.src, c.bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(plan upload)");
  }
  return RBE_OK;
}

}  // namespace

// ---------------------------------------------------------------- C entry points

extern "C" {

int32_t rbe_abi_version(void) { return RBE_ABI_VERSION; }

const char* rbe_status_string(rbe_status s) {
  switch (s) {
    case RBE_OK: return "RBE_OK";
    case RBE_EINVAL: return "RBE_EINVAL: invalid argument";
    case RBE_ENODEV: return "RBE_ENODEV: no HIP device";
    case RBE_EHIP: return "RBE_EHIP: HIP runtime error";
    case RBE_EWORKSPACE: return "RBE_EWORKSPACE: bad workspace";
    case RBE_EUNSUPPORTED: return "RBE_EUNSUPPORTED: not supported";
  }
  return "unknown rbe_status";
}

const char* rbe_last_error(void) { return g_last_error.c_str(); }

rbe_status rbe_normalization(double L, double alpha, double* S_out) {
  if (!finite_pos(L) || !finite_pos(alpha)) return fail(RBE_EINVAL, "L and alpha must be finite and > 0");
  if (S_out == nullptr) return fail(RBE_EINVAL, "S_out is NULL");
  *S_out = normalization(L, alpha);
  return RBE_OK;
}

rbe_status rbe_sample_k(uint64_t seed, uint64_t stream_id, double L, double alpha, int32_t P,
                        int32_t* m_out, double* w_out, double* S_out) {
  if (!finite_pos(L) || !finite_pos(alpha)) return fail(RBE_EINVAL, "L and alpha must be finite and > 0");
  if (P < 0) return fail(RBE_EINVAL, "P must be >= 0 (got %d)", P);
  if (P > 0 && m_out == nullptr) return fail(RBE_EINVAL, "m_out is NULL");
  const ComponentTable t = component_table(L, alpha);
  if (t.c.size() > (1u << 26)) return fail(RBE_EINVAL, "sampling window too large (sigma = %g)", L * std::sqrt(alpha / 2) / M_PI);
  const double Z = t.c.back();
  const double S = normalization(L, alpha);
  for (int32_t l = 0; l < P; ++l) {
    int32_t v[3] = {0, 0, 0};
    bool ok = false;
    for (int a = 0; a < kMaxAttempts && !ok; ++a) {
      U64x4 ctr = {{(uint64_t)l, (uint64_t)a, 0ull, 0ull}};
      const U64x4 r = philox4x64_10(ctr, seed, stream_id);
      for (int d = 0; d < 3; ++d) v[d] = inverse_cdf(t.c.data(), t.M, u01_53(r.v[d]) * Z);
      ok = v[0] != 0 || v[1] != 0 || v[2] != 0;
    }
    if (!ok) return fail(RBE_EINVAL, "zero wave vector drawn %d times in a row", kMaxAttempts);
    m_out[3 * l] = v[0];
    m_out[3 * l + 1] = v[1];
    m_out[3 * l + 2] = v[2];
    if (w_out) w_out[l] = S / (double)P;
  }
  if (S_out) *S_out = S;
  return RBE_OK;
}

rbe_status rbe_sample_k_metropolis(uint64_t seed, uint64_t stream_id, double L, double alpha, int32_t P,
                                   int32_t burn_in, int32_t* m_out, double* w_out, double* S_out) {
  if (!finite_pos(L) || !finite_pos(alpha)) return fail(RBE_EINVAL, "L and alpha must be finite and > 0");
  if (P < 0) return fail(RBE_EINVAL, "P must be >= 0 (got %d)", P);
  if (burn_in < 0) return fail(RBE_EINVAL, "burn_in must be >= 0 (got %d)", burn_in);
  if (P > 0 && m_out == nullptr) return fail(RBE_EINVAL, "m_out is NULL");
  const int32_t D = metropolis_width(L, alpha);
  const double beta = beta_of(L, alpha);
  const double S = normalization(L, alpha);
  for (int32_t l = 0; l < P; ++l) {
    int32_t v[3];
    metropolis_chain(seed, stream_id, (uint64_t)l, burn_in, D, beta, v);
    m_out[3 * l] = v[0];
    m_out[3 * l + 1] = v[1];
    m_out[3 * l + 2] = v[2];
    if (w_out) w_out[l] = S / (double)P;
  }
  if (S_out) *S_out = S;
  return RBE_OK;
}

rbe_status rbe_plan_set_sampler(rbe_plan* p, int32_t sampler, int32_t burn_in) {
  if (!p) return fail(RBE_EINVAL, "plan is NULL");
  if (sampler != RBE_SAMPLER_EXACT && sampler != RBE_SAMPLER_METROPOLIS)
    return fail(RBE_EINVAL, "unknown sampler %d", sampler);
  if (burn_in < 0) return fail(RBE_EINVAL, "burn_in must be >= 0 (got %d)", burn_in);
  p->sampler = sampler;
  p->burn_in = burn_in;
  return RBE_OK;
}

rbe_status rbe_ewald_weights(double L, double alpha, int32_t P, const int32_t* m, double* w_out) {
  if (!finite_pos(L) || !finite_pos(alpha)) return fail(RBE_EINVAL, "L and alpha must be finite and > 0");
  if (P < 0) return fail(RBE_EINVAL, "P must be >= 0");
  if (P > 0 && (m == nullptr || w_out == nullptr)) return fail(RBE_EINVAL, "NULL array");
  const double ks = 2.0 * M_PI / L;
  for (int32_t l = 0; l < P; ++l) {
    const double kx = ks * m[3 * l], ky = ks * m[3 * l + 1], kz = ks * m[3 * l + 2];
    w_out[l] = std::exp(-(kx * kx + ky * ky + kz * kz) / (4.0 * alpha));
  }
  return RBE_OK;
}

rbe_status rbe_plan_create(const rbe_batch_desc* batch, int32_t precision, int32_t phase_mode, rbe_plan** out) {
  if (out == nullptr) return fail(RBE_EINVAL, "out is NULL");
  *out = nullptr;
  if (batch == nullptr) return fail(RBE_EINVAL, "batch descriptor is NULL");
  const int32_t B = batch->B;
  const int64_t* sys_off = batch->sys_off;
  const int64_t* k_off = batch->k_off;
  const double* L = batch->L;
  const double* alpha = batch->alpha;
  if (B <= 0) return fail(RBE_EINVAL, "B must be > 0 (got %d)", B);
  if (!sys_off || !k_off || !L || !alpha) return fail(RBE_EINVAL, "NULL batch array");
  if (precision != RBE_FP64 && precision != RBE_FP32_MIXED && precision != RBE_FP32)
    return fail(RBE_EINVAL, "unknown precision %d", precision);
  if (phase_mode < RBE_PHASE_AUTO || phase_mode > RBE_PHASE_CACHED) return fail(RBE_EINVAL, "unknown phase mode %d", phase_mode);
  if (phase_mode == RBE_PHASE_CACHED && precision != RBE_FP32_MIXED)
    return fail(RBE_EUNSUPPORTED, "the phase cache exists for RBE_FP32_MIXED only");
  if (sys_off[0] != 0 || k_off[0] != 0) return fail(RBE_EINVAL, "offsets must start at 0");
  for (int32_t b = 0; b < B; ++b) {
    if (sys_off[b + 1] < sys_off[b] || k_off[b + 1] < k_off[b])
      return fail(RBE_EINVAL, "offsets must be non-decreasing (system %d)", b);
    if (sys_off[b + 1] - sys_off[b] > (int64_t)INT32_MAX / 2 || k_off[b + 1] - k_off[b] > (int64_t)INT32_MAX / 2)
      return fail(RBE_EINVAL, "system %d too large", b);
    if (!finite_pos(L[b]) || !finite_pos(alpha[b]))
      return fail(RBE_EINVAL, "system %d: L and alpha must be finite and > 0", b);
    // FP32 phases: the rounding error grows with |m|, whose spread under the sampling
    // density is sigma_m = L sqrt(2 alpha) / (2 pi) per component.
    if (precision == RBE_FP32 && L[b] * std::sqrt(2.0 * alpha[b]) / kTwoPi > kFp32PhaseMaxSigma)
      return fail(RBE_EUNSUPPORTED,
                  "system %d: RBE_FP32 phases need L sqrt(2 alpha) / (2 pi) <= %.0f (got %.1f); use RBE_FP32_MIXED",
                  b, kFp32PhaseMaxSigma, L[b] * std::sqrt(2.0 * alpha[b]) / kTwoPi);
  }
  rbe_plan* p = new rbe_plan();
  p->B = B;
  p->sys_off.assign(sys_off, sys_off + B + 1);
  p->k_off.assign(k_off, k_off + B + 1);
  p->L.assign(L, L + B);
  p->alpha.assign(alpha, alpha + B);
  p->precision = precision;
  p->phase_mode = phase_mode;
  // Measured: recomputing phases beats the HBM phase cache at every benchmarked shape.
  p->cached = phase_mode == RBE_PHASE_CACHED;
  // The workspace is sized for the largest layout over all variants, so the
  // autotuner can switch variants without reallocating.
  const int nr = precision == RBE_FP64 ? kNumRhoVariantsF64 : kNumRhoVariantsF32;
  size_t most = 0;
  for (int r = 0; r < nr; ++r)
    for (int f = 0; f < kNumForceVariants; ++f) {
      p->rho_variant = r;
      p->force_variant = f;
      build_layout(p);
      most = std::max(most, p->total);
    }
  p->ws_bytes = most;
  p->rho_variant = 0;
  p->force_variant = 1;
  build_layout(p);
  *out = p;
  return RBE_OK;
}

size_t rbe_plan_workspace_bytes(const rbe_plan* p) { return p ? p->ws_bytes : 0; }

rbe_status rbe_plan_num_variants(const rbe_plan* p, int32_t* n_rho, int32_t* n_force) {
  if (!p || !n_rho || !n_force) return fail(RBE_EINVAL, "NULL argument");
  *n_rho = p->precision == RBE_FP64 ? kNumRhoVariantsF64 : kNumRhoVariantsF32;
  *n_force = kNumForceVariants;
  return RBE_OK;
}

rbe_status rbe_plan_rho_variant_info(const rbe_plan* p, int32_t variant, int32_t* npl, int32_t* kc,
                                     int32_t* krange, int32_t* wpb, int32_t* tile, int32_t* comp) {
  if (!p || !npl || !kc || !krange || !wpb || !tile || !comp) return fail(RBE_EINVAL, "NULL argument");
  const int nr = p->precision == RBE_FP64 ? kNumRhoVariantsF64 : kNumRhoVariantsF32;
  if (variant < 0 || variant >= nr) return fail(RBE_EINVAL, "rho variant %d out of range [0, %d)", variant, nr);
  const RhoVariant& rv = p->precision == RBE_FP64 ? kRhoVariantsF64[variant] : kRhoVariantsF32[variant];
  *npl = rv.npl;
  *kc = rv.kc;
  *krange = rv.krange;
  *wpb = rv.wpb;
  *tile = (p->cached && rv.wpb == 1) ? 64 * rv.npl : rv.tile;
  *comp = rv.comp;
  return RBE_OK;
}

rbe_status rbe_plan_get_tiles(const rbe_plan* p, int32_t* rv, int32_t* fv) {
  if (!p || !rv || !fv) return fail(RBE_EINVAL, "NULL argument");
  *rv = p->rho_variant;
  *fv = p->force_variant;
  return RBE_OK;
}

rbe_status rbe_plan_set_occupancy_clamp(rbe_plan* p, int32_t on) {
  if (!p) return fail(RBE_EINVAL, "plan is NULL");
  p->rho_clamp = on ? 1 : 0;
  return RBE_OK;
}

rbe_status rbe_plan_get_occupancy_clamp(const rbe_plan* p, int32_t* on) {
  if (!p || !on) return fail(RBE_EINVAL, "NULL argument");
  *on = p->rho_clamp;
  return RBE_OK;
}

rbe_status rbe_plan_get_grid_caps(const rbe_plan* p, int32_t* rho_cap, int32_t* force_cap) {
  if (!p || !rho_cap || !force_cap) return fail(RBE_EINVAL, "NULL argument");
  *rho_cap = p->rho_grid_cap;
  *force_cap = p->force_grid_cap;
  return RBE_OK;
}

rbe_status rbe_plan_set_tiles(rbe_plan* p, int32_t rv, int32_t fv) {
  if (!p) return fail(RBE_EINVAL, "plan is NULL");
  const int nr = p->precision == RBE_FP64 ? kNumRhoVariantsF64 : kNumRhoVariantsF32;
  if (rv < -1 || rv >= nr) return fail(RBE_EINVAL, "rho variant %d out of range [0, %d)", rv, nr);
  if (fv < -1 || fv >= kNumForceVariants) return fail(RBE_EINVAL, "force variant %d out of range", fv);
  if (rv >= 0) p->rho_variant = rv;
  if (fv >= 0) p->force_variant = fv;
  build_layout(p);
  return RBE_OK;
}

void rbe_plan_destroy(rbe_plan* p) { delete p; }

rbe_status rbe_plan_upload(const rbe_plan* p, void* ws, void* stream) {
  rbe_status st = check_common(p, ws);
  if (st != RBE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = enqueue_upload(p, ws, s);
  if (st != RBE_OK) return st;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(plan upload)");
  return RBE_OK;
}

rbe_status rbe_structure_factor(const rbe_plan* p, const double* x, const double* y, const double* z,
                                const double* q, const int32_t* m, double* rho, void* ws, void* stream) {
  rbe_status st = check_common(p, ws);
  if (st != RBE_OK) return st;
  const int64_t n = p->n_total(), P = p->p_total();
  if (!need(x, n) || !need(y, n) || !need(z, n) || !need(q, n)) return fail(RBE_EINVAL, "NULL position/charge array");
  if (!need(m, P) || !need(rho, P)) return fail(RBE_EINVAL, "NULL m or rho array");
  hipError_t e = launch_rho(shape_of(p), view_of(p, ws), x, y, z, q, m, nullptr, rho, 0,
                            static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "rho pass launch");
  return RBE_OK;
}

rbe_status rbe_kspace_force(const rbe_plan* p, const double* x, const double* y, const double* z,
                            const double* q, const int32_t* m, const double* w, const double* rho,
                            void* F, double* U, void* ws, void* stream) {
  rbe_status st = check_common(p, ws);
  if (st != RBE_OK) return st;
  const int64_t n = p->n_total(), P = p->p_total();
  if (!need(x, n) || !need(y, n) || !need(z, n) || !need(q, n) || !need(F, n))
    return fail(RBE_EINVAL, "NULL position/charge/force array");
  if (!need(m, P) || !need(w, P) || !need(rho, P)) return fail(RBE_EINVAL, "NULL m, w or rho array");
  if (U == nullptr) return fail(RBE_EINVAL, "U is NULL");
  hipError_t e = launch_force(shape_of(p), view_of(p, ws), x, y, z, q, m, w, rho, F, U, nullptr, 0,
                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "force pass launch");
  return RBE_OK;
}

rbe_status rbe_kspace_virial(const rbe_plan* p, const int32_t* m, const double* w, const double* rho, double* W,
                             void* ws, void* stream) {
  rbe_status st = check_common(p, ws);
  if (st != RBE_OK) return st;
  const int64_t P = p->p_total();
  if (!need(m, P) || !need(w, P) || !need(rho, P)) return fail(RBE_EINVAL, "NULL m, w or rho array");
  if (W == nullptr) return fail(RBE_EINVAL, "W is NULL");
  hipError_t e = launch_virial(shape_of(p), view_of(p, ws), m, w, rho, W, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "virial launch");
  return RBE_OK;
}

rbe_status rbe_kspace_vjp(const rbe_plan* p, const double* x, const double* y, const double* z,
                          const double* q, const int32_t* m, const double* w, const double* rho,
                          const double* gU, const void* gF, double* gr, double* gq, void* ws, void* stream) {
  rbe_status st = check_common(p, ws);
  if (st != RBE_OK) return st;
  const int64_t n = p->n_total(), P = p->p_total();
  if (!need(x, n) || !need(y, n) || !need(z, n) || !need(q, n) || !need(gF, n) || !need(gr, n) || !need(gq, n))
    return fail(RBE_EINVAL, "NULL particle array");
  if (!need(m, P) || !need(w, P) || !need(rho, P)) return fail(RBE_EINVAL, "NULL m, w or rho array");
  if (gU == nullptr) return fail(RBE_EINVAL, "gU is NULL");
  hipError_t e = launch_vjp(shape_of(p), view_of(p, ws), x, y, z, q, m, w, rho, gU, gF, gr, gq,
                            static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "vjp launch");
  return RBE_OK;
}

rbe_status rbe_plan_tune(rbe_plan* p, const double* x, const double* y, const double* z, const double* q,
                         const int32_t* m, const double* w, double* rho, void* F, double* U, void* ws,
                         void* stream, int32_t reps, int32_t* rho_variant, int32_t* force_variant,
                         int32_t* rho_grid_cap, double* rho_ms, double* force_ms) {
  rbe_status st = check_common(p, ws);
  if (st != RBE_OK) return st;
  if (reps <= 0) return fail(RBE_EINVAL, "reps must be > 0");
  hipEvent_t ev[4];
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(RBE_EHIP, "hipEventCreate failed");
  hipEvent_t saved[4] = {p->ev[0], p->ev[1], p->ev[2], p->ev[3]};
  // Time the two kernels the way an evaluation runs them: each rho pass follows a
  // force pass and each force pass follows a rho pass (a kernel's speed depends on
  // what ran before it), with events placed right around each kernel.
  auto measure = [&](float* rho_out, float* force_out) -> rbe_status {
    rbe_status r = rbe_plan_upload(p, ws, stream);
    float tr = 0.f, tf = 0.f;
    for (int i = 0; i <= reps && r == RBE_OK; ++i) {   // the first round is a warm-up
      p->ev[0] = ev[0]; p->ev[1] = ev[1]; p->ev[2] = ev[2]; p->ev[3] = ev[3];
      r = rbe_structure_factor(p, x, y, z, q, m, rho, ws, stream);
      if (r == RBE_OK) r = rbe_kspace_force(p, x, y, z, q, m, w, rho, F, U, ws, stream);
      p->ev[0] = p->ev[1] = p->ev[2] = p->ev[3] = nullptr;
      if (r != RBE_OK) break;
      if (hipEventSynchronize(ev[3]) != hipSuccess) { r = fail(RBE_EHIP, "event wait failed"); break; }
      float a = 0.f, b = 0.f;
      if (hipEventElapsedTime(&a, ev[0], ev[1]) != hipSuccess || hipEventElapsedTime(&b, ev[2], ev[3]) != hipSuccess) {
        r = fail(RBE_EHIP, "hipEventElapsedTime failed");
        break;
      }
      if (i > 0) { tr += a; tf += b; }
    }
    *rho_out = tr / (float)reps;
    *force_out = tf / (float)reps;
    return r;
  };
  const int nr = p->precision == RBE_FP64 ? kNumRhoVariantsF64 : kNumRhoVariantsF32;
  const int orig_r = p->rho_variant, orig_f = p->force_variant;
  const int32_t orig_clamp = p->rho_clamp, orig_cap = p->rho_grid_cap;
  int best_r = p->rho_variant, best_f = p->force_variant;
  float best_rms = 1e30f, best_fms = 1e30f;
  rbe_status r = RBE_OK;
  p->rho_grid_cap = 0;
  int32_t best_clamp = p->rho_clamp;
  for (int v = 0; v < nr && r == RBE_OK; ++v) {
    p->rho_variant = v;
    build_layout(p);
    for (int32_t clamp = 1; clamp >= 0 && r == RBE_OK; --clamp) {
      p->rho_clamp = clamp;
      float a = 0.f, b = 0.f;
      r = measure(&a, &b);
      if (r == RBE_OK && a < best_rms) { best_rms = a; best_r = v; best_clamp = clamp; }
    }
  }
  p->rho_variant = best_r;
  p->rho_clamp = best_clamp;
  for (int v = 0; v < kNumForceVariants && r == RBE_OK; ++v) {
    p->force_variant = v;
    build_layout(p);
    float a = 0.f, b = 0.f;
    r = measure(&a, &b);
    if (r == RBE_OK && b < best_fms) { best_fms = b; best_f = v; }
  }
  p->force_variant = best_f;
  for (int i = 0; i < 4; ++i) {
    (void)hipEventDestroy(ev[i]);
    p->ev[i] = saved[i];
  }
  if (r != RBE_OK) {
    // keep the plan and the workspace consistent: back to the variants the call started
    // with, uploaded again (the workspace holds the tables of the last variant timed)
    const std::string why = g_last_error;
    p->rho_variant = orig_r;
    p->force_variant = orig_f;
    p->rho_clamp = orig_clamp;
    p->rho_grid_cap = orig_cap;
    build_layout(p);
    (void)rbe_plan_upload(p, ws, stream);
    g_last_error = why;
    return r;
  }
  build_layout(p);
  r = rbe_plan_upload(p, ws, stream);
  if (r != RBE_OK) return r;
  if (rho_variant) *rho_variant = best_r;
  if (force_variant) *force_variant = best_f;
  if (rho_grid_cap) *rho_grid_cap = p->rho_grid_cap;
  if (rho_ms) *rho_ms = best_rms;
  if (force_ms) *force_ms = best_fms;
  return RBE_OK;
}

rbe_status rbe_plan_set_grid_caps(rbe_plan* p, int32_t rho_cap, int32_t force_cap) {
  if (!p) return fail(RBE_EINVAL, "plan is NULL");
  if (rho_cap < 0 || force_cap < 0) return fail(RBE_EINVAL, "grid caps must be >= 0");
  p->rho_grid_cap = rho_cap;
  p->force_grid_cap = force_cap;
  return RBE_OK;
}

rbe_status rbe_plan_set_timing_events(rbe_plan* p, void* rho_begin, void* rho_end, void* force_begin,
                                      void* force_end) {
  if (!p) return fail(RBE_EINVAL, "plan is NULL");
  p->ev[0] = static_cast<hipEvent_t>(rho_begin);
  p->ev[1] = static_cast<hipEvent_t>(rho_end);
  p->ev[2] = static_cast<hipEvent_t>(force_begin);
  p->ev[3] = static_cast<hipEvent_t>(force_end);
  return RBE_OK;
}

namespace {

// Arguments of one whole evaluation (device sampling, rho pass, reduction, force pass).
rbe_status check_evaluation(const rbe_plan* p, const double* x, const double* y, const double* z, const double* q,
                            const int32_t* m, const double* w, const double* rho, const void* F, const double* U,
                            void* ws) {
  rbe_status st = check_common(p, ws);
  if (st != RBE_OK) return st;
  if (!p->sampler_ok) return fail(RBE_EINVAL, "a system's zero-vector probability exceeds 1/2 (box too small for alpha)");
  const int64_t n = p->n_total(), P = p->p_total();
  if (!need(x, n) || !need(y, n) || !need(z, n) || !need(q, n) || !need(F, n))
    return fail(RBE_EINVAL, "NULL position/charge/force array");
  if (!need(m, P) || !need(w, P) || !need(rho, P) || U == nullptr) return fail(RBE_EINVAL, "NULL m, w, rho or U");
  return RBE_OK;
}

hipError_t enqueue_evaluation(const rbe_plan* p, uint64_t seed, uint64_t stream_base, uint64_t* step_counter,
                              const double* x, const double* y, const double* z, const double* q, int32_t* m,
                              double* w, double* rho, void* F, double* U, void* ws, hipStream_t st) {
  const LaunchShape shape = shape_of(p);
  const WsView view = view_of(p, ws);
  hipError_t e = launch_sample(shape, view, seed, stream_base, step_counter, m, w, st);
  // the reduction writes the force rows, so the force pass needs no kernel of its own for them
  if (e == hipSuccess) e = launch_rho(shape, view, x, y, z, q, m, w, rho, 1, st);
  if (e == hipSuccess) e = launch_force(shape, view, x, y, z, q, m, w, rho, F, U, step_counter, 1, st);
  return e;
}

// ---------------------------------------------------------------- evaluation without allocation

// Device scratch of rbe_evaluate_static: the plan tables, tile partial sums and force rows
// that rbe_evaluate keeps in the caller's workspace.  Every device the library runs on
// holds its own copy from the time the code object is loaded until the process ends.
// In host code `scratch` names a host-side stand-in, never the device memory: the device
// address comes from hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Per device: the address of its scratch (null until looked up) and the layout whose
// tables were last uploaded into it (0: none).
struct StaticScratch {
  void* ptr = nullptr;
  uint64_t layout_id = 0;
};
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
StaticScratch g_static[kMaxStaticDevices];

}  // namespace

rbe_status rbe_evaluate(const rbe_plan* p, uint64_t seed, uint64_t stream_base, uint64_t* step_counter,
                        const double* x, const double* y, const double* z, const double* q, int32_t* m, double* w,
                        double* rho, void* F, double* U, void* ws, void* stream) {
  rbe_status st = check_evaluation(p, x, y, z, q, m, w, rho, F, U, ws);
  if (st != RBE_OK) return st;
  hipError_t e = enqueue_evaluation(p, seed, stream_base, step_counter, x, y, z, q, m, w, rho, F, U, ws,
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "rbe_evaluate launch");
  return RBE_OK;
}

rbe_status rbe_graph_create(const rbe_plan* p, uint64_t seed, uint64_t stream_base, uint64_t* step_counter,
                            const double* x, const double* y, const double* z, const double* q, int32_t* m,
                            double* w, double* rho, void* F, double* U, void* ws, rbe_graph** out) {
  if (out == nullptr) return fail(RBE_EINVAL, "out is NULL");
  *out = nullptr;
  rbe_status st = check_evaluation(p, x, y, z, q, m, w, rho, F, U, ws);
  if (st != RBE_OK) return st;
  hipStream_t cs;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    hipError_t le = enqueue_evaluation(p, seed, stream_base, step_counter, x, y, z, q, m, w, rho, F, U, ws, cs);
    e = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess) e = le;
  }
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(e, "graph capture");
  }
  rbe_graph* g = new rbe_graph();
  g->graph = graph;
  g->exec = exec;
  *out = g;
  return RBE_OK;
}

rbe_status rbe_graph_launch(const rbe_graph* g, void* stream) {
  if (g == nullptr) return fail(RBE_EINVAL, "graph is NULL");
  hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return RBE_OK;
}

void rbe_graph_destroy(rbe_graph* g) {
  if (g == nullptr) return;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
}

rbe_status rbe_evaluate_static(const rbe_plan* p, uint64_t seed, uint64_t stream_base, uint64_t* step_counter,
                               const double* x, const double* y, const double* z, const double* q, int32_t* m,
                               double* w, double* rho, void* F, double* U, void* stream) {
  if (p == nullptr) return fail(RBE_EINVAL, "plan is NULL");
  if (p->total > kStaticScratchBytes)
    return fail(RBE_EWORKSPACE,
                "the plan needs %zu bytes of scratch, more than the %zu bytes rbe_evaluate_static holds "
                "(use rbe_evaluate with a workspace)",
                p->total, kStaticScratchBytes);
  rbe_status st = device_ok();
  if (st != RBE_OK) return st;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxStaticDevices)
    return fail(RBE_EUNSUPPORTED, "device %d is beyond the %d devices rbe_evaluate_static serves", dev,
                kMaxStaticDevices);
  void* ws = nullptr;
  bool upload = false;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticScratch& slot = g_static[dev];
    if (slot.ptr == nullptr) {
      // first call on this device, which is current: the device address of its copy
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
      if (ptr == nullptr) return fail(RBE_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
      slot.ptr = ptr;
    }
    ws = slot.ptr;
    upload = slot.layout_id != p->layout_id;
  }
  st = check_evaluation(p, x, y, z, q, m, w, rho, F, U, ws);
  if (st != RBE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (upload) {
    st = enqueue_upload(p, ws, s);
    if (st != RBE_OK) return st;
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[dev].layout_id = p->layout_id;
  }
  // every scratch region the evaluation reads (partials, force rows) is written earlier in
  // the same evaluation, so nothing needs clearing between calls
  e = enqueue_evaluation(p, seed, stream_base, step_counter, x, y, z, q, m, w, rho, F, U, ws, s);
  if (e != hipSuccess) return hip_fail(e, "rbe_evaluate_static launch");
  return RBE_OK;
}

rbe_status rbe_sample_k_device(const rbe_plan* p, uint64_t seed, uint64_t stream_id, int32_t* m, double* w,
                               void* ws, void* stream) {
  rbe_status st = check_common(p, ws);
  if (st != RBE_OK) return st;
  if (!p->sampler_ok) return fail(RBE_EINVAL, "a system's zero-vector probability exceeds 1/2 (box too small for alpha)");
  const int64_t P = p->p_total();
  if (!need(m, P) || !need(w, P)) return fail(RBE_EINVAL, "NULL m or w array");
  hipError_t e = launch_sample(shape_of(p), view_of(p, ws), seed, stream_id, nullptr, m, w,
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "sampler launch");
  return RBE_OK;
}

}  // extern "C"
