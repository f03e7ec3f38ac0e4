// gfx950 kernels of the RBE k-space path: structure factor, cross-tile reduction,
// force/energy, adjoint (VJP) passes and the on-device wave-vector sampler.
//
// Data flow of one evaluation (Algorithm 1 steps 2-4):
//   rho pass   : work item = (particle tile, range of wave vectors); one wave64 per item.
//                Each lane keeps NPL particles in registers, loops over chunks of KC
//                wave vectors, accumulates q cos / q sin per lane, then reduce-scatters
//                the 2*KC sums across the wave and writes one FP64 partial per
//                (wave vector, tile).
//   reduce     : one wave per wave vector sums its tile partials in a fixed order (FP64).
//   force pass : work item = particle range; 256-thread blocks; the per-k table
//                (m, c_l S_l, c_l C_l) is built in LDS from rho and w; each lane
//                streams NPLF particles over all wave vectors.  The first block of a
//                system also writes its energy.
//
// Phases.  FP32-mixed: s = r/L mod 1 is held as a 32-bit fixed-point fraction u, so
// the phase in turns m.s mod 1 is the exact wrap-around integer m.u mod 2^32.  Its top
// 23 bits become the mantissa of a float in [1, 2), which v_sin_f32 / v_cos_f32 take
// in revolutions.  Dropping the low 9 bits rotates every phase by half a step on
// average (pi 2^-23 rad); the reduction undoes that rotation on rho and the force table
// re-applies it, so F and U carry no bias from it.
// FP64: t = m.s - rint(m.s) in turns and sin/cos(2 pi t) from near-minimax polynomials
// after an exact quarter-turn reduction.
#include <hip/hip_runtime.h>

#include "philox.h"
#include "rbe_internal.h"
#include "sincos_coeffs.h"

namespace rbe {

const RhoVariant kRhoVariantsF32[kNumRhoVariantsF32] = {{16, 8, 56}, {8, 8, 104}, {16, 8, 104}, {8, 8, 56}};
const RhoVariant kRhoVariantsF64[kNumRhoVariantsF64] = {{8, 4, 52}, {4, 4, 100}, {8, 4, 100}};
const ForceVariant kForceVariants[kNumForceVariants] = {{1}, {2}, {4}};

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kFourPi = 12.566370614359172953850573533118;
constexpr int kTabChunk = 256;

// ------------------------------------------------------------------ phase helpers

// round(frac(x / L) * 2^32) as a 32-bit fixed-point fraction of a turn.
__device__ inline uint32_t fixed_fraction(double x, double invL) {
  const double v = x * invL;
  const double f = v - floor(v);
  const double r = fmin(fma(f, 4294967296.0, 0.5), 4294967295.0);
  return (uint32_t)r;
}

// Top 23 bits of a phase (turns * 2^32) as the float 1 + t/2^32 in [1, 2): revolutions.
__device__ inline float turns_arg(uint32_t t) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, t, 9u));
}

__device__ inline uint32_t phase_u32(int32_t mx, int32_t my, int32_t mz, uint32_t ux, uint32_t uy, uint32_t uz) {
  return (uint32_t)mx * ux + (uint32_t)my * uy + (uint32_t)mz * uz;
}

// sin and cos of 2 pi r for |r| <= 1/2 (turns), FP64.
__device__ inline void sincos_turns(double r, double* s, double* c) {
  const double q4 = rint(4.0 * r);
  const double f = fma(q4, -0.25, r);
  const double f2 = f * f;
  double ps = kSin[kSinTerms - 1];
#pragma unroll
  for (int j = kSinTerms - 2; j >= 0; --j) ps = fma(ps, f2, kSin[j]);
  double pc = kCos[kCosTerms - 1];
#pragma unroll
  for (int j = kCosTerms - 2; j >= 0; --j) pc = fma(pc, f2, kCos[j]);
  const double sn = ps * f;
  const int n = (int)q4;
  double so = (n & 1) ? pc : sn;
  double co = (n & 1) ? sn : pc;
  so = (n & 2) ? -so : so;
  co = ((n + 1) & 2) ? -co : co;
  *s = so;
  *c = co;
}

// phase of m.s in turns, reduced to [-1/2, 1/2].
__device__ inline double phase_f64(double mx, double my, double mz, double sx, double sy, double sz) {
  const double t = fma(mx, sx, fma(my, sy, mz * sz));
  return t - rint(t);
}

// ------------------------------------------------------------------ wave reductions

__device__ inline int bitrev(int v, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
  return r;
}

template <int V> struct Log2 { static constexpr int value = 1 + Log2<V / 2>::value; };
template <> struct Log2<1> { static constexpr int value = 0; };

// Recursive-halving reduce-scatter of V values per lane over the 64 lanes of a wave.
// Afterwards v[0] of lane L holds the wave sum of value index bitrev(L mod V).
template <int V, typename T>
__device__ inline void wave_reduce_scatter(T (&v)[V], int lane) {
  static_assert((V & (V - 1)) == 0 && V <= 64, "V must be a power of two <= 64");
#pragma unroll
  for (int lvl = 0, half = V / 2; half >= 1; ++lvl, half /= 2) {
    const int b = 1 << lvl;
    const bool upper = (lane & b) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const T send = upper ? v[i] : v[i + half];
      const T keep = upper ? v[i + half] : v[i];
      v[i] = keep + __shfl_xor(send, b, 64);
    }
  }
#pragma unroll
  for (int b = V; b < 64; b *= 2) v[0] += __shfl_xor(v[0], b, 64);
}

// ------------------------------------------------------------------ rho pass, FP32-mixed

// With VJP, the same pass forms X_l + i Y_l = sum_i q_i (gF_i . m_l) exp(i theta_il)
// (adjoint pass B1; the 2 pi / L of k_l is applied when the adjoint table is built).
template <int NPL, int KC, bool CACHE, bool VJP>
__global__ __launch_bounds__(64) void rho_f32_kernel(WsView w, const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ q,
                                                     const int32_t* __restrict__ m,
                                                     const float* __restrict__ gF, int64_t n_total) {
  const RhoItem it = w.rho_items[blockIdx.x];
  const SysDesc sd = w.sys[it.sys];
  const int lane = threadIdx.x;
  const int first = it.tile * (64 * NPL);
  const int cnt = min(64 * NPL, sd.n - first);
  const double invL = 1.0 / sd.L;

  uint32_t ux[NPL], uy[NPL], uz[NPL];
  float qv[NPL], qgx[VJP ? NPL : 1], qgy[VJP ? NPL : 1], qgz[VJP ? NPL : 1];
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int li = j * 64 + lane;
    if (li < cnt) {
      const int64_t gi = sd.n_off + first + li;
      ux[j] = fixed_fraction(x[gi], invL);
      uy[j] = fixed_fraction(y[gi], invL);
      uz[j] = fixed_fraction(z[gi], invL);
      qv[j] = (float)q[gi];
      if (VJP) {
        qgx[j] = qv[j] * gF[gi];
        qgy[j] = qv[j] * gF[n_total + gi];
        qgz[j] = qv[j] * gF[2 * n_total + gi];
      }
    } else {
      ux[j] = uy[j] = uz[j] = 0u;
      qv[j] = 0.0f;
      if (VJP) qgx[j] = qgy[j] = qgz[j] = 0.0f;
    }
  }
  double* part = w.partials + 2 * sd.part_off;
  const int32_t* mk = m + 3 * (sd.k_off + it.k0);

  for (int kc = 0; kc < it.nk; kc += KC) {
    int32_t mx[KC], my[KC], mz[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const bool ok = kc + c < it.nk;
      const int kk = ok ? kc + c : it.nk - 1;
      mx[c] = ok ? mk[3 * kk] : 0;
      my[c] = ok ? mk[3 * kk + 1] : 0;
      mz[c] = ok ? mk[3 * kk + 2] : 0;
    }
    float acc[2 * KC];
#pragma unroll
    for (int c = 0; c < 2 * KC; ++c) acc[c] = 0.0f;
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const float a = turns_arg(phase_u32(mx[c], my[c], mz[c], ux[j], uy[j], uz[j]));
        const float sn = __builtin_amdgcn_sinf(a);
        const float cs = __builtin_amdgcn_cosf(a);
        float wt = qv[j];
        if (VJP) wt = fmaf(qgx[j], (float)mx[c], fmaf(qgy[j], (float)my[c], qgz[j] * (float)mz[c]));
        acc[c] = fmaf(wt, cs, acc[c]);
        acc[KC + c] = fmaf(wt, sn, acc[KC + c]);
        if (CACHE) {
          const int li = j * 64 + lane;
          if (li < cnt && kc + c < it.nk) {
            float2* cp = reinterpret_cast<float2*>(w.cache) + sd.cache_off +
                         (int64_t)(it.k0 + kc + c) * sd.n + first + li;
            *cp = make_float2(cs, sn);
          }
        }
      }
    }
    wave_reduce_scatter<2 * KC>(acc, lane);
    if (lane < 2 * KC) {
      const int vi = bitrev(lane, Log2<2 * KC>::value);
      const int c = vi % KC;
      const int comp = vi / KC;
      if (kc + c < it.nk) {
        const int64_t kl = it.k0 + kc + c;
        part[2 * (kl * sd.ntiles + it.tile) + comp] = (double)acc[0];
      }
    }
  }
}

// ------------------------------------------------------------------ rho pass, FP64

template <int NPL, int KC, bool VJP>
__global__ __launch_bounds__(64) void rho_f64_kernel(WsView w, const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ q,
                                                     const int32_t* __restrict__ m,
                                                     const double* __restrict__ gF, int64_t n_total) {
  const RhoItem it = w.rho_items[blockIdx.x];
  const SysDesc sd = w.sys[it.sys];
  const int lane = threadIdx.x;
  const int first = it.tile * (64 * NPL);
  const int cnt = min(64 * NPL, sd.n - first);
  const double invL = 1.0 / sd.L;

  double sx[NPL], sy[NPL], sz[NPL], qv[NPL];
  double qgx[VJP ? NPL : 1], qgy[VJP ? NPL : 1], qgz[VJP ? NPL : 1];
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int li = j * 64 + lane;
    if (li < cnt) {
      const int64_t gi = sd.n_off + first + li;
      const double vx = x[gi] * invL, vy = y[gi] * invL, vz = z[gi] * invL;
      sx[j] = vx - floor(vx);
      sy[j] = vy - floor(vy);
      sz[j] = vz - floor(vz);
      qv[j] = q[gi];
      if (VJP) {
        qgx[j] = qv[j] * gF[gi];
        qgy[j] = qv[j] * gF[n_total + gi];
        qgz[j] = qv[j] * gF[2 * n_total + gi];
      }
    } else {
      sx[j] = sy[j] = sz[j] = 0.0;
      qv[j] = 0.0;
      if (VJP) qgx[j] = qgy[j] = qgz[j] = 0.0;
    }
  }
  double* part = w.partials + 2 * sd.part_off;
  const int32_t* mk = m + 3 * (sd.k_off + it.k0);

  for (int kc = 0; kc < it.nk; kc += KC) {
    double mx[KC], my[KC], mz[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const bool ok = kc + c < it.nk;
      const int kk = ok ? kc + c : it.nk - 1;
      mx[c] = ok ? (double)mk[3 * kk] : 0.0;
      my[c] = ok ? (double)mk[3 * kk + 1] : 0.0;
      mz[c] = ok ? (double)mk[3 * kk + 2] : 0.0;
    }
    double acc[2 * KC];
#pragma unroll
    for (int c = 0; c < 2 * KC; ++c) acc[c] = 0.0;
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        double sn, cs;
        sincos_turns(phase_f64(mx[c], my[c], mz[c], sx[j], sy[j], sz[j]), &sn, &cs);
        double wt = qv[j];
        if (VJP) wt = fma(qgx[j], mx[c], fma(qgy[j], my[c], qgz[j] * mz[c]));
        acc[c] = fma(wt, cs, acc[c]);
        acc[KC + c] = fma(wt, sn, acc[KC + c]);
      }
    }
    wave_reduce_scatter<2 * KC>(acc, lane);
    if (lane < 2 * KC) {
      const int vi = bitrev(lane, Log2<2 * KC>::value);
      const int c = vi % KC;
      const int comp = vi / KC;
      if (kc + c < it.nk) {
        const int64_t kl = it.k0 + kc + c;
        part[2 * (kl * sd.ntiles + it.tile) + comp] = acc[0];
      }
    }
  }
}

// ------------------------------------------------------------------ cross-tile reduction

// One wave per wave vector: out[g] = sum over the system's tiles of partial[g][tile],
// lanes stride the tiles, then a fixed butterfly; optionally rotated by exp(i delta).
__global__ __launch_bounds__(kReduceBlock) void reduce_kernel(WsView w, int64_t p_total,
                                                              double* __restrict__ out,
                                                              double rot_c, double rot_s) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (kReduceBlock / 64) + (threadIdx.x >> 6);
  if (g >= p_total) return;
  const SysDesc sd = w.sys[w.ksys[g]];
  const int64_t l = g - sd.k_off;
  const double* src = w.partials + 2 * (sd.part_off + l * sd.ntiles);
  double re = 0.0, im = 0.0;
  for (int t = lane; t < sd.ntiles; t += 64) {
    re += src[2 * t];
    im += src[2 * t + 1];
  }
#pragma unroll
  for (int b = 32; b >= 1; b >>= 1) {
    re += __shfl_xor(re, b, 64);
    im += __shfl_xor(im, b, 64);
  }
  if (lane == 0) {
    out[2 * g] = re * rot_c - im * rot_s;
    out[2 * g + 1] = re * rot_s + im * rot_c;
  }
}

// ------------------------------------------------------------------ energy helper

// Fixed-order block sum of one double per thread; thread 0 gets the total.
__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kForceBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// ------------------------------------------------------------------ force pass, FP32-mixed

struct TabF32 {
  int32_t mx, my, mz;
  float a;              // c_l * S'_l
  float fx, fy, fz;     // m_l as float
  float b;              // c_l * C'_l
};

template <int NPLF, bool CACHED>
__global__ __launch_bounds__(kForceBlock) void force_f32_kernel(
    WsView w, int64_t n_total, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ q, const int32_t* __restrict__ m,
    const double* __restrict__ wk, const double* __restrict__ rho, float* __restrict__ F,
    double* __restrict__ U, double rot_c, double rot_s) {
  __shared__ TabF32 tab[kTabChunk];
  __shared__ double red[kForceBlock];
  const ForceItem it = w.force_items[blockIdx.x];
  const SysDesc sd = w.sys[it.sys];
  const int tid = threadIdx.x;
  const double invL = 1.0 / sd.L;
  const double kscale = kTwoPi * invL;
  const double vol = sd.L * sd.L * sd.L;

  uint32_t ux[NPLF], uy[NPLF], uz[NPLF];
  float fx[NPLF], fy[NPLF], fz[NPLF];
  int li[NPLF];
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    li[j] = it.p0 + j * kForceBlock + tid;
    const bool ok = j * kForceBlock + tid < it.np;
    if (ok && !CACHED) {
      const int64_t gi = sd.n_off + li[j];
      ux[j] = fixed_fraction(x[gi], invL);
      uy[j] = fixed_fraction(y[gi], invL);
      uz[j] = fixed_fraction(z[gi], invL);
    } else {
      ux[j] = uy[j] = uz[j] = 0u;
    }
    fx[j] = fy[j] = fz[j] = 0.0f;
  }
  double usum = 0.0;
  for (int t0 = 0; t0 < sd.p; t0 += kTabChunk) {
    const int cnt = min(kTabChunk, sd.p - t0);
    __syncthreads();
    for (int e = tid; e < cnt; e += kForceBlock) {
      const int64_t g = sd.k_off + t0 + e;
      const int32_t mx = m[3 * g], my = m[3 * g + 1], mz = m[3 * g + 2];
      const double k2 = kscale * kscale * ((double)mx * mx + (double)my * my + (double)mz * mz);
      const double c = (k2 > 0.0) ? wk[g] * kFourPi / (vol * k2) : 0.0;
      const double C = rho[2 * g], S = rho[2 * g + 1];
      const double Cr = C * rot_c + S * rot_s;
      const double Sr = S * rot_c - C * rot_s;
      TabF32 tb;
      tb.mx = mx; tb.my = my; tb.mz = mz;
      tb.a = (float)(c * Sr);
      tb.b = (float)(c * Cr);
      tb.fx = (float)mx; tb.fy = (float)my; tb.fz = (float)mz;
      tab[e] = tb;
      if (it.flags & 1) usum += 0.5 * c * (C * C + S * S);
    }
    __syncthreads();
    for (int e = 0; e < cnt; ++e) {
      const TabF32 tb = tab[e];
#pragma unroll
      for (int j = 0; j < NPLF; ++j) {
        float sn, cs;
        if (CACHED) {
          if (j * kForceBlock + tid < it.np) {
            const float2 v = reinterpret_cast<const float2*>(w.cache)[sd.cache_off + (int64_t)(t0 + e) * sd.n + li[j]];
            cs = v.x;
            sn = v.y;
          } else {
            cs = sn = 0.0f;
          }
        } else {
          const float a = turns_arg(phase_u32(tb.mx, tb.my, tb.mz, ux[j], uy[j], uz[j]));
          sn = __builtin_amdgcn_sinf(a);
          cs = __builtin_amdgcn_cosf(a);
        }
        const float g = tb.a * cs - tb.b * sn;
        fx[j] = fmaf(g, tb.fx, fx[j]);
        fy[j] = fmaf(g, tb.fy, fy[j]);
        fz[j] = fmaf(g, tb.fz, fz[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    if (j * kForceBlock + tid < it.np) {
      const int64_t gi = sd.n_off + li[j];
      const double s = -q[gi] * kscale;
      F[gi] = (float)(s * fx[j]);
      F[n_total + gi] = (float)(s * fy[j]);
      F[2 * n_total + gi] = (float)(s * fz[j]);
    }
  }
  if (it.flags & 1) {
    const double tot = block_sum(usum, red);
    if (tid == 0) U[it.sys] = tot;
  }
}

// ------------------------------------------------------------------ force pass, FP64

struct TabF64 {
  double mx, my, mz;
  double a;   // c_l * S_l
  double b;   // c_l * C_l
};

template <int NPLF>
__global__ __launch_bounds__(kForceBlock) void force_f64_kernel(
    WsView w, int64_t n_total, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ q, const int32_t* __restrict__ m,
    const double* __restrict__ wk, const double* __restrict__ rho, double* __restrict__ F,
    double* __restrict__ U) {
  __shared__ TabF64 tab[kTabChunk];
  __shared__ double red[kForceBlock];
  const ForceItem it = w.force_items[blockIdx.x];
  const SysDesc sd = w.sys[it.sys];
  const int tid = threadIdx.x;
  const double invL = 1.0 / sd.L;
  const double kscale = kTwoPi * invL;
  const double vol = sd.L * sd.L * sd.L;

  double sx[NPLF], sy[NPLF], sz[NPLF], fx[NPLF], fy[NPLF], fz[NPLF];
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    const bool ok = j * kForceBlock + tid < it.np;
    if (ok) {
      const int64_t gi = sd.n_off + it.p0 + j * kForceBlock + tid;
      const double vx = x[gi] * invL, vy = y[gi] * invL, vz = z[gi] * invL;
      sx[j] = vx - floor(vx);
      sy[j] = vy - floor(vy);
      sz[j] = vz - floor(vz);
    } else {
      sx[j] = sy[j] = sz[j] = 0.0;
    }
    fx[j] = fy[j] = fz[j] = 0.0;
  }
  double usum = 0.0;
  for (int t0 = 0; t0 < sd.p; t0 += kTabChunk) {
    const int cnt = min(kTabChunk, sd.p - t0);
    __syncthreads();
    for (int e = tid; e < cnt; e += kForceBlock) {
      const int64_t g = sd.k_off + t0 + e;
      const int32_t mx = m[3 * g], my = m[3 * g + 1], mz = m[3 * g + 2];
      const double k2 = kscale * kscale * ((double)mx * mx + (double)my * my + (double)mz * mz);
      const double c = (k2 > 0.0) ? wk[g] * kFourPi / (vol * k2) : 0.0;
      const double C = rho[2 * g], S = rho[2 * g + 1];
      TabF64 tb;
      tb.mx = mx; tb.my = my; tb.mz = mz;
      tb.a = c * S;
      tb.b = c * C;
      tab[e] = tb;
      if (it.flags & 1) usum += 0.5 * c * (C * C + S * S);
    }
    __syncthreads();
    for (int e = 0; e < cnt; ++e) {
      const TabF64 tb = tab[e];
#pragma unroll
      for (int j = 0; j < NPLF; ++j) {
        double sn, cs;
        sincos_turns(phase_f64(tb.mx, tb.my, tb.mz, sx[j], sy[j], sz[j]), &sn, &cs);
        const double g = tb.a * cs - tb.b * sn;
        fx[j] = fma(g, tb.mx, fx[j]);
        fy[j] = fma(g, tb.my, fy[j]);
        fz[j] = fma(g, tb.mz, fz[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    if (j * kForceBlock + tid < it.np) {
      const int64_t gi = sd.n_off + it.p0 + j * kForceBlock + tid;
      const double s = -q[gi] * kscale;
      F[gi] = s * fx[j];
      F[n_total + gi] = s * fy[j];
      F[2 * n_total + gi] = s * fz[j];
    }
  }
  if (it.flags & 1) {
    const double tot = block_sum(usum, red);
    if (tid == 0) U[it.sys] = tot;
  }
}


// ------------------------------------------------------------------ adjoint pass B2

// With a_l = c_l / 2, Chat + i Shat = 2 a_l (gU rho_l - i (X_l + i Y_l)) and
// Z2 = 2 a_l (2 pi / L) rho_l, every adjoint term is a real or imaginary part of
// exp(-i theta) Z:
//   dL/dr_i = q_i (2 pi / L) sum_l m_l [Im(e^{-i th} Z1) + (gF_i . m_l) Re(e^{-i th} Z2)]
//   dL/dq_i =                sum_l     [Re(e^{-i th} Z1) - (gF_i . m_l) Im(e^{-i th} Z2)]
struct AdjTab {
  double z1r, z1i, z2r, z2i;
};

// Builds the adjoint row of wave vector g (FP64); X + iY = xy[g] * (2 pi / L).
__device__ inline AdjTab adjoint_row(const SysDesc& sd, int64_t g, const int32_t* m, const double* wk,
                                     const double* rho, const double* xy, double gu, double kscale,
                                     double vol) {
  const int32_t mx = m[3 * g], my = m[3 * g + 1], mz = m[3 * g + 2];
  const double k2 = kscale * kscale * ((double)mx * mx + (double)my * my + (double)mz * mz);
  const double c = (k2 > 0.0) ? wk[g] * kFourPi / (vol * k2) : 0.0;
  const double C = rho[2 * g], S = rho[2 * g + 1];
  const double X = xy[2 * g] * kscale, Y = xy[2 * g + 1] * kscale;
  AdjTab t;
  t.z1r = c * (gu * C + Y);
  t.z1i = c * (gu * S - X);
  t.z2r = c * kscale * C;
  t.z2i = c * kscale * S;
  return t;
}

struct TabAdjF32 {
  int32_t mx, my, mz;
  float fx, fy, fz;
  float z1r, z1i, z2r, z2i;
};

template <int NPLF>
__global__ __launch_bounds__(kForceBlock) void vjp_b2_f32_kernel(
    WsView w, int64_t n_total, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ q, const int32_t* __restrict__ m,
    const double* __restrict__ wk, const double* __restrict__ rho, const double* __restrict__ gU,
    const float* __restrict__ gF, float* __restrict__ gr, float* __restrict__ gq, double rot_c,
    double rot_s) {
  __shared__ TabAdjF32 tab[kTabChunk];
  const ForceItem it = w.force_items[blockIdx.x];
  const SysDesc sd = w.sys[it.sys];
  const int tid = threadIdx.x;
  const double invL = 1.0 / sd.L;
  const double kscale = kTwoPi * invL;
  const double vol = sd.L * sd.L * sd.L;
  const double gu = gU[it.sys];

  uint32_t ux[NPLF], uy[NPLF], uz[NPLF];
  float gx[NPLF], gy[NPLF], gz[NPLF], rx[NPLF], ry[NPLF], rz[NPLF], rq[NPLF];
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    const bool ok = j * kForceBlock + tid < it.np;
    if (ok) {
      const int64_t gi = sd.n_off + it.p0 + j * kForceBlock + tid;
      ux[j] = fixed_fraction(x[gi], invL);
      uy[j] = fixed_fraction(y[gi], invL);
      uz[j] = fixed_fraction(z[gi], invL);
      gx[j] = gF[gi];
      gy[j] = gF[n_total + gi];
      gz[j] = gF[2 * n_total + gi];
    } else {
      ux[j] = uy[j] = uz[j] = 0u;
      gx[j] = gy[j] = gz[j] = 0.0f;
    }
    rx[j] = ry[j] = rz[j] = rq[j] = 0.0f;
  }
  for (int t0 = 0; t0 < sd.p; t0 += kTabChunk) {
    const int cnt = min(kTabChunk, sd.p - t0);
    __syncthreads();
    for (int e = tid; e < cnt; e += kForceBlock) {
      const int64_t g = sd.k_off + t0 + e;
      const AdjTab a = adjoint_row(sd, g, m, wk, rho, w.xy, gu, kscale, vol);
      TabAdjF32 tb;
      tb.mx = m[3 * g]; tb.my = m[3 * g + 1]; tb.mz = m[3 * g + 2];
      tb.fx = (float)tb.mx; tb.fy = (float)tb.my; tb.fz = (float)tb.mz;
      // rotate by exp(-i delta) to match the truncated phases
      tb.z1r = (float)(a.z1r * rot_c + a.z1i * rot_s);
      tb.z1i = (float)(a.z1i * rot_c - a.z1r * rot_s);
      tb.z2r = (float)(a.z2r * rot_c + a.z2i * rot_s);
      tb.z2i = (float)(a.z2i * rot_c - a.z2r * rot_s);
      tab[e] = tb;
    }
    __syncthreads();
    for (int e = 0; e < cnt; ++e) {
      const TabAdjF32 tb = tab[e];
#pragma unroll
      for (int j = 0; j < NPLF; ++j) {
        const float a = turns_arg(phase_u32(tb.mx, tb.my, tb.mz, ux[j], uy[j], uz[j]));
        const float sn = __builtin_amdgcn_sinf(a);
        const float cs = __builtin_amdgcn_cosf(a);
        const float gm = fmaf(gx[j], tb.fx, fmaf(gy[j], tb.fy, gz[j] * tb.fz));
        const float p1 = tb.z1i * cs - tb.z1r * sn;
        const float p2 = tb.z2r * cs + tb.z2i * sn;
        const float q1 = tb.z1r * cs + tb.z1i * sn;
        const float q2 = tb.z2i * cs - tb.z2r * sn;
        const float sr = fmaf(gm, p2, p1);
        rx[j] = fmaf(sr, tb.fx, rx[j]);
        ry[j] = fmaf(sr, tb.fy, ry[j]);
        rz[j] = fmaf(sr, tb.fz, rz[j]);
        rq[j] += fmaf(-gm, q2, q1);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    if (j * kForceBlock + tid < it.np) {
      const int64_t gi = sd.n_off + it.p0 + j * kForceBlock + tid;
      const double s = q[gi] * kscale;
      gr[gi] = (float)(s * rx[j]);
      gr[n_total + gi] = (float)(s * ry[j]);
      gr[2 * n_total + gi] = (float)(s * rz[j]);
      gq[gi] = rq[j];
    }
  }
}

template <int NPLF>
__global__ __launch_bounds__(kForceBlock) void vjp_b2_f64_kernel(
    WsView w, int64_t n_total, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ q, const int32_t* __restrict__ m,
    const double* __restrict__ wk, const double* __restrict__ rho, const double* __restrict__ gU,
    const double* __restrict__ gF, double* __restrict__ gr, double* __restrict__ gq) {
  __shared__ double tabm[kTabChunk][3];
  __shared__ AdjTab tab[kTabChunk];
  const ForceItem it = w.force_items[blockIdx.x];
  const SysDesc sd = w.sys[it.sys];
  const int tid = threadIdx.x;
  const double invL = 1.0 / sd.L;
  const double kscale = kTwoPi * invL;
  const double vol = sd.L * sd.L * sd.L;
  const double gu = gU[it.sys];

  double sx[NPLF], sy[NPLF], sz[NPLF], gx[NPLF], gy[NPLF], gz[NPLF];
  double rx[NPLF], ry[NPLF], rz[NPLF], rq[NPLF];
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    const bool ok = j * kForceBlock + tid < it.np;
    if (ok) {
      const int64_t gi = sd.n_off + it.p0 + j * kForceBlock + tid;
      const double vx = x[gi] * invL, vy = y[gi] * invL, vz = z[gi] * invL;
      sx[j] = vx - floor(vx);
      sy[j] = vy - floor(vy);
      sz[j] = vz - floor(vz);
      gx[j] = gF[gi];
      gy[j] = gF[n_total + gi];
      gz[j] = gF[2 * n_total + gi];
    } else {
      sx[j] = sy[j] = sz[j] = gx[j] = gy[j] = gz[j] = 0.0;
    }
    rx[j] = ry[j] = rz[j] = rq[j] = 0.0;
  }
  for (int t0 = 0; t0 < sd.p; t0 += kTabChunk) {
    const int cnt = min(kTabChunk, sd.p - t0);
    __syncthreads();
    for (int e = tid; e < cnt; e += kForceBlock) {
      const int64_t g = sd.k_off + t0 + e;
      tab[e] = adjoint_row(sd, g, m, wk, rho, w.xy, gu, kscale, vol);
      tabm[e][0] = m[3 * g];
      tabm[e][1] = m[3 * g + 1];
      tabm[e][2] = m[3 * g + 2];
    }
    __syncthreads();
    for (int e = 0; e < cnt; ++e) {
      const AdjTab tb = tab[e];
      const double mx = tabm[e][0], my = tabm[e][1], mz = tabm[e][2];
#pragma unroll
      for (int j = 0; j < NPLF; ++j) {
        double sn, cs;
        sincos_turns(phase_f64(mx, my, mz, sx[j], sy[j], sz[j]), &sn, &cs);
        const double gm = fma(gx[j], mx, fma(gy[j], my, gz[j] * mz));
        const double p1 = tb.z1i * cs - tb.z1r * sn;
        const double p2 = tb.z2r * cs + tb.z2i * sn;
        const double q1 = tb.z1r * cs + tb.z1i * sn;
        const double q2 = tb.z2i * cs - tb.z2r * sn;
        const double sr = fma(gm, p2, p1);
        rx[j] = fma(sr, mx, rx[j]);
        ry[j] = fma(sr, my, ry[j]);
        rz[j] = fma(sr, mz, rz[j]);
        rq[j] += fma(-gm, q2, q1);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    if (j * kForceBlock + tid < it.np) {
      const int64_t gi = sd.n_off + it.p0 + j * kForceBlock + tid;
      const double s = q[gi] * kscale;
      gr[gi] = s * rx[j];
      gr[n_total + gi] = s * ry[j];
      gr[2 * n_total + gi] = s * rz[j];
      gq[gi] = rq[j];
    }
  }
}

// ------------------------------------------------------------------ sampler

// One thread per wave vector of every system: Philox key (seed + b, stream_id),
// counter (l, attempt, 0, 0), inverse CDF per component, zero vector redrawn.
__global__ __launch_bounds__(256) void sample_kernel(WsView w, int64_t p_total, uint64_t seed,
                                                     uint64_t stream_id, int32_t* __restrict__ m,
                                                     double* __restrict__ wk) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= p_total) return;
  const int32_t b = w.ksys[g];
  const SysDesc sd = w.sys[b];
  const int64_t l = g - sd.k_off;
  const double S = w.cdf[sd.cdf_off];
  const double* c = w.cdf + sd.cdf_off + 1;
  const int32_t M = (sd.cdf_len - 1) / 2;
  const double Z = c[2 * M];
  int32_t v[3] = {0, 0, 0};
  for (int a = 0; a < kMaxAttempts; ++a) {
    U64x4 ctr = {{(uint64_t)l, (uint64_t)a, 0ull, 0ull}};
    const U64x4 r = philox4x64_10(ctr, seed + (uint64_t)b, stream_id);
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] = inverse_cdf(c, M, u01_53(r.v[d]) * Z);
    if (v[0] != 0 || v[1] != 0 || v[2] != 0) break;
  }
  m[3 * g] = v[0];
  m[3 * g + 1] = v[1];
  m[3 * g + 2] = v[2];
  wk[g] = (v[0] != 0 || v[1] != 0 || v[2] != 0) ? S / (double)sd.p : 0.0;
}

// ------------------------------------------------------------------ dispatch helpers

template <int NPL, int KC, bool CACHE, bool VJP>
void launch_rho_f32_t(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const float* gF,
                      hipStream_t st) {
  hipLaunchKernelGGL((rho_f32_kernel<NPL, KC, CACHE, VJP>), dim3(s.n_rho_items), dim3(64), 0, st, w,
                     x, y, z, q, m, gF, s.n_total);
}

template <int NPL, int KC, bool VJP>
void launch_rho_f64_t(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const double* gF,
                      hipStream_t st) {
  hipLaunchKernelGGL((rho_f64_kernel<NPL, KC, VJP>), dim3(s.n_rho_items), dim3(64), 0, st, w, x, y,
                     z, q, m, gF, s.n_total);
}

// Particle-tile pass over every (tile, k-range) item; VJP selects adjoint pass B1.
template <bool VJP>
void launch_tile_pass(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const void* gF,
                      hipStream_t st) {
  if (s.precision == RBE_FP32_MIXED) {
    const float* g = static_cast<const float*>(gF);
    const bool c = s.cached != 0 && !VJP;
    if (s.rv.npl == 16) {
      c ? launch_rho_f32_t<16, 8, true, VJP>(s, w, x, y, z, q, m, g, st)
        : launch_rho_f32_t<16, 8, false, VJP>(s, w, x, y, z, q, m, g, st);
    } else {
      c ? launch_rho_f32_t<8, 8, true, VJP>(s, w, x, y, z, q, m, g, st)
        : launch_rho_f32_t<8, 8, false, VJP>(s, w, x, y, z, q, m, g, st);
    }
  } else {
    const double* g = static_cast<const double*>(gF);
    if (s.rv.npl == 4) launch_rho_f64_t<4, 4, VJP>(s, w, x, y, z, q, m, g, st);
    else launch_rho_f64_t<8, 4, VJP>(s, w, x, y, z, q, m, g, st);
  }
}

// exp(i delta) with delta = pi 2^-23: mean phase drop of the 23-bit truncation.
void truncation_rotation(int precision, double* c, double* s) {
  if (precision == RBE_FP32_MIXED) {
    const double delta = 3.14159265358979323846 / 8388608.0;
    *c = cos(delta);
    *s = sin(delta);
  } else {
    *c = 1.0;
    *s = 0.0;
  }
}

}  // namespace

hipError_t launch_rho(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, double* rho,
                      hipStream_t st) {
  if (s.n_rho_items > 0) {
    launch_tile_pass<false>(s, w, x, y, z, q, m, nullptr, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (s.p_total > 0) {
    double rc, rs;
    truncation_rotation(s.precision, &rc, &rs);
    const int per = kReduceBlock / 64;
    const int64_t blocks = (s.p_total + per - 1) / per;
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(kReduceBlock), 0, st, w, s.p_total, rho, rc, rs);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_force(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                        const double* z, const double* q, const int32_t* m, const double* wk,
                        const double* rho, void* F, double* U, hipStream_t st) {
  if (s.n_force_items == 0) return hipSuccess;
  const dim3 grid(s.n_force_items), block(kForceBlock);
  if (s.precision == RBE_FP32_MIXED) {
    double rc, rs;
    truncation_rotation(s.precision, &rc, &rs);
    float* Ff = static_cast<float*>(F);
    if (s.cached) {
      switch (s.fv.nplf) {
        case 1: hipLaunchKernelGGL((force_f32_kernel<1, true>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Ff, U, rc, rs); break;
        case 2: hipLaunchKernelGGL((force_f32_kernel<2, true>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Ff, U, rc, rs); break;
        default: hipLaunchKernelGGL((force_f32_kernel<4, true>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Ff, U, rc, rs); break;
      }
    } else {
      switch (s.fv.nplf) {
        case 1: hipLaunchKernelGGL((force_f32_kernel<1, false>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Ff, U, rc, rs); break;
        case 2: hipLaunchKernelGGL((force_f32_kernel<2, false>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Ff, U, rc, rs); break;
        default: hipLaunchKernelGGL((force_f32_kernel<4, false>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Ff, U, rc, rs); break;
      }
    }
  } else {
    double* Fd = static_cast<double*>(F);
    switch (s.fv.nplf) {
      case 1: hipLaunchKernelGGL((force_f64_kernel<1>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Fd, U); break;
      case 2: hipLaunchKernelGGL((force_f64_kernel<2>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Fd, U); break;
      default: hipLaunchKernelGGL((force_f64_kernel<4>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, Fd, U); break;
    }
  }
  return hipGetLastError();
}


hipError_t launch_vjp(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const double* wk,
                      const double* rho, const double* gU, const void* gF, void* gr, void* gq,
                      hipStream_t st) {
  double rc, rs;
  truncation_rotation(s.precision, &rc, &rs);
  if (s.n_rho_items > 0) {
    launch_tile_pass<true>(s, w, x, y, z, q, m, gF, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (s.p_total > 0) {
    const int per = kReduceBlock / 64;
    const int64_t blocks = (s.p_total + per - 1) / per;
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(kReduceBlock), 0, st, w, s.p_total, w.xy, rc, rs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (s.n_force_items == 0) return hipSuccess;
  const dim3 grid(s.n_force_items), block(kForceBlock);
  if (s.precision == RBE_FP32_MIXED) {
    const float* g = static_cast<const float*>(gF);
    float* r = static_cast<float*>(gr);
    float* qq = static_cast<float*>(gq);
    switch (s.fv.nplf) {
      case 1: hipLaunchKernelGGL((vjp_b2_f32_kernel<1>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs); break;
      case 2: hipLaunchKernelGGL((vjp_b2_f32_kernel<2>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs); break;
      default: hipLaunchKernelGGL((vjp_b2_f32_kernel<4>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs); break;
    }
  } else {
    const double* g = static_cast<const double*>(gF);
    double* r = static_cast<double*>(gr);
    double* qq = static_cast<double*>(gq);
    switch (s.fv.nplf) {
      case 1: hipLaunchKernelGGL((vjp_b2_f64_kernel<1>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq); break;
      case 2: hipLaunchKernelGGL((vjp_b2_f64_kernel<2>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq); break;
      default: hipLaunchKernelGGL((vjp_b2_f64_kernel<4>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_sample(const LaunchShape& s, const WsView& w, uint64_t seed, uint64_t stream_id,
                         int32_t* m, double* wk, hipStream_t st) {
  if (s.p_total == 0) return hipSuccess;
  const int64_t blocks = (s.p_total + 255) / 256;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, s.p_total, seed, stream_id, m, wk);
  return hipGetLastError();
}

}  // namespace rbe
