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

#include <algorithm>

#include "metropolis.h"
#include "philox.h"
#include "rbe_internal.h"
#include "sincos_coeffs.h"

namespace rbe {

// {particles per lane, wave vectors per chunk, wave vectors per work item, waves per block,
// particles per tile}
const RhoVariant kRhoVariantsF32[kNumRhoVariantsF32] = {
    {8, 8, 56, 4, 512}, {8, 8, 40, 4, 512}, {8, 8, 32, 4, 512}, {8, 8, 104, 4, 512}, {16, 8, 56, 4, 1024},
    {8, 4, 28, 4, 512}, {8, 4, 12, 4, 512}, {8, 8, 8, 16, 512}, {8, 4, 4, 16, 512},
    // k-lane layout (wpb 1: one item per 256-thread block): 5 wave vectors per lane, 3 x 21
    // lanes, so an item covers up to 105 wave vectors; tiles of 512 and 256 particles, and of
    // 492 = 4 waves x 41 steps x 3 (about 1M particles then fill 8 blocks per CU in one
    // round); the last one with compensated FP32 sums (forward pass)
    {8, 5, 105, 1, 512}, {4, 5, 105, 1, 256}, {8, 5, 105, 1, 492}, {8, 5, 105, 1, 492, 1}};
const RhoVariant kRhoVariantsF64[kNumRhoVariantsF64] = {
    {8, 4, 52, 4, 512}, {8, 2, 50, 4, 512}, {8, 2, 34, 4, 512}, {8, 4, 36, 4, 512}, {8, 4, 100, 4, 512},
    {4, 4, 100, 4, 256}, {4, 8, 104, 4, 256}, {4, 4, 4, 16, 256},
    // k-lane layout (wpb 1): 5 wave vectors on each of 3 x 21 lanes, tiles of 512 and 492
    {8, 5, 105, 1, 512}, {8, 5, 105, 1, 492}};
const ForceVariant kForceVariants[kNumForceVariants] = {{1}, {2}, {4}};

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kFourPi = 12.566370614359172953850573533118;
constexpr int kTabChunk = 256;
constexpr int kUnroll = 4;   // table rows per step of the force-shaped passes
constexpr int kPairs = 2;    // particles per step of the FP32 rho pass

// ------------------------------------------------------------------ phase helpers

// round(frac(x / L) * 2^32) as a 32-bit fixed-point fraction of a turn.
__device__ inline uint32_t fixed_fraction(double x, double invL) {
  const double v = x * invL;
  const double f = v - floor(v);
  const double r = fmin(fma(f, 4294967296.0, 0.5), 4294967295.0);
  return (uint32_t)r;
}

// q, or NaN when a coordinate is NaN or infinite (x * 0 is 0 for finite x and NaN
// otherwise).  The fixed-point fraction of a non-finite coordinate is a finite number, so
// the FP32-mixed passes carry the charge of such a particle as NaN instead: rho, and with
// it every force and the energy, come out NaN.
__device__ inline double finite_or_nan(double q, double x, double y, double z) {
  return q + (x * 0.0 + y * 0.0 + z * 0.0);
}

// Top 23 bits of a phase (turns * 2^32) as the float 1 + t/2^32 in [1, 2): revolutions.
__device__ inline float turns_arg(uint32_t t) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, t, 9u));
}

// m.u mod 2^32 from three v_mad_u64_u32 (32 x 32 + 64 -> 64 bits, issued at the rate of
// v_mul_lo_u32): one half-rate instruction per term fewer than three v_mul_lo_u32 and a
// v_add3_u32.  The low word of m u + c depends only on the low words of the operands, so
// it is the phase mod 2^32 with m taken as unsigned.  The 64-bit sums go through an empty
// asm (keep_u64) before their low words are used; otherwise the compiler narrows them back
// to 32-bit multiplies and an add.  One asm covers a group of sums, so the group's
// multiply-add chains can interleave.
__device__ inline uint64_t phase_u64(int32_t mx, int32_t my, int32_t mz, uint32_t ux, uint32_t uy, uint32_t uz) {
  uint64_t t = (uint64_t)(uint32_t)mz * uz;
  t = (uint64_t)(uint32_t)my * uy + t;
  return (uint64_t)(uint32_t)mx * ux + t;
}
// m.u + d mod 2^32, a phase shifted by the fixed-point offset in the low word of d (the high
// word may hold anything: it does not reach the low 32 bits of the sum).  d is the first
// addend, so the shift costs no instruction.
__device__ inline uint64_t phase_u64_off(int32_t mx, int32_t my, int32_t mz, uint32_t ux, uint32_t uy, uint32_t uz,
                                         uint64_t d) {
  uint64_t t = (uint64_t)(uint32_t)mz * uz + d;
  t = (uint64_t)(uint32_t)my * uy + t;
  return (uint64_t)(uint32_t)mx * ux + t;
}
template <int K> __device__ inline void keep_u64(uint64_t (&t)[K]);
template <> __device__ inline void keep_u64<1>(uint64_t (&t)[1]) { asm("" : "+v"(t[0])); }
template <> __device__ inline void keep_u64<2>(uint64_t (&t)[2]) { asm("" : "+v"(t[0]), "+v"(t[1])); }
template <> __device__ inline void keep_u64<4>(uint64_t (&t)[4]) {
  asm("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]));
}
template <> __device__ inline void keep_u64<5>(uint64_t (&t)[5]) {
  asm("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]));
}
template <> __device__ inline void keep_u64<8>(uint64_t (&t)[8]) {
  asm("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]), "+v"(t[7]));
}

// Phase arithmetic of the FP32 passes.  Both give the argument of v_sin_f32 / v_cos_f32,
// which take revolutions.
//   Phase<false> (RBE_FP32_MIXED): 32-bit fixed-point fractions; m.s mod 1 is exact,
//     then truncated to 23 bits (3 integer multiply-adds and alignbit per term).
//   Phase<true> (RBE_FP32): fractions centred in [-1/2, 1/2] held in FP32 and the phase
//     m.s by an FMA chain (3 ops per term).  Its rounding error grows with |m.s|, and
//     v_sin / v_cos accept |m.s| <= 256 turns.
template <bool FPH> struct Phase;
template <> struct Phase<false> {
  using Coord = uint32_t;
  __device__ static inline Coord coord(double x, double invL) { return fixed_fraction(x, invL); }
  // K terms of one particle: a[c] for wave vector c
  template <int K>
  __device__ static inline void args(const int32_t (&mx)[K], const int32_t (&my)[K], const int32_t (&mz)[K],
                                     const float (&)[K], const float (&)[K], const float (&)[K], Coord ux,
                                     Coord uy, Coord uz, float (&a)[K]) {
    uint64_t t[K];
#pragma unroll
    for (int c = 0; c < K; ++c) t[c] = phase_u64(mx[c], my[c], mz[c], ux, uy, uz);
    keep_u64<K>(t);
#pragma unroll
    for (int c = 0; c < K; ++c) a[c] = turns_arg((uint32_t)t[c]);
  }
  __device__ static inline float arg(int32_t mx, int32_t my, int32_t mz, float fx, float fy, float fz, Coord ux,
                                     Coord uy, Coord uz) {
    float a[1];
    args<1>({mx}, {my}, {mz}, {fx}, {fy}, {fz}, ux, uy, uz, a);
    return a[0];
  }
  // K terms of one particle, each phase shifted by its offset (fixed-point d[c])
  template <int K>
  __device__ static inline void args_off(const int32_t (&mx)[K], const int32_t (&my)[K], const int32_t (&mz)[K],
                                         const float (&)[K], const float (&)[K], const float (&)[K],
                                         const uint64_t (&d)[K], const float (&)[K], Coord ux, Coord uy, Coord uz,
                                         float (&a)[K]) {
    uint64_t t[K];
#pragma unroll
    for (int c = 0; c < K; ++c) t[c] = phase_u64_off(mx[c], my[c], mz[c], ux, uy, uz, d[c]);
    keep_u64<K>(t);
#pragma unroll
    for (int c = 0; c < K; ++c) a[c] = turns_arg((uint32_t)t[c]);
  }
};
template <> struct Phase<true> {
  using Coord = float;
  __device__ static inline Coord coord(double x, double invL) {
    const double v = x * invL;
    return (float)(v - rint(v));
  }
  __device__ static inline float arg(int32_t, int32_t, int32_t, float fx, float fy, float fz, Coord ux,
                                     Coord uy, Coord uz) {
    return fmaf(fx, ux, fmaf(fy, uy, fz * uz));
  }
  template <int K>
  __device__ static inline void args(const int32_t (&)[K], const int32_t (&)[K], const int32_t (&)[K],
                                     const float (&fx)[K], const float (&fy)[K], const float (&fz)[K], Coord ux,
                                     Coord uy, Coord uz, float (&a)[K]) {
#pragma unroll
    for (int c = 0; c < K; ++c) a[c] = fmaf(fx[c], ux, fmaf(fy[c], uy, fz[c] * uz));
  }
  // shifted by the offset in turns (dt[c]), the first addend of the chain
  template <int K>
  __device__ static inline void args_off(const int32_t (&)[K], const int32_t (&)[K], const int32_t (&)[K],
                                         const float (&fx)[K], const float (&fy)[K], const float (&fz)[K],
                                         const uint64_t (&)[K], const float (&dt)[K], Coord ux, Coord uy, Coord uz,
                                         float (&a)[K]) {
#pragma unroll
    for (int c = 0; c < K; ++c) a[c] = fmaf(fx[c], ux, fmaf(fy[c], uy, fmaf(fz[c], uz, dt[c])));
  }
};

// sin and cos of 2 pi r for |r| <= 1/2 (turns), FP64.  With q = rint(4 r) in {-2..2}
// and f = r - q/4 (exact, |f| <= 1/8): exp(2 pi i r) = i^q exp(2 pi i f), and
// i^q = (1 - |q|) + i q (2 - |q|) exactly, so the quarter-turn rotation is two
// exact products and two FMAs instead of selects.
__device__ inline void sincos_turns(double r, double* s, double* c) {
  const double q = rint(4.0 * r);
  const double f = fma(q, -0.25, r);
  const double f2 = f * f;
  double ps = kSin[kSinTerms - 1];
#pragma unroll
  for (int j = kSinTerms - 2; j >= 0; --j) ps = fma(ps, f2, kSin[j]);
  double pc = kCos[kCosTerms - 1];
#pragma unroll
  for (int j = kCosTerms - 2; j >= 0; --j) pc = fma(pc, f2, kCos[j]);
  const double sn = ps * f;
  const double aq = fabs(q);
  const double cq = 1.0 - aq;            // cos(pi q / 2)
  const double sq = q * (2.0 - aq);      // sin(pi q / 2)
  *s = fma(sn, cq, pc * sq);
  *c = fma(pc, cq, -(sn * sq));
}

// Table of (cos, sin) of 2 pi q / kTurnSteps for q = 0 .. kTurnSteps - 1 (8 KB of LDS),
// built by a block from sincos_turns (rows past the half turn use q - kTurnSteps).
constexpr int kTurnRows = kTurnSteps;
static_assert((kTurnSteps & (kTurnSteps - 1)) == 0, "the table index is q mod kTurnSteps");
__device__ inline void build_turn_table(double2* tab) {
  for (int i = threadIdx.x; i < kTurnRows; i += blockDim.x) {
    double s, c;
    const int qi = i <= kTurnSteps / 2 ? i : i - kTurnSteps;
    sincos_turns((double)qi * (1.0 / kTurnSteps), &s, &c);
    tab[i] = make_double2(c, s);
  }
}

// Fractional coordinate frac(x / L) in units of 1/kTurnSteps turn (the product with the
// power of two is exact), so that m.s comes out in the table's unit.
__device__ inline double table_coord(double x, double invL) {
  const double v = x * invL;
  return (v - floor(v)) * (double)kTurnSteps;
}

// sin and cos of 2 pi t / N (N = kTurnSteps) for a phase t in units of 1/N turn (any size
// that keeps q below 2^31), FP64, from the table: with q = rint(t) and g = t - q (exact:
// q is within a factor 2 of t unless q = 0; |g| <= 1/2), exp(2 pi i t / N) =
// t_(q mod N) exp(2 pi i g / N).  The short polynomials give sin(2 pi g / N) and
// cos(2 pi g / N) - 1, which are small, so their products with the table entry are
// corrections added to it.
__device__ inline void sincos_phase_tab(double t, const double2* tab, double* s, double* c) {
  const double q = rint(t);
  const double g = t - q;
  const double u = g * g;
  static_assert(kSinShortTerms == 3 && kCosm1ShortTerms == 2, "the polynomials below are unrolled");
  const double sf = g * fma(fma(kSinShort[2], u, kSinShort[1]), u, kSinShort[0]);
  const double cm1 = u * fma(kCosm1Short[1], u, kCosm1Short[0]);
  const double2 e = tab[(int)q & (kTurnSteps - 1)];
  *s = fma(e.y, cm1, fma(e.x, sf, e.y));
  *c = fma(e.x, cm1, fma(-e.y, sf, e.x));
}

// phase m.s (not reduced), in the unit of s.
__device__ inline double dot_f64(double mx, double my, double mz, double sx, double sy, double sz) {
  return fma(mx, sx, fma(my, sy, mz * sz));
}


// ------------------------------------------------------------------ wave reductions

template <int V> struct Log2 { static constexpr int value = 1 + Log2<V / 2>::value; };
template <> struct Log2<1> { static constexpr int value = 0; };

// Cross-lane exchange with a DPP row permutation (VALU, no LDS round trip).
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const int2 a = *reinterpret_cast<const int2*>(&v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(0, a.x, CTRL, 0xF, 0xF, false);
  r.y = __builtin_amdgcn_update_dpp(0, a.y, CTRL, 0xF, 0xF, false);
  return *reinterpret_cast<const double*>(&r);
}

// DPP controls of the four in-row reduce-scatter levels and the lane bit that
// selects the kept half at each level.  Partners: lane ^ 1 and lane ^ 2 (quad
// permutations), lane ^ 7 within 8 (half-row mirror), lane ^ 8 within 16 (row
// rotation by 8).  The kept-half selectors s1 = b0^b2, s2 = b1^b2, s3 = b2,
// s4 = b3 make every pair of partners hold the same value subset.
constexpr int kDppCtrl[4] = {0xB1, 0x4E, 0x141, 0x128};

__device__ inline bool keep_upper(int level, int lane) {
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  switch (level) {
    case 0: return (b0 ^ b2) != 0;
    case 1: return (b1 ^ b2) != 0;
    case 2: return b2 != 0;
    default: return b3 != 0;
  }
}

// Value index that lane L holds after the in-row levels (inverse of the selectors).
__device__ inline int scatter_index(int lane, int levels) {
  int idx = 0;
  for (int j = 0; j < levels; ++j) idx = 2 * idx + (keep_upper(j, lane) ? 1 : 0);
  return idx;
}

template <int LEVEL, int HALF, typename T, int V>
struct ReduceScatter {
  __device__ static inline void run(T (&v)[V], int lane) {
    const bool upper = keep_upper(LEVEL, lane);
#pragma unroll
    for (int i = 0; i < HALF; ++i) {
      const T send = upper ? v[i] : v[i + HALF];
      const T keep = upper ? v[i + HALF] : v[i];
      v[i] = keep + dpp_move<kDppCtrl[LEVEL]>(send);
    }
    ReduceScatter<LEVEL + 1, HALF / 2, T, V>::run(v, lane);
  }
};
template <int LEVEL, typename T, int V>
struct ReduceScatter<LEVEL, 0, T, V> {
  __device__ static inline void run(T (&v)[V], int lane) {
    if constexpr (LEVEL < 4) {
      // remaining in-row levels: the partners already hold the same value index
      v[0] += dpp_move<kDppCtrl[LEVEL]>(v[0]);
      ReduceScatter<LEVEL + 1, 0, T, V>::run(v, lane);
    } else {
      // sum the four rows of 16 lanes
      v[0] += __shfl_xor(v[0], 16, 64);
      v[0] += __shfl_xor(v[0], 32, 64);
    }
  }
};

// Reduce-scatter of V values per lane over the 64 lanes of a wave: afterwards v[0] of
// lane L holds the wave sum of value index scatter_index(L mod 16, log2 V).  Every
// index is a compile-time constant, so the values stay in registers.
template <int V, typename T>
__device__ inline void wave_reduce_scatter(T (&v)[V], int lane) {
  static_assert(V == 2 || V == 4 || V == 8 || V == 16, "V must be 2, 4, 8 or 16");
  ReduceScatter<0, V / 2, T, V>::run(v, lane);
}

// Work schedules of the rho-shaped passes (template parameter WPB, waves per block).
//
// WPB = 4: four independent waves per 256-thread block, one per SIMD, each taking one
// (tile, k-range) item (capped grids stride over the items).  The waves sharing a SIMD
// come from different blocks and the hardware serves them oldest first, so the oldest
// finish early and the last ones run alone, too few to hide latency (one resident wave
// keeps a SIMD about half busy, four nearly fully).  Each wave therefore raises its issue
// priority with the chunks it has left (most remaining first, exact over the last three).
//
// WPB = 16: one 1024-thread block per CU (four waves per SIMD) over single-chunk items in
// tile-major order.  Each block owns an equal contiguous range of items, split into 16
// home ranges, one per wave.  A wave claims items from its home range through an LDS
// counter and, once that is used up, claims from the other waves' ranges in turn, so all
// sixteen waves stay busy until the CU's share is done.  Particles are reloaded only when
// the claimed item's tile differs from the one in registers.  Every claim is an atomic
// increment of a finite range and a wave stops after one fruitless pass over all ranges,
// so every wave exits.  Results do not depend on which wave runs an item.
constexpr int kCoopWaves = 16;

__device__ inline void remaining_priority(int chunks_left) {
  switch (chunks_left) {
    case 1: __builtin_amdgcn_s_setprio(0); break;
    case 2: __builtin_amdgcn_s_setprio(1); break;
    case 3: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
  }
}

template <int WPB> struct RhoSchedule;

template <> struct RhoSchedule<4> {
  int32_t item, n_items, stride;
  __device__ RhoSchedule(int32_t n, int32_t wave, int32_t*) : item(-1), n_items(n), stride(0) {
    item = (int32_t)blockIdx.x * 4 + wave;
    stride = (int32_t)gridDim.x * 4;
  }
  __device__ int32_t first() { return item < n_items ? item : -1; }
  __device__ int32_t next() {
    item += stride;
    return item < n_items ? item : -1;
  }
  // issue priority for a wave with chunks_left chunks of its current item to go
  __device__ void priority(int chunks_left) const {
    remaining_priority(item + stride < n_items ? 4 : chunks_left);
  }
};

template <> struct RhoSchedule<kCoopWaves> {
  int32_t* next_;   // LDS: next item of each home range, then the range ends
  int32_t wave, victim;
  __device__ RhoSchedule(int32_t n, int32_t wv, int32_t* lds) : next_(lds), wave(wv), victim(wv) {
    if (threadIdx.x < kCoopWaves) {
      const int64_t b0 = (int64_t)n * blockIdx.x / gridDim.x;
      const int64_t len = (int64_t)n * (blockIdx.x + 1) / gridDim.x - b0;
      const int t = threadIdx.x;
      lds[t] = (int32_t)(b0 + len * t / kCoopWaves);
      lds[kCoopWaves + t] = (int32_t)(b0 + len * (t + 1) / kCoopWaves);
    }
    __syncthreads();
  }
  __device__ int32_t claim() {
    for (;;) {
      int32_t idx = 0;
      if ((threadIdx.x & 63) == 0) idx = atomicAdd(&next_[victim], 1);
      idx = __builtin_amdgcn_readfirstlane(idx);
      const int32_t end = __builtin_amdgcn_readfirstlane(next_[kCoopWaves + victim]);
      if (idx < end) return idx;
      victim = (victim + 1) & (kCoopWaves - 1);
      if (victim == wave) return -1;
    }
  }
  __device__ int32_t first() { return claim(); }
  __device__ int32_t next() { return claim(); }
  __device__ void priority(int) const {}
};

// Wave vectors kc .. kc+KC-1 of an item (zero past its end); uniform, so scalar loads.
template <int KC>
__device__ inline void load_chunk(const int32_t* mk, int kc, int nk, int32_t (&mx)[KC], int32_t (&my)[KC],
                                  int32_t (&mz)[KC]) {
  if (kc + KC <= nk) {
    // whole chunk: 3 KC contiguous words (wide scalar loads)
    const int32_t* r = mk + 3 * kc;
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      mx[c] = r[3 * c];
      my[c] = r[3 * c + 1];
      mz[c] = r[3 * c + 2];
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int kk = min(kc + c, nk - 1);
    const int32_t a = mk[3 * kk], b = mk[3 * kk + 1], d = mk[3 * kk + 2];
    const bool ok = kc + c < nk;
    mx[c] = ok ? a : 0;
    my[c] = ok ? b : 0;
    mz[c] = ok ? d : 0;
  }
}

// ------------------------------------------------------------------ rho pass, FP32-mixed

// With VJP, the same pass forms X_l + i Y_l = sum_i q_i (gF_i . m_l) exp(i theta_il)
// (adjoint pass B1; the 2 pi / L of k_l is applied when the adjoint table is built).
template <int NPL, int KC, bool CACHE, bool VJP, bool FPH, int WPB>
__global__ __launch_bounds__(64 * WPB) void rho_f32_kernel(WsView w, const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ q,
                                                          const int32_t* __restrict__ m,
                                                          const float* __restrict__ gF, int64_t n_total,
                                                          int32_t n_items) {
  __shared__ int32_t sched_lds[WPB == kCoopWaves ? 2 * kCoopWaves : 1];
  const int lane = threadIdx.x & 63;
  const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  RhoSchedule<WPB> sched(n_items, wave, sched_lds);

  // particles per step: the cooperative blocks are limited to 128 VGPRs per wave
  constexpr int PAIRS = kPairs;
  using Ph = Phase<FPH>;
  typename Ph::Coord ux[NPL], uy[NPL], uz[NPL];
  float qv[NPL], qgx[VJP ? NPL : 1], qgy[VJP ? NPL : 1], qgz[VJP ? NPL : 1];
  int32_t cur_sys = -1, cur_tile = -1;   // tile held in registers

  for (int32_t item = sched.first(); item >= 0; item = sched.next()) {
    // the item index is wave-uniform; saying so keeps the item and its wave vectors in
    // scalar registers and scalar loads
    const RhoItem it = w.rho_items[__builtin_amdgcn_readfirstlane(item)];
    const SysDesc sd = w.sys[it.sys];
    const int first = it.tile * (64 * NPL);
    const int cnt = min(64 * NPL, sd.n - first);
    if (it.sys != cur_sys || it.tile != cur_tile) {
      cur_sys = it.sys;
      cur_tile = it.tile;
      const double invL = 1.0 / sd.L;
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const int li = j * 64 + lane;
        if (li < cnt) {
          const int64_t gi = sd.n_off + first + li;
          const double px = x[gi], py = y[gi], pz = z[gi];
          ux[j] = Ph::coord(px, invL);
          uy[j] = Ph::coord(py, invL);
          uz[j] = Ph::coord(pz, invL);
          qv[j] = (float)finite_or_nan(q[gi], px, py, pz);
          if (VJP) {
            qgx[j] = qv[j] * gF[gi];
            qgy[j] = qv[j] * gF[n_total + gi];
            qgz[j] = qv[j] * gF[2 * n_total + gi];
          }
        } else {
          ux[j] = uy[j] = uz[j] = 0;
          qv[j] = 0.0f;
          if (VJP) qgx[j] = qgy[j] = qgz[j] = 0.0f;
        }
        // reload in groups of four particles: bounds the FP64 loads in flight (registers)
        if (WPB == kCoopWaves && (j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    double* part = w.partials + 2 * sd.part_off;
    const int32_t* mk = m + 3 * (sd.k_off + it.k0);

    // wave vectors of the next chunk are loaded (scalar loads) one chunk ahead
    int32_t nmx[KC], nmy[KC], nmz[KC];
    load_chunk<KC>(mk, 0, it.nk, nmx, nmy, nmz);
    for (int kc = 0; kc < it.nk; kc += KC) {
      sched.priority((it.nk - kc + KC - 1) / KC);
      int32_t mx[KC], my[KC], mz[KC];
      float fmx[KC], fmy[KC], fmz[KC];   // used by the FP32 phase only
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        mx[c] = nmx[c];
        my[c] = nmy[c];
        mz[c] = nmz[c];
        fmx[c] = (float)mx[c];
        fmy[c] = (float)my[c];
        fmz[c] = (float)mz[c];
      }
      if (kc + KC < it.nk) load_chunk<KC>(mk, kc + KC, it.nk, nmx, nmy, nmz);
      float acc[2 * KC];
#pragma unroll
      for (int c = 0; c < 2 * KC; ++c) acc[c] = 0.0f;
#pragma unroll
      for (int j0 = 0; j0 < NPL; j0 += PAIRS) {
        // PAIRS particles against the KC wave vectors, stage by stage for instruction-level
        // parallelism (PAIRS * KC independent phase -> sin/cos -> FMA chains)
        float a[PAIRS][KC], sn[PAIRS][KC], cs[PAIRS][KC];
#pragma unroll
        for (int jj = 0; jj < PAIRS; ++jj)
          Ph::template args<KC>(mx, my, mz, fmx, fmy, fmz, ux[j0 + jj], uy[j0 + jj], uz[j0 + jj], a[jj]);
#pragma unroll
        for (int jj = 0; jj < PAIRS; ++jj)
#pragma unroll
          for (int c = 0; c < KC; ++c) sn[jj][c] = __builtin_amdgcn_sinf(a[jj][c]);
#pragma unroll
        for (int jj = 0; jj < PAIRS; ++jj)
#pragma unroll
          for (int c = 0; c < KC; ++c) cs[jj][c] = __builtin_amdgcn_cosf(a[jj][c]);
#pragma unroll
        for (int jj = 0; jj < PAIRS; ++jj) {
          const int j = j0 + jj;
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            float wt = qv[j];
            if (VJP) wt = fmaf(qgx[j], fmx[c], fmaf(qgy[j], fmy[c], qgz[j] * fmz[c]));
            acc[c] = fmaf(wt, cs[jj][c], acc[c]);
            acc[KC + c] = fmaf(wt, sn[jj][c], acc[KC + c]);
            if (CACHE) {
              const int li = j * 64 + lane;
              if (li < cnt && kc + c < it.nk) {
                float2* cp = reinterpret_cast<float2*>(w.cache) + sd.cache_off +
                             (int64_t)(it.k0 + kc + c) * sd.n + first + li;
                *cp = make_float2(cs[jj][c], sn[jj][c]);
              }
            }
          }
        }
      }
      wave_reduce_scatter<2 * KC>(acc, lane);
      if (lane < 2 * KC) {
        const int vi = scatter_index(lane, Log2<2 * KC>::value);
        const int c = vi % KC;
        const int comp = vi / KC;
        if (kc + c < it.nk) {
          const int64_t kl = it.k0 + kc + c;
          part[2 * (kl * sd.ntiles + it.tile) + comp] = (double)acc[0];
        }
      }
    }
  }
}

// ------------------------------------------------------------------ rho pass, k-lane layout

// The rho pass with wave vectors across the lanes instead of particles.  A 256-thread block
// takes one (tile, k-range) item: the tile's TILE particles are staged in LDS as fixed-
// point (or FP32) fractions and FP32 charges, and each wave takes a quarter of them.  Lane
// (g, kl) of a wave, g < G, kl < 64 / G, holds the KPL wave vectors k0 + kl + (64 / G) c and
// sums them over particles g, g + G, ... of the wave's quarter, reading each particle from
// LDS once for its KPL terms.  No value crosses lanes until the item is done; then the
// 4 G partial sums of each (wave vector, component) are added in a fixed order in FP64.
// This takes the per-chunk wave reduce-scatter and the particle registers out of the
// inner loop.  With VJP it forms X + iY of the adjoint pass B1, the per-term weight
// q_i (gF_i . m_l) coming from the staged q_i gF_i.  The phase cache runs the per-wave
// kernel over the same items and tiles.  TILE (512 or 256 particles) is 64 NPL of the
// variant, the tile of the per-wave kernel with the same NPL.

template <bool FPH> struct KlParticle;
template <> struct KlParticle<false> { uint32_t ux, uy, uz; float q; };
template <> struct KlParticle<true> { float ux, uy, uz; float q; };

// Compensated FP32 sums (the COMP variant): runs of kCompBlock plain FP32 steps, each run's
// sum then added into a per-lane (hi, lo) pair with an error-free TwoSum; the lane groups
// and waves are combined as (hi, lo) pairs, so FP64 enters only across tiles.
constexpr int kCompBlock = 16;

// hi + lo += b: TwoSum of hi and b, its rounding error added to lo.
__device__ inline void two_sum_into(float& hi, float& lo, float b) {
  const float s = hi + b;
  const float bb = s - hi;
  const float e = (hi - (s - bb)) + (b - bb);
  hi = s;
  lo += e;
}

// (h, l) += (h2, l2) for unevaluated sums of two floats: TwoSum of the high parts, the low
// parts added to its error, then renormalised (Fast2Sum).
__device__ inline void pair_add(float& h, float& l, float h2, float l2) {
  const float s = h + h2;
  const float bb = s - h;
  float e = (h - (s - bb)) + (h2 - bb);
  e += l + l2;
  h = s + e;
  l = e - (h - s);
}

template <int TILE, int G, int KPL, bool VJP, bool FPH, bool COMP>
__device__ __forceinline__ void rho_klane_body(const WsView& w, const double* __restrict__ x,
                                               const double* __restrict__ y, const double* __restrict__ z,
                                               const double* __restrict__ q, const int32_t* __restrict__ m,
                                               const float* __restrict__ gF, int64_t n_total, int32_t n_items) {
  constexpr int KL = 64 / G;              // k-lanes per wave
  constexpr int PW = TILE / 4;            // particles per wave
  constexpr int STEPS = (PW + G - 1) / G; // particle steps of every lane
  constexpr int PWP = STEPS * G;          // a wave's LDS slots: its particles, then zero ones
  using Ph = Phase<FPH>;
  using Pt = KlParticle<FPH>;
  static_assert(sizeof(Pt) == 16, "one 16-byte LDS read per particle");
  // G slots past the last wave's are read (never used) by the two-step loop below
  __shared__ __align__(16) Pt tile[4 * PWP + G];
  __shared__ __align__(16) float4 tgw[VJP ? 4 * PWP + G : 1];   // q gF of each slot (VJP)
  __shared__ float red[COMP ? 1 : 4][G][2 * KPL][KL];
  __shared__ float2 redc[COMP ? 4 : 1][2 * KPL][KL];   // (hi, lo) per wave (COMP)
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kl = lane % KL;
  const int g = lane / KL;                // G for the 64 - G KL idle lanes
  for (int32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const RhoItem it = w.rho_items[__builtin_amdgcn_readfirstlane(item)];
    const SysDesc sd = w.sys[it.sys];
    const int first = it.tile * TILE;
    const int cnt = min(TILE, sd.n - first);
    const double invL = 1.0 / sd.L;
    // this lane's wave vectors (zero past the item's end or on idle lanes)
    int32_t mx[KPL], my[KPL], mz[KPL];
    float fmx[KPL], fmy[KPL], fmz[KPL];
#pragma unroll
    for (int c = 0; c < KPL; ++c) {
      const int kk = kl + KL * c;
      const bool ok = g < G && kk < it.nk;
      const int64_t gk = sd.k_off + it.k0 + min(kk, max(it.nk - 1, 0));
      const int32_t a = m[3 * gk], b = m[3 * gk + 1], d = m[3 * gk + 2];
      mx[c] = ok ? a : 0;
      my[c] = ok ? b : 0;
      mz[c] = ok ? d : 0;
      fmx[c] = (float)mx[c];
      fmy[c] = (float)my[c];
      fmz[c] = (float)mz[c];
    }
    __syncthreads();   // the previous item's readers of tile and red are done
    for (int i = tid; i < 4 * PWP; i += 256) {
      // slot i is particle (i / PWP) PW + i % PWP of the tile, or a zero pad slot
      const int wv = i / PWP, sl = i % PWP;
      const int pi = wv * PW + sl;
      Pt v;
      float4 qg = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (sl < PW && pi < cnt) {
        const int64_t gi = sd.n_off + first + pi;
        const double px = x[gi], py = y[gi], pz = z[gi];
        v.ux = Ph::coord(px, invL);
        v.uy = Ph::coord(py, invL);
        v.uz = Ph::coord(pz, invL);
        v.q = (float)finite_or_nan(q[gi], px, py, pz);
        if (VJP) qg = make_float4(v.q * gF[gi], v.q * gF[n_total + gi], v.q * gF[2 * n_total + gi], 0.0f);
      } else {
        v.ux = v.uy = v.uz = 0;
        v.q = 0.0f;
      }
      tile[i] = v;
      if (VJP) tgw[i] = qg;
    }
    __syncthreads();
    float acc[2 * KPL];
    float chi[COMP ? 2 * KPL : 1], clo[COMP ? 2 * KPL : 1];   // (hi, lo) pairs (COMP)
#pragma unroll
    for (int c = 0; c < 2 * KPL; ++c) acc[c] = 0.0f;
    if (COMP) {
#pragma unroll
      for (int c = 0; c < (COMP ? 2 * KPL : 1); ++c) chi[c] = clo[c] = 0.0f;
    }
    if (g < G) {
      // the same number of steps on every lane (zero slots pad the last one).  Forward pass:
      // two steps per iteration, each particle read from LDS one step before its terms into
      // one of two register sets that alternate, so no step copies a particle between them
      const Pt* tp = tile + wave * PWP + g;
      const float4* gp = tgw + (VJP ? wave * PWP + g : 0);
      auto step = [&](const Pt& v, int j) {
        float4 qg = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (VJP) qg = gp[j * G];
        float a[KPL], sn[KPL], cs[KPL];
        Ph::template args<KPL>(mx, my, mz, fmx, fmy, fmz, v.ux, v.uy, v.uz, a);
#pragma unroll
        for (int c = 0; c < KPL; ++c) sn[c] = __builtin_amdgcn_sinf(a[c]);
#pragma unroll
        for (int c = 0; c < KPL; ++c) cs[c] = __builtin_amdgcn_cosf(a[c]);
#pragma unroll
        for (int c = 0; c < KPL; ++c) {
          float wt = v.q;
          if (VJP) wt = fmaf(qg.x, fmx[c], fmaf(qg.y, fmy[c], qg.z * fmz[c]));
          acc[c] = fmaf(wt, cs[c], acc[c]);
          acc[KPL + c] = fmaf(wt, sn[c], acc[KPL + c]);
        }
      };
      // steps j0 .. j1 - 1, two per iteration, each particle read one step before its terms
      // into one of two register sets that alternate, so no step copies a particle
      auto run = [&](int j0, int j1) {
        Pt pa = tp[j0 * G];
        int j = j0;
        for (; j + 1 < j1; j += 2) {
          const Pt pb = tp[(j + 1) * G];
          step(pa, j);
          // nothing moves across: pa's registers are free when its next value is read
          __builtin_amdgcn_sched_barrier(0);
          pa = tp[(j + 2) * G];   // slot (j + 2) G <= STEPS G: inside the padded tile
          step(pb, j + 1);
          __builtin_amdgcn_sched_barrier(0);
        }
        if ((j1 - j0) & 1) step(pa, j1 - 1);
      };
      if constexpr (!VJP && !COMP) {
        run(0, STEPS);
      } else if constexpr (!VJP) {
#pragma unroll
        for (int c = 0; c < 2 * KPL; ++c) chi[c] = clo[c] = 0.0f;
        for (int j0 = 0; j0 < STEPS; j0 += kCompBlock) {
          run(j0, min(j0 + kCompBlock, STEPS));
#pragma unroll
          for (int c = 0; c < 2 * KPL; ++c) {
            two_sum_into(chi[c], clo[c], acc[c]);
            acc[c] = 0.0f;
          }
        }
      } else {
        // pass B1 carries more registers: one step per iteration, the next particle read
        // while this one's terms are computed
        Pt nxt = tp[0];
        for (int j = 0; j < STEPS; ++j) {
          const Pt v = nxt;
          if (j + 1 < STEPS) nxt = tp[(j + 1) * G];
          step(v, j);
        }
      }
      if constexpr (!COMP) {
#pragma unroll
        for (int c = 0; c < 2 * KPL; ++c) red[wave][g][c][kl] = acc[c];
      }
    }
    double* part = w.partials + 2 * sd.part_off;
    if constexpr (COMP) {
      // the G lane groups of each k-lane (lanes kl, kl + KL, ...) as (hi, lo) pairs in a
      // fixed order (lanes past the groups hold zeros), then the 4 waves; the pair becomes the
      // tile's FP64 partial exactly
#pragma unroll
      for (int c = 0; c < 2 * KPL; ++c) {
        float h = chi[c], l = clo[c];
#pragma unroll
        for (int gg = 1; gg < G; ++gg) pair_add(h, l, __shfl(chi[c], kl + KL * gg, 64), __shfl(clo[c], kl + KL * gg, 64));
        if (g == 0) redc[wave][c][kl] = make_float2(h, l);
      }
      __syncthreads();
      for (int o = tid; o < 2 * it.nk; o += 256) {
        const int kk = o >> 1, comp = o & 1;
        const int c = kk / KL, r = kk % KL;
        float2 v = redc[0][comp * KPL + c][r];
#pragma unroll
        for (int wv = 1; wv < 4; ++wv) {
          const float2 u = redc[wv][comp * KPL + c][r];
          pair_add(v.x, v.y, u.x, u.y);
        }
        const int64_t kidx = it.k0 + kk;
        part[2 * (kidx * sd.ntiles + it.tile) + comp] = (double)v.x + (double)v.y;
      }
    } else {
      __syncthreads();
      // output o = (wave vector kk, component): the 4 G partial sums in a fixed order
      for (int o = tid; o < 2 * it.nk; o += 256) {
        const int kk = o >> 1, comp = o & 1;
        const int c = kk / KL, r = kk % KL;
        double sum = 0.0;
#pragma unroll
        for (int wv = 0; wv < 4; ++wv)
#pragma unroll
          for (int gg = 0; gg < G; ++gg) sum += (double)red[wv][gg][comp * KPL + c][r];
        const int64_t kidx = it.k0 + kk;
        part[2 * (kidx * sd.ntiles + it.tile) + comp] = sum;
      }
    }
  }
}

// The forward k-lane pass keeps 8 waves per SIMD (64 VGPRs): a 1M-particle system's 1,954
// blocks then fit in one round of 8 blocks per CU.  Pass B1 carries more registers.
template <int TILE, int G, int KPL, bool FPH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void rho_klane_kernel(
    WsView w, const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ q, const int32_t* __restrict__ m, int64_t n_total, int32_t n_items) {
  rho_klane_body<TILE, G, KPL, false, FPH, false>(w, x, y, z, q, m, nullptr, n_total, n_items);
}

// The forward pass with compensated FP32 sums (more registers: 6 waves per SIMD).
template <int TILE, int G, int KPL, bool FPH>
__global__ __launch_bounds__(256) void rho_klane_comp_kernel(
    WsView w, const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ q, const int32_t* __restrict__ m, int64_t n_total, int32_t n_items) {
  rho_klane_body<TILE, G, KPL, false, FPH, true>(w, x, y, z, q, m, nullptr, n_total, n_items);
}

template <int TILE, int G, int KPL, bool FPH>
__global__ __launch_bounds__(256) void rho_klane_vjp_kernel(WsView w, const double* __restrict__ x,
                                                           const double* __restrict__ y,
                                                           const double* __restrict__ z,
                                                           const double* __restrict__ q,
                                                           const int32_t* __restrict__ m,
                                                           const float* __restrict__ gF, int64_t n_total,
                                                           int32_t n_items) {
  rho_klane_body<TILE, G, KPL, true, FPH, false>(w, x, y, z, q, m, gF, n_total, n_items);
}

// ------------------------------------------------------------------ rho pass, FP64 k-lane

// The k-lane layout of rho_klane_kernel in FP64: lane (g, kl) sums its KPL wave vectors
// over particles g, g + G, ... of its wave's quarter of the tile, from fractional
// coordinates in table units staged in LDS, with the table form of sin/cos.  At the end of
// an item the G subgroups of a wave are added by fixed-order shuffles, then the 4 waves
// through LDS, all in FP64.  With VJP the per-term weight is q_i (gF_i . m_l).
struct KlParticleF64 { double sx, sy, sz, q; };

template <int TILE, int G, int KPL, bool VJP>
__global__ __launch_bounds__(256) void rho_klane_f64_kernel(WsView w, const double* __restrict__ x,
                                                           const double* __restrict__ y,
                                                           const double* __restrict__ z,
                                                           const double* __restrict__ q,
                                                           const int32_t* __restrict__ m,
                                                           const double* __restrict__ gF, int64_t n_total,
                                                           int32_t n_items) {
  constexpr int KL = 64 / G;
  constexpr int PW = TILE / 4;
  constexpr int STEPS = (PW + G - 1) / G;
  constexpr int PWP = STEPS * G;
  using Pt = KlParticleF64;
  __shared__ double2 turns[kTurnRows];
  __shared__ __align__(16) Pt tile[4 * PWP];
  __shared__ __align__(16) Pt tgw[VJP ? 4 * PWP : 1];   // q gF of each slot (VJP)
  __shared__ double red[4][2 * KPL][KL];
  build_turn_table(turns);   // the item loop's first barrier precedes every use
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kl = lane % KL;
  const int g = lane / KL;
  for (int32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const RhoItem it = w.rho_items[__builtin_amdgcn_readfirstlane(item)];
    const SysDesc sd = w.sys[it.sys];
    const int first = it.tile * TILE;
    const int cnt = min(TILE, sd.n - first);
    const double invL = 1.0 / sd.L;
    double mx[KPL], my[KPL], mz[KPL];
#pragma unroll
    for (int c = 0; c < KPL; ++c) {
      const int kk = kl + KL * c;
      const bool ok = g < G && kk < it.nk;
      const int64_t gk = sd.k_off + it.k0 + min(kk, max(it.nk - 1, 0));
      const int32_t a = m[3 * gk], b = m[3 * gk + 1], d = m[3 * gk + 2];
      mx[c] = ok ? (double)a : 0.0;
      my[c] = ok ? (double)b : 0.0;
      mz[c] = ok ? (double)d : 0.0;
    }
    __syncthreads();   // the previous item's readers of tile and red are done
    for (int i = tid; i < 4 * PWP; i += 256) {
      const int wv = i / PWP, sl = i % PWP;
      const int pi = wv * PW + sl;
      Pt v = {0.0, 0.0, 0.0, 0.0}, qg = {0.0, 0.0, 0.0, 0.0};
      if (sl < PW && pi < cnt) {
        const int64_t gi = sd.n_off + first + pi;
        v.sx = table_coord(x[gi], invL);
        v.sy = table_coord(y[gi], invL);
        v.sz = table_coord(z[gi], invL);
        v.q = q[gi];
        if (VJP) qg = Pt{v.q * gF[gi], v.q * gF[n_total + gi], v.q * gF[2 * n_total + gi], 0.0};
      }
      tile[i] = v;
      if (VJP) tgw[i] = qg;
    }
    __syncthreads();
    double acc[2 * KPL];
#pragma unroll
    for (int c = 0; c < 2 * KPL; ++c) acc[c] = 0.0;
    if (g < G) {
      const Pt* tp = tile + wave * PWP + g;
      const Pt* gp = tgw + (VJP ? wave * PWP + g : 0);
      for (int j = 0; j < STEPS; ++j) {
        const Pt v = tp[j * G];
        Pt qg = {0.0, 0.0, 0.0, 0.0};
        if (VJP) qg = gp[j * G];
#pragma unroll
        for (int c = 0; c < KPL; ++c) {
          double sn, cs;
          sincos_phase_tab(dot_f64(mx[c], my[c], mz[c], v.sx, v.sy, v.sz), turns, &sn, &cs);
          double wt = v.q;
          if (VJP) wt = fma(qg.sx, mx[c], fma(qg.sy, my[c], qg.sz * mz[c]));
          acc[c] = fma(wt, cs, acc[c]);
          acc[KPL + c] = fma(wt, sn, acc[KPL + c]);
        }
      }
    }
    // the G subgroups of the wave (lanes kl, kl + KL, ...) in a fixed order
#pragma unroll
    for (int c = 0; c < 2 * KPL; ++c) {
      double sum = 0.0;
#pragma unroll
      for (int gg = 0; gg < G; ++gg) sum += __shfl(acc[c], kl + KL * gg, 64);
      if (g == 0) red[wave][c][kl] = sum;
    }
    __syncthreads();
    double* part = w.partials + 2 * sd.part_off;
    for (int o = tid; o < 2 * it.nk; o += 256) {
      const int kk = o >> 1, comp = o & 1;
      const int c = kk / KL, r = kk % KL;
      double sum = 0.0;
#pragma unroll
      for (int wv = 0; wv < 4; ++wv) sum += red[wv][comp * KPL + c][r];
      const int64_t kidx = it.k0 + kk;
      part[2 * (kidx * sd.ntiles + it.tile) + comp] = sum;
    }
  }
}

// ------------------------------------------------------------------ rho pass, FP64

template <int NPL, int KC, bool VJP, int WPB>
__global__ __launch_bounds__(64 * WPB) void rho_f64_kernel(WsView w, const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ q,
                                                          const int32_t* __restrict__ m,
                                                          const double* __restrict__ gF, int64_t n_total,
                                                          int32_t n_items) {
  __shared__ int32_t sched_lds[WPB == kCoopWaves ? 2 * kCoopWaves : 1];
  __shared__ double2 turns[kTurnRows];
  build_turn_table(turns);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  RhoSchedule<WPB> sched(n_items, wave, sched_lds);

  double sx[NPL], sy[NPL], sz[NPL], qv[NPL];
  double qgx[VJP ? NPL : 1], qgy[VJP ? NPL : 1], qgz[VJP ? NPL : 1];
  int32_t cur_sys = -1, cur_tile = -1;   // tile held in registers

  for (int32_t item = sched.first(); item >= 0; item = sched.next()) {
    // the item index is wave-uniform; saying so keeps the item and its wave vectors in
    // scalar registers and scalar loads
    const RhoItem it = w.rho_items[__builtin_amdgcn_readfirstlane(item)];
    const SysDesc sd = w.sys[it.sys];
    if (it.sys != cur_sys || it.tile != cur_tile) {
      cur_sys = it.sys;
      cur_tile = it.tile;
      const int first = it.tile * (64 * NPL);
      const int cnt = min(64 * NPL, sd.n - first);
      const double invL = 1.0 / sd.L;
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const int li = j * 64 + lane;
        if (li < cnt) {
          const int64_t gi = sd.n_off + first + li;
          sx[j] = table_coord(x[gi], invL);
          sy[j] = table_coord(y[gi], invL);
          sz[j] = table_coord(z[gi], invL);
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
    }
    double* part = w.partials + 2 * sd.part_off;
    const int32_t* mk = m + 3 * (sd.k_off + it.k0);

    for (int kc = 0; kc < it.nk; kc += KC) {
      sched.priority((it.nk - kc + KC - 1) / KC);
      double mx[KC], my[KC], mz[KC];
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const int kk = min(kc + c, it.nk - 1);
        const int32_t a = mk[3 * kk], b = mk[3 * kk + 1], d = mk[3 * kk + 2];
        const bool ok = kc + c < it.nk;
        mx[c] = ok ? (double)a : 0.0;
        my[c] = ok ? (double)b : 0.0;
        mz[c] = ok ? (double)d : 0.0;
      }
      double acc[2 * KC];
#pragma unroll
      for (int c = 0; c < 2 * KC; ++c) acc[c] = 0.0;
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          double sn, cs;
          sincos_phase_tab(dot_f64(mx[c], my[c], mz[c], sx[j], sy[j], sz[j]), turns, &sn, &cs);
          double wt = qv[j];
          if (VJP) wt = fma(qgx[j], mx[c], fma(qgy[j], my[c], qgz[j] * mz[c]));
          acc[c] = fma(wt, cs, acc[c]);
          acc[KC + c] = fma(wt, sn, acc[KC + c]);
        }
      }
      wave_reduce_scatter<2 * KC>(acc, lane);
      if (lane < 2 * KC) {
        const int vi = scatter_index(lane, Log2<2 * KC>::value);
        const int c = vi % KC;
        const int comp = vi / KC;
        if (kc + c < it.nk) {
          const int64_t kl = it.k0 + kc + c;
          part[2 * (kl * sd.ntiles + it.tile) + comp] = acc[0];
        }
      }
    }
  }
}

// ------------------------------------------------------------------ cross-tile reduction

// Force-pass row of wave vector g of system sd from the reduced rho (C, S): c_l from the
// weight and |k_l|^2, rho rotated by exp(-i delta) back onto the truncated phases of the
// FP32-mixed form (delta = 0 otherwise), and from it the amplitude R_l and the phase offset
// delta_l of the one-cosine form of the force term.
__device__ inline ForceRowF32 force_row(const SysDesc& sd, int64_t g, const int32_t* __restrict__ m,
                                        const double* __restrict__ wk, double C, double S, double rot_c,
                                        double rot_s) {
  const double invL = 1.0 / sd.L;
  const double kscale = kTwoPi * invL;
  const double vol = sd.L * sd.L * sd.L;
  const int32_t mx = m[3 * g], my = m[3 * g + 1], mz = m[3 * g + 2];
  const double k2 = kscale * kscale * ((double)mx * mx + (double)my * my + (double)mz * mz);
  const double c = (k2 > 0.0) ? wk[g] * kFourPi / (vol * k2) : 0.0;
  const double Cr = C * rot_c + S * rot_s;
  const double Sr = S * rot_c - C * rot_s;
  const double R = c * sqrt(Cr * Cr + Sr * Sr);
  // delta = 1/4 - arg(rho') / (2 pi), reduced to [0, 1): R cos(theta + 2 pi delta)
  // = R sin(arg(rho') - theta) = c (S' cos theta - C' sin theta)
  double dl = 0.25 - atan2(Sr, Cr) / kTwoPi;
  dl -= floor(dl);
  if (!(dl >= 0.0 && dl < 1.0)) dl = 0.0;   // non-finite rho: R is NaN and carries it
  ForceRowF32 r;
  r.d = (uint32_t)(uint64_t)llrint(dl * 4294967296.0);   // 2^32 wraps to 0
  r.mx = mx; r.my = my; r.mz = mz;
  r.gx = r.hx = (float)(R * mx);
  r.gy = r.hy = (float)(R * my);
  r.gz = r.hz = (float)(R * mz);
  r.pad0 = 0.0f;
  r.fx = (float)mx; r.fy = (float)my; r.fz = (float)mz;
  r.dt = (float)dl;
  r.r = (float)R;
  return r;
}

// One block per wave vector: out[g] = sum over the system's tiles of partial[g][tile].
// Thread t sums tiles t, t + 256, ... in order, each wave combines its lanes with a fixed
// butterfly, and thread 0 adds the four wave sums in order; the result is optionally
// rotated by exp(i delta).  With ROWS, thread 0 also writes the wave vector's force row.
template <bool ROWS>
__global__ __launch_bounds__(kReduceBlock) void reduce_kernel(WsView w, double* __restrict__ out,
                                                              double rot_c, double rot_s,
                                                              const int32_t* __restrict__ m,
                                                              const double* __restrict__ wk) {
  constexpr int kWaves = kReduceBlock / 64;
  __shared__ double wsum[2][kWaves];
  const int64_t g = blockIdx.x;
  const int tid = threadIdx.x;
  const KRed r = w.kred[g];
  // (re, im) pairs: 16-byte aligned (the workspace and every partial slot are)
  const double2* src = reinterpret_cast<const double2*>(w.partials) + r.slot;
  double re = 0.0, im = 0.0;
#pragma unroll 4
  for (int t = tid; t < r.ntiles; t += kReduceBlock) {
    const double2 v = src[t];
    re += v.x;
    im += v.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o, 64);
    im += __shfl_xor(im, o, 64);
  }
  if ((tid & 63) == 0) {
    wsum[0][tid >> 6] = re;
    wsum[1][tid >> 6] = im;
  }
  __syncthreads();
  if (tid == 0) {
    re = wsum[0][0];
    im = wsum[1][0];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) {
      re += wsum[0][i];
      im += wsum[1][i];
    }
    const double C = re * rot_c - im * rot_s;
    const double S = re * rot_s + im * rot_c;
    out[2 * g] = C;
    out[2 * g + 1] = S;
    if (ROWS) w.frows[g] = force_row(w.sys[r.sys], g, m, wk, C, S, rot_c, rot_s);
  }
}

// Force rows of every wave vector from a given rho (a force pass without a reduction before it).
__global__ __launch_bounds__(kReduceBlock) void force_rows_kernel(WsView w, int64_t p_total,
                                                                  const int32_t* __restrict__ m,
                                                                  const double* __restrict__ wk,
                                                                  const double* __restrict__ rho,
                                                                  double rot_c, double rot_s) {
  const int64_t g = (int64_t)blockIdx.x * kReduceBlock + threadIdx.x;
  if (g >= p_total) return;
  w.frows[g] = force_row(w.sys[w.kred[g].sys], g, m, wk, rho[2 * g], rho[2 * g + 1], rot_c, rot_s);
}

// ------------------------------------------------------------------ virial

// k-space virial tensor of system b (one block per system), the negative derivative of
// the long-range energy term under a symmetric strain at fixed fractional coordinates:
//   W_ab = sum_l U_l (delta_ab - 2 k_la k_lb (1/k_l^2 + 1/(4 alpha))),  U_l = (c_l/2)|rho_l|^2.
// The 1/(4 alpha) part is the strain derivative of the Ewald kernel exp(-k^2/4 alpha); with
// RBE weights the sum is the importance-sampled estimate of the Ewald virial.  Thread t
// sums k = t, t + 256, ... in order, then a fixed tree per component; W[6b ..] = xx, yy,
// zz, xy, xz, yz.
__global__ __launch_bounds__(kReduceBlock) void virial_kernel(WsView w, const int32_t* __restrict__ m,
                                                              const double* __restrict__ wk,
                                                              const double* __restrict__ rho,
                                                              double* __restrict__ W) {
  __shared__ double red[6][kReduceBlock];
  const SysDesc sd = w.sys[blockIdx.x];
  const int tid = threadIdx.x;
  const double kscale = kTwoPi / sd.L;
  const double vol = sd.L * sd.L * sd.L;
  const double g4 = 1.0 / (4.0 * sd.alpha);
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int l = tid; l < sd.p; l += kReduceBlock) {
    const int64_t g = sd.k_off + l;
    const double kx = kscale * m[3 * g], ky = kscale * m[3 * g + 1], kz = kscale * m[3 * g + 2];
    const double k2 = kx * kx + ky * ky + kz * kz;
    if (k2 > 0.0) {
      const double c = wk[g] * kFourPi / (vol * k2);
      const double u = 0.5 * c * (rho[2 * g] * rho[2 * g] + rho[2 * g + 1] * rho[2 * g + 1]);
      const double f = 2.0 * (1.0 / k2 + g4);
      acc[0] += u * (1.0 - f * kx * kx);
      acc[1] += u * (1.0 - f * ky * ky);
      acc[2] += u * (1.0 - f * kz * kz);
      acc[3] -= u * f * kx * ky;
      acc[4] -= u * f * kx * kz;
      acc[5] -= u * f * ky * kz;
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) red[c][tid] = acc[c];
  __syncthreads();
  for (int h = kReduceBlock / 2; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int c = 0; c < 6; ++c) red[c][tid] += red[c][tid + h];
    }
    __syncthreads();
  }
  if (tid < 6) W[6 * (int64_t)blockIdx.x + tid] = red[tid][0];
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

// The force kernel's LDS table row: the two quarters of a ForceRowF32 that its form reads
// (fixed-point phases: quarters 0 and 1; FP32 phases and the phase cache: 2 and 3; the
// phase-cache pass stores m as float, c S', c C' instead).
struct TabF32 { int4 lo, hi; };

// A row as the phase-cache pass keeps it: (m as float, c S') and (c C', 0, 0, 0), where
// c S' = R cos(2 pi delta) and c C' = R sin(2 pi delta).
__device__ inline TabF32 cached_tab_row(int4 q2, int4 q3) {
  const float dt = __int_as_float(q2.w), R = __int_as_float(q3.w);
  const float a = R * __builtin_amdgcn_cosf(dt), b = R * __builtin_amdgcn_sinf(dt);
  return TabF32{make_int4(q2.x, q2.y, q2.z, __float_as_int(a)), make_int4(__float_as_int(b), 0, 0, 0)};
}

template <int NPLF, bool CACHED, bool FPH>
__global__ __launch_bounds__(kForceBlock) void force_f32_kernel(
    WsView w, int64_t n_total, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ q, const int32_t* __restrict__ m,
    const double* __restrict__ wk, const double* __restrict__ rho, const ForceRowF32* __restrict__ frows,
    float* __restrict__ F, double* __restrict__ U, int32_t n_items, uint64_t* __restrict__ counter, SysDesc sys0,
    int32_t single) {
  static_assert(kTabChunk == kForceBlock, "one table row per thread and chunk");
  __shared__ __align__(16) TabF32 tab[kTabChunk];
  __shared__ double red[kForceBlock];
for (int32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
  // with one system the item and the system follow from the block index and the arguments
  // (the items are consecutive particle ranges of 256 NPLF), so no load precedes the
  // particle and row loads
  ForceItem it;
  SysDesc sd;
  if (single) {
    const int p0 = item * (kForceBlock * NPLF);
    it = ForceItem{0, p0, max(0, min(kForceBlock * NPLF, sys0.n - p0)), item == 0 ? 1 : 0};
    sd = sys0;
  } else {
    it = w.force_items[item];
    sd = w.sys[it.sys];
  }
  const int tid = threadIdx.x;
  const double invL = 1.0 / sd.L;
  const double kscale = kTwoPi * invL;
  const double vol = sd.L * sd.L * sd.L;
  // this thread's row of the first table chunk (two 16-byte halves), requested before the
  // particles so that the two loads overlap.  The load is unconditional (a valid address for
  // every thread: a clamped row, or the system table when the system has no rows), so the
  // particle loads need not wait for it; only rows e < P are stored.
  constexpr int kQ0 = (CACHED || FPH) ? 2 : 0;   // first quarter of a row this form reads
  const int4* rows = reinterpret_cast<const int4*>(frows + sd.k_off);
  const int4* r0 = sd.p > 0 ? rows + 4 * min(tid, sd.p - 1) + kQ0 : reinterpret_cast<const int4*>(w.sys);
  const int4 row0a = r0[0], row0b = r0[1];

  using Ph = Phase<FPH>;
  typename Ph::Coord ux[NPLF], uy[NPLF], uz[NPLF];
  float fx[NPLF], fy[NPLF], fz[NPLF];
  int li[NPLF];
  double cx[NPLF], cy[NPLF], cz[NPLF];   // the particles as loaded
  float bad[NPLF];                        // 0, or NaN for a non-finite position
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    li[j] = it.p0 + j * kForceBlock + tid;
    const bool ok = j * kForceBlock + tid < it.np;
    cx[j] = cy[j] = cz[j] = 0.0;
    if (ok && !CACHED) {
      const int64_t gi = sd.n_off + li[j];
      cx[j] = x[gi];
      cy[j] = y[gi];
      cz[j] = z[gi];
    }
    fx[j] = fy[j] = fz[j] = 0.0f;
  }
  // the first chunk's rows go to LDS as soon as they arrive (once the previous item's
  // readers are done), which frees their registers before the particles are converted
  __syncthreads();
  if (tid < min(kTabChunk, sd.p)) tab[tid] = CACHED ? cached_tab_row(row0a, row0b) : TabF32{row0a, row0b};
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    if (j * kForceBlock + tid < it.np && !CACHED) {
      ux[j] = Ph::coord(cx[j], invL);
      uy[j] = Ph::coord(cy[j], invL);
      uz[j] = Ph::coord(cz[j], invL);
    } else {
      ux[j] = uy[j] = uz[j] = 0;
    }
    bad[j] = (float)finite_or_nan(0.0, cx[j], cy[j], cz[j]);
  }
  for (int t0 = 0; t0 < sd.p; t0 += kTabChunk) {
    const int cnt = min(kTabChunk, sd.p - t0);
    if (t0 > 0) {
      __syncthreads();
      if (tid < cnt) {
        const int4 lo = rows[4 * (t0 + tid) + kQ0], hi = rows[4 * (t0 + tid) + kQ0 + 1];
        tab[tid] = CACHED ? cached_tab_row(lo, hi) : TabF32{lo, hi};
      }
    }
    // zero rows pad the chunk to a multiple of kUnroll (m = 0, R = a = b = 0: no contribution)
    const int cntp = (cnt + kUnroll - 1) / kUnroll * kUnroll;
    for (int e = cnt + tid; e < cntp; e += kForceBlock) tab[e] = TabF32{make_int4(0, 0, 0, 0), make_int4(0, 0, 0, 0)};
    __syncthreads();
    for (int e = 0; e < cntp; e += kUnroll) {
      TabF32 tb[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) tb[u] = tab[e + u];
#pragma unroll
      for (int j = 0; j < NPLF; ++j) {
        if (CACHED) {
          // g = c (S' cos - C' sin) from the cached (cos, sin); quarters 2 and 3: m as float,
          // c S', c C'
          float sn[kUnroll], cs[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            if (j * kForceBlock + tid < it.np && e + u < cnt) {
              const float2 v = reinterpret_cast<const float2*>(w.cache)[sd.cache_off + (int64_t)(t0 + e + u) * sd.n + li[j]];
              cs[u] = v.x;
              sn[u] = v.y;
            } else {
              cs[u] = sn[u] = 0.0f;
            }
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const float g = __int_as_float(tb[u].lo.w) * cs[u] - __int_as_float(tb[u].hi.x) * sn[u];
            fx[j] = fmaf(g, __int_as_float(tb[u].lo.x), fx[j]);
            fy[j] = fmaf(g, __int_as_float(tb[u].lo.y), fy[j]);
            fz[j] = fmaf(g, __int_as_float(tb[u].lo.z), fz[j]);
          }
        } else {
          // one cosine per term: m_l g = (R_l m_l) cos(theta + 2 pi delta_l), the offset
          // entering the phase as its first addend
          float a[kUnroll], gx[kUnroll], gy[kUnroll], gz[kUnroll];
          int32_t rmx[kUnroll], rmy[kUnroll], rmz[kUnroll];
          uint64_t rd[kUnroll];
          float rfx[kUnroll], rfy[kUnroll], rfz[kUnroll], rdt[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            if (FPH) {   // quarter 2: m as float, delta in turns; quarter 3: R m
              rfx[u] = __int_as_float(tb[u].lo.x); rfy[u] = __int_as_float(tb[u].lo.y);
              rfz[u] = __int_as_float(tb[u].lo.z); rdt[u] = __int_as_float(tb[u].lo.w);
              gx[u] = __int_as_float(tb[u].hi.x); gy[u] = __int_as_float(tb[u].hi.y);
              gz[u] = __int_as_float(tb[u].hi.z);
              rmx[u] = rmy[u] = rmz[u] = 0;
              rd[u] = 0u;
            } else {     // quarter 0: the offset and m; quarter 1: R m.  The 64-bit addend is
                         // the register pair (d, m_x) as loaded: its high word does not reach
                         // the low 32 bits of the sum, which are all the phase uses
              rd[u] = ((uint64_t)(uint32_t)tb[u].lo.y << 32) | (uint32_t)tb[u].lo.x;
              rmx[u] = tb[u].lo.y; rmy[u] = tb[u].lo.z; rmz[u] = tb[u].lo.w;
              gx[u] = __int_as_float(tb[u].hi.x); gy[u] = __int_as_float(tb[u].hi.y);
              gz[u] = __int_as_float(tb[u].hi.z);
              rfx[u] = rfy[u] = rfz[u] = rdt[u] = 0.0f;
            }
          }
          Ph::template args_off<kUnroll>(rmx, rmy, rmz, rfx, rfy, rfz, rd, rdt, ux[j], uy[j], uz[j], a);
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const float cs = __builtin_amdgcn_cosf(a[u]);
            fx[j] = fmaf(gx[u], cs, fx[j]);
            fy[j] = fmaf(gy[u], cs, fy[j]);
            fz[j] = fmaf(gz[u], cs, fz[j]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    if (j * kForceBlock + tid < it.np) {
      const int64_t gi = sd.n_off + li[j];
      const double s = -(q[gi] + bad[j]) * kscale;
      F[gi] = (float)(s * fx[j]);
      F[n_total + gi] = (float)(s * fy[j]);
      F[2 * n_total + gi] = (float)(s * fz[j]);
    }
  }
  if (it.flags & 1) {
    // energy of the system in FP64: U = sum_l (c_l / 2) |rho_l|^2, thread t over l = t, t + 256, ...
    double usum = 0.0;
    for (int l = tid; l < sd.p; l += kForceBlock) {
      const int64_t g = sd.k_off + l;
      const int32_t mx = m[3 * g], my = m[3 * g + 1], mz = m[3 * g + 2];
      const double k2 = kscale * kscale * ((double)mx * mx + (double)my * my + (double)mz * mz);
      const double c = (k2 > 0.0) ? wk[g] * kFourPi / (vol * k2) : 0.0;
      const double C = rho[2 * g], S = rho[2 * g + 1];
      usum += 0.5 * c * (C * C + S * S);
    }
    const double tot = block_sum(usum, red);
    if (tid == 0) {
      U[it.sys] = tot;
      // graph replays: advance the device step counter the sampler reads
      if (counter != nullptr && it.sys == 0) counter[0] += 1;
    }
  }
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
    double* __restrict__ U, int32_t n_items, uint64_t* __restrict__ counter) {
  __shared__ TabF64 tab[kTabChunk];
  __shared__ double red[kForceBlock];
  __shared__ double2 turns[kTurnRows];
  build_turn_table(turns);   // the item loop's first barrier precedes every use
for (int32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
  const ForceItem it = w.force_items[item];
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
      sx[j] = table_coord(x[gi], invL);
      sy[j] = table_coord(y[gi], invL);
      sz[j] = table_coord(z[gi], invL);
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
        sincos_phase_tab(dot_f64(tb.mx, tb.my, tb.mz, sx[j], sy[j], sz[j]), turns, &sn, &cs);
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
    if (tid == 0) {
      U[it.sys] = tot;
      // graph replays: advance the device step counter the sampler reads
      if (counter != nullptr && it.sys == 0) counter[0] += 1;
    }
  }
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

template <int NPLF, bool FPH>
__global__ __launch_bounds__(kForceBlock) void vjp_b2_f32_kernel(
    WsView w, int64_t n_total, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ q, const int32_t* __restrict__ m,
    const double* __restrict__ wk, const double* __restrict__ rho, const double* __restrict__ gU,
    const float* __restrict__ gF, double* __restrict__ gr, double* __restrict__ gq, double rot_c,
    double rot_s, int32_t n_items) {
  __shared__ TabAdjF32 tab[kTabChunk];
for (int32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
  const ForceItem it = w.force_items[item];
  const SysDesc sd = w.sys[it.sys];
  const int tid = threadIdx.x;
  const double invL = 1.0 / sd.L;
  const double kscale = kTwoPi * invL;
  const double vol = sd.L * sd.L * sd.L;
  const double gu = gU[it.sys];

  using Ph = Phase<FPH>;
  typename Ph::Coord ux[NPLF], uy[NPLF], uz[NPLF];
  float gx[NPLF], gy[NPLF], gz[NPLF], rx[NPLF], ry[NPLF], rz[NPLF], rq[NPLF];
#pragma unroll
  for (int j = 0; j < NPLF; ++j) {
    const bool ok = j * kForceBlock + tid < it.np;
    if (ok) {
      const int64_t gi = sd.n_off + it.p0 + j * kForceBlock + tid;
      ux[j] = Ph::coord(x[gi], invL);
      uy[j] = Ph::coord(y[gi], invL);
      uz[j] = Ph::coord(z[gi], invL);
      gx[j] = gF[gi];
      gy[j] = gF[n_total + gi];
      gz[j] = gF[2 * n_total + gi];
    } else {
      ux[j] = uy[j] = uz[j] = 0;
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
        const float a = Ph::arg(tb.mx, tb.my, tb.mz, tb.fx, tb.fy, tb.fz, ux[j], uy[j], uz[j]);
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
      gr[gi] = s * rx[j];
      gr[n_total + gi] = s * ry[j];
      gr[2 * n_total + gi] = s * rz[j];
      gq[gi] = rq[j];
    }
  }
  }
}

template <int NPLF>
__global__ __launch_bounds__(kForceBlock) void vjp_b2_f64_kernel(
    WsView w, int64_t n_total, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ q, const int32_t* __restrict__ m,
    const double* __restrict__ wk, const double* __restrict__ rho, const double* __restrict__ gU,
    const double* __restrict__ gF, double* __restrict__ gr, double* __restrict__ gq, int32_t n_items) {
  __shared__ double tabm[kTabChunk][3];
  __shared__ AdjTab tab[kTabChunk];
  __shared__ double2 turns[kTurnRows];
  build_turn_table(turns);   // the item loop's first barrier precedes every use
for (int32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
  const ForceItem it = w.force_items[item];
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
      sx[j] = table_coord(x[gi], invL);
      sy[j] = table_coord(y[gi], invL);
      sz[j] = table_coord(z[gi], invL);
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
        sincos_phase_tab(dot_f64(mx, my, mz, sx[j], sy[j], sz[j]), turns, &sn, &cs);
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
}

// ------------------------------------------------------------------ sampler

// One block per system, its inverse-CDF table staged in LDS when it fits (else read
// from the workspace).  Thread t draws wave vectors t, t + 128, ... of the system with
// Philox key (seed + b, stream_id), counter (l, attempt, 0, 0); a zero vector is redrawn.
constexpr int kSampleBlock = 128;

// The three components' inverse-CDF searches in lockstep (the same number of halvings,
// so their table reads overlap): for each t, the smallest j in [-M, M] with
// t < c[j + M], or M if there is none -- the same result as inverse_cdf.
__device__ inline void inverse_cdf3(const double* c, int32_t M, const double (&t)[3], int32_t (&v)[3]) {
  const int32_t n = 2 * M + 1;
  int32_t base[3] = {0, 0, 0};
  for (int32_t len = n; len > 1;) {
    const int32_t half = len >> 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) base[d] = (c[base[d] + half - 1] <= t[d]) ? base[d] + half : base[d];
    len -= half;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int32_t idx = base[d] + (c[base[d]] <= t[d] ? 1 : 0);
    v[d] = idx >= n ? M : idx - M;
  }
}

__global__ __launch_bounds__(kSampleBlock) void sample_kernel(WsView w, uint64_t seed, uint64_t stream_base,
                                                              const uint64_t* __restrict__ counter,
                                                              int32_t stride, int32_t in_lds, int32_t sampler,
                                                              int32_t burn_in, int32_t* __restrict__ m,
                                                              double* __restrict__ wk) {
  extern __shared__ double table[];
  const int32_t b = blockIdx.x;
  // the stream id is stream_base plus the device step counter when one is given
  const uint64_t stream_id = stream_base + (counter != nullptr ? counter[0] : 0ull);
  // the table's address follows from b alone, so its load overlaps the counter's
  const double* h = w.cdf + (int64_t)b * stride;
  if (in_lds) {
    for (int i = threadIdx.x; i < stride; i += kSampleBlock) table[i] = h[i];
    __syncthreads();
    h = table;
  }
  const double S = h[0];
  const int32_t len = (int32_t)h[1];
  const int32_t np = (int32_t)h[2];
  const int64_t k_off = (int64_t)h[3];
  if (np == 0 || len == 0) return;
  const double* c = h + kCdfHeader;
  const int32_t M = (len - 1) / 2;
  const double Z = c[2 * M];
  if (sampler == RBE_SAMPLER_METROPOLIS) {
    // one Metropolis chain per wave vector (the table is not read)
    const int32_t D = (int32_t)h[4];
    const double beta = h[5];
    for (int32_t l = threadIdx.x; l < np; l += kSampleBlock) {
      int32_t v[3];
      metropolis_chain(seed + (uint64_t)b, stream_id, (uint64_t)l, burn_in, D, beta, v);
      const int64_t g = k_off + l;
      m[3 * g] = v[0];
      m[3 * g + 1] = v[1];
      m[3 * g + 2] = v[2];
      wk[g] = S / (double)np;
    }
    return;
  }
  for (int32_t l = threadIdx.x; l < np; l += kSampleBlock) {
    int32_t v[3] = {0, 0, 0};
    for (int a = 0; a < kMaxAttempts; ++a) {
      U64x4 ctr = {{(uint64_t)l, (uint64_t)a, 0ull, 0ull}};
      const U64x4 r = philox4x64_10(ctr, seed + (uint64_t)b, stream_id);
      const double t[3] = {u01_53(r.v[0]) * Z, u01_53(r.v[1]) * Z, u01_53(r.v[2]) * Z};
      inverse_cdf3(c, M, t, v);
      if (v[0] != 0 || v[1] != 0 || v[2] != 0) break;
    }
    const int64_t g = k_off + l;
    m[3 * g] = v[0];
    m[3 * g + 1] = v[1];
    m[3 * g + 2] = v[2];
    wk[g] = (v[0] != 0 || v[1] != 0 || v[2] != 0) ? S / (double)np : 0.0;
  }
}

// ------------------------------------------------------------------ dispatch helpers

// Blocks of a pass: one per work item, or at most `cap` persistent blocks that stride
// over the items (cap = 0: no cap).
dim3 grid_for(int32_t n_items, int32_t cap) {
  return dim3((unsigned)((cap > 0 && cap < n_items) ? cap : n_items));
}

// Occupancy clamp of the rho-shaped passes.  Their waves are few per SIMD (about
// items / (4 x CUs)); if the previous kernel's tail frees some CUs early, the dispatcher
// would pack those CUs up to their register-limited occupancy and leave the rest short.
// Reserving unused LDS per block caps the 4-wave blocks per CU at
// ceil(items / (4 x CUs)), so every CU gets its share wherever the blocks land.
size_t occupancy_clamp_lds(int32_t n_waves, size_t static_bytes) {
  static int cus = 0, lds_per_cu = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        cus <= 0 || lds_per_cu <= 0) {
      cus = -1;
    }
  }
  if (cus <= 0) return 0;
  const int64_t per_simd = std::max<int64_t>((n_waves + 4LL * cus - 1) / (4LL * cus), 1);
  // the share less the kernel's own static LDS, with 256 bytes to spare
  const int64_t bytes = (int64_t)(lds_per_cu / per_simd) / 256 * 256 - 256 - (int64_t)static_bytes;
  return (size_t)std::min<int64_t>(std::max<int64_t>(bytes, 0), 64 * 1024);
}

int num_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    cus = (hipGetDevice(&dev) == hipSuccess &&
           hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
              ? v
              : 256;
  }
  return cus;
}

// Blocks of the rho-shaped passes.  WPB = 4: one wave per item (at most cap waves when
// cap > 0).  WPB = 16: one block per CU (fewer for small item counts, at most cap / 16).
dim3 rho_grid(int32_t n_items, int32_t cap, int wpb) {
  if (wpb == kCoopWaves) {
    int64_t blocks = std::min<int64_t>(num_cus(), ((int64_t)n_items + kCoopWaves - 1) / kCoopWaves);
    if (cap > 0) blocks = std::min<int64_t>(blocks, ((int64_t)cap + kCoopWaves - 1) / kCoopWaves);
    return dim3((unsigned)std::max<int64_t>(blocks, 1));
  }
  const int32_t waves = (cap > 0 && cap < n_items) ? cap : n_items;
  return dim3((unsigned)((waves + 3) / 4));
}

template <int NPL, int KC, bool CACHE, bool VJP, bool FPH, int WPB>
void launch_rho_f32_t(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const float* gF,
                      hipStream_t st) {
  const dim3 grid = rho_grid(s.n_rho_items, s.rho_grid_cap, WPB);
  const size_t lds = (WPB == 4 && s.rho_clamp) ? occupancy_clamp_lds((int32_t)grid.x * 4, 0) : 0;
  hipLaunchKernelGGL((rho_f32_kernel<NPL, KC, CACHE, VJP, FPH, WPB>), grid, dim3(64 * WPB), lds, st, w, x, y, z,
                     q, m, gF, s.n_total, s.n_rho_items);
}

template <int NPL, int KC, bool VJP, int WPB>
void launch_rho_f64_t(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const double* gF,
                      hipStream_t st) {
  const dim3 grid = rho_grid(s.n_rho_items, s.rho_grid_cap, WPB);
  const size_t lds = (WPB == 4 && s.rho_clamp) ? occupancy_clamp_lds((int32_t)grid.x * 4, sizeof(double2) * kTurnRows) : 0;
  hipLaunchKernelGGL((rho_f64_kernel<NPL, KC, VJP, WPB>), grid, dim3(64 * WPB), lds, st, w, x, y, z, q, m, gF,
                     s.n_total, s.n_rho_items);
}

// FP64 k-lane rho pass: one 256-thread block per item (rho_grid_cap counts waves, four a block)
template <int TILE, int G, int KPL, bool VJP>
void launch_rho_klane_f64_t(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                            const double* z, const double* q, const int32_t* m, const double* gF, hipStream_t st) {
  int32_t blocks = s.n_rho_items;
  if (s.rho_grid_cap > 0) blocks = std::min<int32_t>(blocks, std::max<int32_t>((s.rho_grid_cap + 3) / 4, 1));
  hipLaunchKernelGGL((rho_klane_f64_kernel<TILE, G, KPL, VJP>), dim3((unsigned)std::max<int32_t>(blocks, 1)),
                     dim3(256), 0, st, w, x, y, z, q, m, gF, s.n_total, s.n_rho_items);
}

// k-lane rho pass: one 256-thread block per item (rho_grid_cap counts waves, four a block)
template <int TILE, int G, int KPL, bool VJP, bool FPH>
void launch_rho_klane_t(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                        const double* z, const double* q, const int32_t* m, const float* gF, hipStream_t st) {
  int32_t blocks = s.n_rho_items;
  if (s.rho_grid_cap > 0) blocks = std::min<int32_t>(blocks, std::max<int32_t>((s.rho_grid_cap + 3) / 4, 1));
  if constexpr (VJP)
    hipLaunchKernelGGL((rho_klane_vjp_kernel<TILE, G, KPL, FPH>), dim3((unsigned)std::max<int32_t>(blocks, 1)),
                       dim3(256), 0, st, w, x, y, z, q, m, gF, s.n_total, s.n_rho_items);
  else if (s.rv.comp)
    hipLaunchKernelGGL((rho_klane_comp_kernel<TILE, G, KPL, FPH>), dim3((unsigned)std::max<int32_t>(blocks, 1)),
                       dim3(256), 0, st, w, x, y, z, q, m, s.n_total, s.n_rho_items);
  else
    hipLaunchKernelGGL((rho_klane_kernel<TILE, G, KPL, FPH>), dim3((unsigned)std::max<int32_t>(blocks, 1)),
                       dim3(256), 0, st, w, x, y, z, q, m, s.n_total, s.n_rho_items);
}

// Particle-tile pass over every (tile, k-range) item; VJP selects adjoint pass B1.
template <bool CACHE, bool VJP, bool FPH>
void tile_pass_f32(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                   const double* z, const double* q, const int32_t* m, const float* g, hipStream_t st) {
  switch (s.rv.wpb * 10000 + s.rv.npl * 100 + s.rv.kc) {
    case 10805:
    case 10405:
      // the k-lane layout (3 x 21 lanes, 5 wave vectors each) computes the forward pass and
      // pass B1; the phase cache uses the per-wave kernel on the same tiles (of 64 npl
      // particles: the plan gives k-lane variants those tiles in that mode)
      if constexpr (!CACHE) {
        if (s.rv.tile == 512) launch_rho_klane_t<512, 3, 5, VJP, FPH>(s, w, x, y, z, q, m, g, st);
        else if (s.rv.tile == 492) launch_rho_klane_t<492, 3, 5, VJP, FPH>(s, w, x, y, z, q, m, g, st);
        else launch_rho_klane_t<256, 3, 5, VJP, FPH>(s, w, x, y, z, q, m, g, st);
      } else {
        if (s.rv.npl == 8) launch_rho_f32_t<8, 8, CACHE, VJP, FPH, 4>(s, w, x, y, z, q, m, g, st);
        else launch_rho_f32_t<4, 8, CACHE, VJP, FPH, 4>(s, w, x, y, z, q, m, g, st);
      }
      break;
    case 160808: launch_rho_f32_t<8, 8, CACHE, VJP, FPH, 16>(s, w, x, y, z, q, m, g, st); break;
    case 160804: launch_rho_f32_t<8, 4, CACHE, VJP, FPH, 16>(s, w, x, y, z, q, m, g, st); break;
    case 41608: launch_rho_f32_t<16, 8, CACHE, VJP, FPH, 4>(s, w, x, y, z, q, m, g, st); break;
    case 40808: launch_rho_f32_t<8, 8, CACHE, VJP, FPH, 4>(s, w, x, y, z, q, m, g, st); break;
    case 40804: launch_rho_f32_t<8, 4, CACHE, VJP, FPH, 4>(s, w, x, y, z, q, m, g, st); break;
    default: break;
  }
}

template <bool VJP>
void launch_tile_pass(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const void* gF,
                      hipStream_t st) {
  if (s.precision == RBE_FP32_MIXED) {
    const float* g = static_cast<const float*>(gF);
    if constexpr (!VJP) {
      if (s.cached != 0) {
        tile_pass_f32<true, false, false>(s, w, x, y, z, q, m, g, st);
        return;
      }
    }
    tile_pass_f32<false, VJP, false>(s, w, x, y, z, q, m, g, st);
  } else if (s.precision == RBE_FP32) {   // the plan rejects the phase cache here
    tile_pass_f32<false, VJP, true>(s, w, x, y, z, q, m, static_cast<const float*>(gF), st);
  } else {
    const double* g = static_cast<const double*>(gF);
    switch (s.rv.wpb * 10000 + s.rv.npl * 100 + s.rv.kc) {
      case 10805:
        if (s.rv.tile == 492) launch_rho_klane_f64_t<492, 3, 5, VJP>(s, w, x, y, z, q, m, g, st);
        else launch_rho_klane_f64_t<512, 3, 5, VJP>(s, w, x, y, z, q, m, g, st);
        break;
      case 160404: launch_rho_f64_t<4, 4, VJP, 16>(s, w, x, y, z, q, m, g, st); break;
      case 40804: launch_rho_f64_t<8, 4, VJP, 4>(s, w, x, y, z, q, m, g, st); break;
      case 40404: launch_rho_f64_t<4, 4, VJP, 4>(s, w, x, y, z, q, m, g, st); break;
      case 40408: launch_rho_f64_t<4, 8, VJP, 4>(s, w, x, y, z, q, m, g, st); break;
      case 40802: launch_rho_f64_t<8, 2, VJP, 4>(s, w, x, y, z, q, m, g, st); break;
      default: break;
    }
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

template <int NPLF, bool CACHED, bool FPH>
void force_f32_t(const LaunchShape& s, const WsView& w, const double* x, const double* y, const double* z,
                 const double* q, const int32_t* m, const double* wk, const double* rho, float* F, double* U,
                 uint64_t* counter, hipStream_t st) {
  hipLaunchKernelGGL((force_f32_kernel<NPLF, CACHED, FPH>), grid_for(s.n_force_items, s.force_grid_cap),
                     dim3(kForceBlock), 0, st, w, s.n_total, x, y, z, q, m, wk, rho, w.frows, F, U,
                     s.n_force_items, counter, s.sys0, s.B == 1 ? 1 : 0);
}

template <int NPLF>
void force_f64_t(const LaunchShape& s, const WsView& w, const double* x, const double* y, const double* z,
                 const double* q, const int32_t* m, const double* wk, const double* rho, double* F, double* U,
                 uint64_t* counter, hipStream_t st) {
  hipLaunchKernelGGL((force_f64_kernel<NPLF>), grid_for(s.n_force_items, s.force_grid_cap), dim3(kForceBlock),
                     0, st, w, s.n_total, x, y, z, q, m, wk, rho, F, U, s.n_force_items, counter);
}

}  // namespace

hipError_t launch_rho(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const double* wk, double* rho,
                      int rows, hipStream_t st) {
  if (s.n_rho_items > 0) {
    if (s.ev_rho_begin != nullptr) (void)hipEventRecord(s.ev_rho_begin, st);
    launch_tile_pass<false>(s, w, x, y, z, q, m, nullptr, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (s.ev_rho_end != nullptr) (void)hipEventRecord(s.ev_rho_end, st);
  }
  if (s.p_total > 0) {
    double rc, rs;
    truncation_rotation(s.precision, &rc, &rs);
    if (rows != 0 && s.precision != RBE_FP64)
      hipLaunchKernelGGL(reduce_kernel<true>, dim3((unsigned)s.p_total), dim3(kReduceBlock), 0, st, w, rho, rc, rs,
                         m, wk);
    else
      hipLaunchKernelGGL(reduce_kernel<false>, dim3((unsigned)s.p_total), dim3(kReduceBlock), 0, st, w, rho, rc,
                         rs, nullptr, nullptr);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_force(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                        const double* z, const double* q, const int32_t* m, const double* wk,
                        const double* rho, void* F, double* U, uint64_t* counter, int rows_ready,
                        hipStream_t st) {
  if (s.n_force_items == 0) return hipSuccess;
  if (s.precision != RBE_FP64 && rows_ready == 0 && s.p_total > 0) {
    double rc, rs;
    truncation_rotation(s.precision, &rc, &rs);
    hipLaunchKernelGGL(force_rows_kernel, dim3((unsigned)((s.p_total + kReduceBlock - 1) / kReduceBlock)),
                       dim3(kReduceBlock), 0, st, w, s.p_total, m, wk, rho, rc, rs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (s.ev_force_begin != nullptr) (void)hipEventRecord(s.ev_force_begin, st);
  if (s.precision == RBE_FP32_MIXED) {
    float* Ff = static_cast<float*>(F);
    if (s.cached) {
      switch (s.fv.nplf) {
        case 1: force_f32_t<1, true, false>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
        case 2: force_f32_t<2, true, false>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
        default: force_f32_t<4, true, false>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
      }
    } else {
      switch (s.fv.nplf) {
        case 1: force_f32_t<1, false, false>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
        case 2: force_f32_t<2, false, false>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
        default: force_f32_t<4, false, false>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
      }
    }
  } else if (s.precision == RBE_FP32) {
    float* Ff = static_cast<float*>(F);
    switch (s.fv.nplf) {
      case 1: force_f32_t<1, false, true>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
      case 2: force_f32_t<2, false, true>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
      default: force_f32_t<4, false, true>(s, w, x, y, z, q, m, wk, rho, Ff, U, counter, st); break;
    }
  } else {
    double* Fd = static_cast<double*>(F);
    switch (s.fv.nplf) {
      case 1: force_f64_t<1>(s, w, x, y, z, q, m, wk, rho, Fd, U, counter, st); break;
      case 2: force_f64_t<2>(s, w, x, y, z, q, m, wk, rho, Fd, U, counter, st); break;
      default: force_f64_t<4>(s, w, x, y, z, q, m, wk, rho, Fd, U, counter, st); break;
    }
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && s.ev_force_end != nullptr) (void)hipEventRecord(s.ev_force_end, st);
  return e;
}

hipError_t launch_vjp(const LaunchShape& s, const WsView& w, const double* x, const double* y,
                      const double* z, const double* q, const int32_t* m, const double* wk,
                      const double* rho, const double* gU, const void* gF, double* gr, double* gq,
                      hipStream_t st) {
  double rc, rs;
  truncation_rotation(s.precision, &rc, &rs);
  if (s.n_rho_items > 0) {
    launch_tile_pass<true>(s, w, x, y, z, q, m, gF, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (s.p_total > 0) {
    hipLaunchKernelGGL(reduce_kernel<false>, dim3((unsigned)s.p_total), dim3(kReduceBlock), 0, st, w, w.xy, rc, rs,
                       nullptr, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (s.n_force_items == 0) return hipSuccess;
  const dim3 grid = grid_for(s.n_force_items, s.force_grid_cap), block(kForceBlock);
  const int32_t ni = s.n_force_items;
  if (s.precision == RBE_FP32_MIXED || s.precision == RBE_FP32) {
    const float* g = static_cast<const float*>(gF);
    double* r = gr;
    double* qq = gq;
    const bool fph = s.precision == RBE_FP32;
    switch (s.fv.nplf * 2 + (fph ? 1 : 0)) {
      case 2: hipLaunchKernelGGL((vjp_b2_f32_kernel<1, false>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs, ni); break;
      case 3: hipLaunchKernelGGL((vjp_b2_f32_kernel<1, true>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs, ni); break;
      case 4: hipLaunchKernelGGL((vjp_b2_f32_kernel<2, false>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs, ni); break;
      case 5: hipLaunchKernelGGL((vjp_b2_f32_kernel<2, true>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs, ni); break;
      case 9: hipLaunchKernelGGL((vjp_b2_f32_kernel<4, true>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs, ni); break;
      default: hipLaunchKernelGGL((vjp_b2_f32_kernel<4, false>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, rc, rs, ni); break;
    }
  } else {
    const double* g = static_cast<const double*>(gF);
    double* r = gr;
    double* qq = gq;
    switch (s.fv.nplf) {
      case 1: hipLaunchKernelGGL((vjp_b2_f64_kernel<1>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, ni); break;
      case 2: hipLaunchKernelGGL((vjp_b2_f64_kernel<2>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, ni); break;
      default: hipLaunchKernelGGL((vjp_b2_f64_kernel<4>), grid, block, 0, st, w, s.n_total, x, y, z, q, m, wk, rho, gU, g, r, qq, ni); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_sample(const LaunchShape& s, const WsView& w, uint64_t seed, uint64_t stream_id,
                         const uint64_t* counter, int32_t* m, double* wk, hipStream_t st) {
  if (s.p_total == 0) return hipSuccess;
  // tables of up to 8192 doubles (64 KB) are staged in LDS, longer ones are read in place
  const int32_t in_lds = s.cdf_stride <= 8192 ? 1 : 0;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)s.B), dim3(kSampleBlock),
                     in_lds ? sizeof(double) * (size_t)s.cdf_stride : 0, st, w, seed, stream_id, counter,
                     s.cdf_stride, in_lds, s.sampler, s.burn_in, m, wk);
  return hipGetLastError();
}

hipError_t launch_virial(const LaunchShape& s, const WsView& w, const int32_t* m, const double* wk,
                         const double* rho, double* W, hipStream_t st) {
  if (s.B == 0) return hipSuccess;
  hipLaunchKernelGGL(virial_kernel, dim3((unsigned)s.B), dim3(kReduceBlock), 0, st, w, m, wk, rho, W);
  return hipGetLastError();
}

}  // namespace rbe
