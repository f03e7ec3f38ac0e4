// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), usable on the host and on gfx950.
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace rbe {

struct U64x4 { uint64_t v[4]; };

__host__ __device__ inline void mul_hilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  *lo = a * b;
  *hi = __umul64hi(a, b);
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  *lo = (uint64_t)p;
  *hi = (uint64_t)(p >> 64);
#endif
}

// Ten rounds; the key advances by the Weyl increments before rounds 2..10.
__host__ __device__ inline U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mul_hilo64(M0, c.v[0], &hi0, &lo0);
    mul_hilo64(M1, c.v[2], &hi1, &lo1);
    U64x4 o;
    o.v[0] = hi1 ^ c.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ c.v[3] ^ k1;
    o.v[3] = lo0;
    c = o;
  }
  return c;
}

// Uniform in [0, 1) from the top 53 bits of a word.
__host__ __device__ inline double u01_53(uint64_t w) {
  return (double)(w >> 11) * 1.1102230246251565404236316680908203125e-16;  // 2^-53
}

// Smallest j in [-M, M] with t < c[j + M]; M if none (c: 2M+1 prefix sums, non-decreasing).
__host__ __device__ inline int32_t inverse_cdf(const double* c, int32_t M, double t) {
  int32_t lo = 0, hi = 2 * M;   // answer index in [0, 2M]
  if (!(t < c[hi])) return M;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (t < c[mid]) hi = mid; else lo = mid + 1;
  }
  return lo - M;
}

}  // namespace rbe
