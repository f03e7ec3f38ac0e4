// The Metropolis wave-vector sampler (paper Sec. 2.2; Algorithm 1, step 1), on the host and
// on gfx950.  The paper names the procedure but fixes no proposal, start or burn-in; the
// chain implemented here:
//   target   pi(m) ~ exp(-beta |m|^2) on Z^3 \ {0}, beta = pi^2 / (alpha L^2)
//            (= exp(-k^2 / 4 alpha) with k = 2 pi m / L);
//   start    m = (1, 0, 0);
//   proposal m' = m + d, d_j = min(floor(u_j (2D + 1)), 2D) - D, i.e. uniform on {-D..D}
//            per component, D = max(1, ceil(1.5 sigma)), sigma = L sqrt(alpha / 2) / pi;
//   accept   m' != 0 and (n = |m'|^2 - |m|^2 <= 0 or u_3 < exp(-beta n));
//   output   the state after `burn_in` steps; chain l gives wave vector l.
// Step t of chain l draws Philox4x64-10 with key (k0, k1) and counter (l, t, 1, 0); words
// 0..2 give u_0..u_2 and word 3 gives u_3 (top 53 bits each).
#pragma once

#include <cmath>
#include <cstdint>
#include <hip/hip_runtime.h>

#include "philox.h"

namespace rbe {

// Proposal half-width D of the chain for a box L and splitting alpha.
__host__ __device__ inline int32_t metropolis_width(double L, double alpha) {
  const double sigma = L * sqrt(alpha / 2.0) / M_PI;
  const double d = ceil(1.5 * sigma);
  return d < 1.0 ? 1 : (int32_t)d;
}

__host__ __device__ inline void metropolis_chain(uint64_t k0, uint64_t k1, uint64_t l, int32_t burn_in,
                                                 int32_t D, double beta, int32_t (&m)[3]) {
  m[0] = 1; m[1] = 0; m[2] = 0;
  const double span = 2.0 * (double)D + 1.0;
  for (int32_t t = 0; t < burn_in; ++t) {
    U64x4 ctr = {{l, (uint64_t)t, 1ull, 0ull}};
    const U64x4 r = philox4x64_10(ctr, k0, k1);
    int32_t p[3];
    for (int j = 0; j < 3; ++j) {
      int32_t i = (int32_t)floor(u01_53(r.v[j]) * span);
      i = i < 2 * D ? i : 2 * D;
      p[j] = m[j] + i - D;
    }
    if (p[0] == 0 && p[1] == 0 && p[2] == 0) continue;
    const int64_t n = ((int64_t)p[0] * p[0] + (int64_t)p[1] * p[1] + (int64_t)p[2] * p[2]) -
                      ((int64_t)m[0] * m[0] + (int64_t)m[1] * m[1] + (int64_t)m[2] * m[2]);
    if (n <= 0 || u01_53(r.v[3]) < exp(-beta * (double)n)) {
      m[0] = p[0]; m[1] = p[1]; m[2] = p[2];
    }
  }
}

}  // namespace rbe
