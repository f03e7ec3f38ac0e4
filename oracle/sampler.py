"""Oracle side of the wave-vector sampler (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU baseline import this
module.  It shares no code with the product library, which implements the
same sampler independently in C++/HIP; the two are compared bit for bit.

What is sampled (paper, Sec. 2.2 and Algorithm 1, step 1): P wave vectors
k = 2 pi m / L, m in Z^3 \\ {0}, with probability proportional to
exp(-k^2 / 4 alpha).  The paper draws them with a Metropolis chain; its
unbiasedness statement assumes independent, identically distributed samples,
so the default sampler of this build draws them exactly and independently
(the Metropolis variant is at the end of this module):

  * exp(-k^2/4 alpha) = prod_d exp(-beta m_d^2) with beta = pi^2 / (alpha L^2),
    so each component is an independent 1-D discrete Gaussian on Z with
    standard deviation sigma = L sqrt(alpha / 2) / pi;
  * each component is drawn by inverse CDF over the window |m_d| <= M,
    M = ceil(9 sigma) + 1 (the mass outside is below 2^-53);
  * a draw with m = (0, 0, 0) is rejected and all three components redrawn.

Uniform numbers come from the counter-based generator Philox4x64-10 (Salmon,
Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11),
implemented here from that definition: key = (seed, stream), counter =
(sample index l, attempt a, 0, 0); output words 0, 1, 2 become the uniforms
u_d = (word_d >> 11) * 2^-53 for the x, y, z components.

Inverse CDF, exactly as both sides evaluate it in FP64: e_j = exp(-beta * j*j)
for j = -M..M, running prefix sums c_j in increasing j, Z = c_M; the
component is the smallest j with u * Z < c_j (j = M if none).

Normalisation Q (the paper's Q for the density exp(-k^2/4 alpha) / Q with
k != 0):  Q = S = (sum_{m in Z} exp(-beta m^2))^3 - 1, and every sampled
wave vector carries the RBE weight S / P (Eq. frbe).
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
# Philox4x64 round multipliers and Weyl key increments (Salmon et al., SC'11).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
MAX_ATTEMPTS = 1024


def philox4x64_10(counter, key):
    """Philox4x64 with 10 rounds on a 4-word counter and 2-word key (Python ints)."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def beta_of(L: float, alpha: float) -> float:
    return (math.pi * math.pi) / (alpha * L * L)


def sigma_of(L: float, alpha: float) -> float:
    return L * math.sqrt(alpha / 2.0) / math.pi


def window_of(L: float, alpha: float) -> int:
    return int(math.ceil(9.0 * sigma_of(L, alpha))) + 1


def component_table(L: float, alpha: float):
    """(M, prefix sums c_j for j = -M..M) in FP64, summed in increasing j."""
    M = window_of(L, alpha)
    beta = beta_of(L, alpha)
    c = []
    acc = 0.0
    for j in range(-M, M + 1):
        acc = acc + math.exp(-beta * float(j * j))
        c.append(acc)
    return M, c


def draw_component(u: float, M: int, c) -> int:
    t = u * c[-1]
    for idx, cj in enumerate(c):
        if t < cj:
            return idx - M
    return M


def normalization_S(L: float, alpha: float) -> float:
    """S = (sum_m exp(-beta m^2))^3 - 1, sum over |m| <= M plus margin, exactly rounded."""
    M = window_of(L, alpha) + 8
    beta = beta_of(L, alpha)
    z = math.fsum(math.exp(-beta * float(j * j)) for j in range(-M, M + 1))
    return z * z * z - 1.0


def sample_k(seed: int, stream: int, L: float, alpha: float, P: int):
    """P wave-vector index triples (P x 3 int32) and S."""
    M, c = component_table(L, alpha)
    out = np.zeros((P, 3), dtype=np.int32)
    for l in range(P):
        for a in range(MAX_ATTEMPTS):
            words = philox4x64_10((l, a, 0, 0), (seed, stream))
            m = [draw_component((words[d] >> 11) * 2.0 ** -53, M, c) for d in range(3)]
            if m != [0, 0, 0]:
                break
        else:
            raise RuntimeError("zero wave vector drawn MAX_ATTEMPTS times")
        out[l] = m
    return out, normalization_S(L, alpha)


def component_pmf(L: float, alpha: float, M: int):
    """Exact pmf of one component on -M..M from the paper's density exp(-k^2/4 alpha), k = 2 pi m / L."""
    j = np.arange(-M, M + 1, dtype=np.float64)
    k = 2.0 * np.pi * j / L
    e = np.exp(-k * k / (4.0 * alpha))
    return j.astype(np.int64), e / e.sum()


def all_vectors(mmax: int) -> np.ndarray:
    """Every m with |m_d| <= mmax except 0, as a (K, 3) int32 array (full Ewald k-space sum)."""
    r = np.arange(-mmax, mmax + 1)
    a, b, c = np.meshgrid(r, r, r, indexing="ij")
    m = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)
    keep = np.any(m != 0, axis=1)
    return m[keep].astype(np.int32)


def ewald_weights(m: np.ndarray, L: float, alpha: float) -> np.ndarray:
    """w_l = exp(-k_l^2 / 4 alpha), the full-Ewald weight of each wave vector (Eq. long)."""
    k = 2.0 * np.pi * m.astype(np.float64) / L
    k2 = np.sum(k * k, axis=1)
    return np.exp(-k2 / (4.0 * alpha))


# ---------------------------------------------------------------- Metropolis sampler
#
# The paper draws the P frequencies with the Metropolis procedure (Sec. 2.2; Algorithm 1,
# step 1) without fixing its proposal, start, burn-in or thinning.  Reading used here:
#   * one chain per wave vector l = 0..P-1, on Z^3 \ {0}, started at m = (1, 0, 0);
#   * proposal m' = m + d, each component d_j uniform on {-D..D}, D = max(1, ceil(1.5 sigma));
#   * target exp(-beta |m|^2) with beta = pi^2 / (alpha L^2) (that is exp(-k^2 / 4 alpha));
#     m' = 0 is rejected; n = |m'|^2 - |m|^2 <= 0 is accepted; otherwise accepted when
#     u < exp(-beta n);
#   * B burn-in steps; the chain's state after step B is the sample (no thinning: the P
#     chains are independent).
# Step t of chain l uses Philox4x64-10 with key (seed, stream) and counter (l, t, 1, 0):
# words 0..2 give the proposal, d_j = min(floor(u_j (2D + 1)), 2D) - D with
# u_j = (word_j >> 11) 2^-53, and word 3 the acceptance uniform.

METROPOLIS_BURN_IN = 64


def metropolis_width(L: float, alpha: float) -> int:
    return max(1, int(math.ceil(1.5 * sigma_of(L, alpha))))


def metropolis_step(m, words, D: int, beta: float):
    """One Metropolis step from m (a 3-list of ints) with the four Philox words of the step."""
    u = [(w >> 11) * 2.0 ** -53 for w in words]
    prop = [m[j] + min(int(math.floor(u[j] * (2 * D + 1))), 2 * D) - D for j in range(3)]
    if prop == [0, 0, 0]:
        return m
    n = sum(v * v for v in prop) - sum(v * v for v in m)
    if n <= 0 or u[3] < math.exp(-beta * float(n)):
        return prop
    return m


def metropolis_k(seed: int, stream: int, L: float, alpha: float, P: int, burn_in: int = METROPOLIS_BURN_IN):
    """P wave-vector index triples (P x 3 int32) from P Metropolis chains, and S."""
    D = metropolis_width(L, alpha)
    beta = beta_of(L, alpha)
    out = np.zeros((P, 3), dtype=np.int32)
    for l in range(P):
        m = [1, 0, 0]
        for t in range(burn_in):
            m = metropolis_step(m, philox4x64_10((l, t, 1, 0), (seed, stream)), D, beta)
        out[l] = m
    return out, normalization_S(L, alpha)
