"""Pins for the oracle's wave-vector sampler and normalisation (CPU only).

The sampler follows the paper's importance density exp(-k^2/4 alpha)/Q with
k != 0 (Sec. 2.2, Algorithm 1 step 1), drawn exactly and i.i.d.  Pins:
  * Philox4x64-10 against numpy's independent Philox bit generator;
  * chi-square of sampled components against the exact pmf evaluated from
    the paper's density in k (not the simplified exponent the sampler uses);
  * the zero wave vector is never drawn; determinism per (seed, stream);
  * S against the Poisson-summation (Jacobi theta) closed form.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import sampler


@pytest.mark.parametrize("key,ctr", [((5, 7), (0, 0, 0, 0)), ((2**64 - 1, 12345), (3, 9, 1, 2**63)),
                                     ((0, 0), (2**64 - 2, 0, 0, 0))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox increments the 256-bit counter before producing each block.
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = bg.random_raw(8)
    c = list(ctr)
    for blk in range(2):
        carry = 1
        for w in range(4):
            s = c[w] + carry
            c[w] = s & sampler.MASK64
            carry = s >> 64
        out = sampler.philox4x64_10(tuple(c), key)
        assert [int(v) for v in raw[4 * blk:4 * blk + 4]] == list(out)


def _conditional_marginal(L, alpha, M):
    """pmf of one component given m != 0, from the paper's density in k."""
    j, p = sampler.component_pmf(L, alpha, M)
    p0 = p[j == 0][0]
    cond = p.copy()
    cond[j == 0] *= (1.0 - p0 * p0) / 1.0
    cond = cond / (1.0 - p0 ** 3)
    return j, cond


@pytest.mark.parametrize("L,alpha", [(31.0, 0.1), (10.0, 0.362), (66.9, 0.048)])
def test_components_chi_square(L, alpha):
    P = 6000
    m, _ = sampler.sample_k(77, 3, L, alpha, P)
    M = sampler.window_of(L, alpha)
    j, cond = _conditional_marginal(L, alpha, M)
    for d in range(3):
        counts = np.array([np.sum(m[:, d] == v) for v in j], dtype=np.float64)
        expected = cond * P
        # pool the tails so that every bin expects at least 5 draws
        keep = expected >= 5
        obs = np.concatenate([counts[keep], [counts[~keep].sum()]])
        exp = np.concatenate([expected[keep], [expected[~keep].sum()]])
        if exp[-1] == 0:
            obs, exp = obs[:-1], exp[:-1]
        chi2 = np.sum((obs - exp) ** 2 / exp)
        pval = stats.chi2.sf(chi2, len(obs) - 1)
        assert pval > 1e-4, (d, chi2, pval)
        # second moment against the exact conditional pmf
        mean_sq = np.mean(m[:, d].astype(np.float64) ** 2)
        exact = np.sum(cond * j.astype(np.float64) ** 2)
        sd = math.sqrt((np.sum(cond * j.astype(np.float64) ** 4) - exact ** 2) / P)
        assert abs(mean_sq - exact) < 5 * sd


def test_never_zero_and_deterministic():
    # tiny box: P(m_d = 0) is large, so rejection is exercised often
    L, alpha = 2.0, 1.5
    m1, S1 = sampler.sample_k(11, 0, L, alpha, 500)
    m2, S2 = sampler.sample_k(11, 0, L, alpha, 500)
    m3, _ = sampler.sample_k(11, 1, L, alpha, 500)
    assert not np.any(np.all(m1 == 0, axis=1))
    assert np.array_equal(m1, m2) and S1 == S2
    assert not np.array_equal(m1, m3)


def _S_poisson(L, alpha):
    # sum_m exp(-pi^2 m^2/(alpha L^2)) = L sqrt(alpha/pi) sum_n exp(-alpha L^2 n^2)
    theta = math.fsum(math.exp(-alpha * L * L * n * n) for n in range(-20, 21))
    z = L * math.sqrt(alpha / math.pi) * theta
    return z ** 3 - 1.0


@pytest.mark.parametrize("L,alpha", [(31.0, 0.1), (144.1289, 0.08), (217.0535, 0.06), (467.6275, 0.06),
                                     (126.0, 0.08), (2.0, 1.5), (10.0, 0.362), (66.9, 0.048)])
def test_S_poisson_closed_form(L, alpha):
    assert abs(sampler.normalization_S(L, alpha) / _S_poisson(L, alpha) - 1.0) < 1e-14


def test_S_values_for_benchmark_boxes():
    # S = L^3 (alpha/pi)^(3/2) - 1 whenever alpha L^2 is large (all benchmark boxes)
    for L, alpha in [(31.0, 0.1), (217.0535, 0.06), (126.0, 0.08)]:
        ref = L ** 3 * (alpha / math.pi) ** 1.5 - 1.0
        assert abs(sampler.normalization_S(L, alpha) - ref) / ref < 1e-13
    assert abs(sampler.normalization_S(31.0, 0.1) - 168.18438322540) < 1e-9


def test_window_mass_below_double_resolution():
    for L, alpha in [(31.0, 0.1), (467.6275, 0.06), (2.0, 1.5)]:
        M = sampler.window_of(L, alpha)
        beta = sampler.beta_of(L, alpha)
        tail = 2 * sum(math.exp(-beta * j * j) for j in range(M + 1, M + 400))
        total = sum(math.exp(-beta * j * j) for j in range(-M - 400, M + 400))
        assert tail / total < 2.0 ** -53
