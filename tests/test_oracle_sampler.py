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


# ---------------------------------------------------------------- Metropolis variant
#
# The paper samples with the Metropolis procedure (Sec. 2.2; Algorithm 1, step 1) but
# fixes no proposal, start or burn-in; the oracle's chain follows the reading written in
# oracle/sampler.py.  Pins:
#   * one step from fixed states: the distribution of the next state over many Philox
#     counters against the transition probabilities of a symmetric uniform proposal with
#     acceptance min(1, pi(m') / pi(m)), pi evaluated from the density in k;
#   * the kernel those probabilities define leaves pi invariant (detailed balance, checked
#     numerically on every pair of states of a box);
#   * after the burn-in, the chains' outputs against the exact pmf of |m|^2 (chi-square).


def _pi_k(m, L, alpha):
    k = 2.0 * np.pi * np.asarray(m, dtype=np.float64) / L
    return np.exp(-np.sum(k * k, axis=-1) / (4.0 * alpha))


def _one_step_probs(m0, L, alpha, D):
    """Exact next-state probabilities of one step from m0: {state tuple: probability}."""
    m0 = np.asarray(m0)
    r = np.arange(-D, D + 1)
    d = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    prop = m0 + d
    p_prop = 1.0 / len(d)
    ratio = _pi_k(prop, L, alpha) / _pi_k(m0, L, alpha)
    acc = np.where(np.all(prop == 0, axis=1), 0.0, np.minimum(1.0, ratio))
    out = {}
    for mp, a in zip(map(tuple, prop), acc):
        if a > 0:
            out[mp] = out.get(mp, 0.0) + p_prop * a
    out[tuple(m0)] = out.get(tuple(m0), 0.0) + p_prop * float(np.sum(1.0 - acc))
    return out


@pytest.mark.parametrize("m0", [(1, 0, 0), (3, -2, 1), (0, 0, -1)])
def test_metropolis_one_step_distribution(m0):
    L, alpha = 31.0, 0.1
    D = sampler.metropolis_width(L, alpha)
    beta = sampler.beta_of(L, alpha)
    n = 60000
    counts = {}
    for l in range(n):
        nxt = tuple(sampler.metropolis_step(list(m0), sampler.philox4x64_10((l, 0, 1, 0), (9, 4)), D, beta))
        counts[nxt] = counts.get(nxt, 0) + 1
    probs = _one_step_probs(m0, L, alpha, D)
    assert set(counts) <= set(probs)          # never a state the kernel cannot reach (nor 0)
    keys = sorted(probs, key=lambda s: -probs[s])
    exp = np.array([probs[s] * n for s in keys])
    obs = np.array([counts.get(s, 0) for s in keys], dtype=np.float64)
    big = exp >= 5
    e = np.append(exp[big], exp[~big].sum())
    o = np.append(obs[big], obs[~big].sum())
    chi2 = float(np.sum((o - e) ** 2 / e))
    assert stats.chi2.sf(chi2, len(e) - 1) > 1e-4, chi2


def test_metropolis_detailed_balance():
    """pi(m) T(m -> m') = pi(m') T(m' -> m) for every pair of states in a box (so pi is
    stationary), with T the one-step probabilities the first pin checks the chain against."""
    L, alpha = 31.0, 0.1
    D = sampler.metropolis_width(L, alpha)
    r = range(-3, 4)
    states = [(a, b, c) for a in r for b in r for c in r if (a, b, c) != (0, 0, 0)]
    T = {s: _one_step_probs(s, L, alpha, D) for s in states}
    for s in states:
        for t, p in T[s].items():
            if t in T and t != s:
                lhs = _pi_k(s, L, alpha) * p
                rhs = _pi_k(t, L, alpha) * T[t].get(s, 0.0)
                assert abs(lhs - rhs) <= 1e-15 * max(lhs, rhs, 1e-300), (s, t)
        assert abs(sum(T[s].values()) - 1.0) < 1e-12


@pytest.mark.parametrize("L,alpha", [(31.0, 0.1), (66.9, 0.048)])
def test_metropolis_output_chi_square(L, alpha):
    """After the default burn-in the chains' states follow pi: |m|^2 against its exact pmf."""
    P = 2500
    samples = np.concatenate([sampler.metropolis_k(101 + s, s, L, alpha, P)[0] for s in range(2)])
    assert not np.any(np.all(samples == 0, axis=1))
    M = sampler.window_of(L, alpha)
    r = np.arange(-M, M + 1)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    g = g[np.any(g != 0, axis=1)]
    pk = _pi_k(g, L, alpha)
    s2 = np.sum(g * g, axis=1)
    # |m|^2 in bins of about equal probability
    order = np.argsort(s2)
    cum = np.cumsum(pk[order]) / pk.sum()
    edges = [0]
    for q in np.linspace(0.05, 0.95, 19):
        edges.append(int(s2[order][np.searchsorted(cum, q)]))
    edges = sorted(set(edges)) + [int(s2.max()) + 1]
    exp = np.array([pk[(s2 >= a) & (s2 < b)].sum() for a, b in zip(edges[:-1], edges[1:])]) / pk.sum()
    ss = np.sum(samples.astype(np.int64) ** 2, axis=1)
    obs = np.array([np.sum((ss >= a) & (ss < b)) for a, b in zip(edges[:-1], edges[1:])], dtype=np.float64)
    e = exp * len(ss)
    chi2 = float(np.sum((obs - e) ** 2 / e))
    assert stats.chi2.sf(chi2, len(e) - 1) > 1e-4, (chi2, len(e))


def test_metropolis_start_and_determinism():
    m, S = sampler.metropolis_k(5, 1, 31.0, 0.1, 7, burn_in=0)
    assert np.all(m == np.array([1, 0, 0]))
    a, _ = sampler.metropolis_k(5, 1, 31.0, 0.1, 20)
    b, _ = sampler.metropolis_k(5, 1, 31.0, 0.1, 20)
    c, _ = sampler.metropolis_k(5, 2, 31.0, 0.1, 20)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert abs(S / sampler.normalization_S(31.0, 0.1) - 1) == 0
