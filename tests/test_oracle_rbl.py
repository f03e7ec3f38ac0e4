"""Pins for the oracle's random batch list (RBL) short-range force (CPU only).

The oracle follows Sec. 2.3 (Eqs. (short), (fshell), the momentum correction) and
Algorithm 2 with the pair force of Eqs. (lj) and (fshort).  Pins:
  * with a batch at least as large as every shell (the exact truncated force), F = -grad U
    by central finite differences of the separately written truncated short-range energy;
  * closed forms: the LJ force vanishes at r = 2^(1/6) sigma and is 24 eps / sigma at
    r = sigma; at alpha -> 0 the real-space Coulomb term is Coulomb's law q_i q_j / r^2;
  * total momentum: sum_i F_i = 0 after the correction, for any batch;
  * unbiasedness: the mean over many batch draws equals the exact truncated force (z-test);
  * the systematic batch includes every shell particle with probability p / N_s: over a
    fine grid of offsets u each member is picked the same number of times.
"""
import math

import numpy as np
import pytest

import oracle
import rbe_inputs as ri


def _two(d, qi=0.0, qj=0.0, eps=1.0, sig=1.0):
    x = np.array([0.0, d]) + 5.0
    y = np.array([5.0, 5.0])
    z = np.array([5.0, 5.0])
    return x, y, z, np.array([qi, qj]), np.array([eps, eps]), np.array([sig, sig])


def _exact(s, alpha, rc, rs):
    big = s.n   # the batch covers every shell
    return oracle.rbl_short_force(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, alpha, rc, rs, big, np.zeros(s.n))


def test_lj_closed_forms():
    L = 40.0
    x, y, z, q, e, sg = _two(2.0 ** (1.0 / 6.0))
    F, _ = oracle.rbl_short_force(x, y, z, q, e, sg, L, 0.0, 3.0, 6.0, 4, np.zeros(2))
    assert np.max(np.abs(F)) < 1e-12
    x, y, z, q, e, sg = _two(1.0, eps=0.7, sig=1.0)
    F, _ = oracle.rbl_short_force(x, y, z, q, e, sg, L, 0.0, 3.0, 6.0, 4, np.zeros(2))
    # particle 0 sits at the lower x: pushed towards -x with 24 eps / sigma
    assert abs(F[0, 0] + 24.0 * 0.7) < 1e-12 and abs(F[0, 1] - 24.0 * 0.7) < 1e-12
    # Lorentz-Berthelot: sigma_ij = (1 + 2)/2, eps_ij = sqrt(0.5 * 2): zero force at
    # 2^(1/6) sigma_ij, 24 eps_ij / sigma_ij at sigma_ij
    for d, f0 in ((2.0 ** (1.0 / 6.0) * 1.5, 0.0), (1.5, -24.0 * 1.0 / 1.5)):
        x, y, z, q, e, sg = _two(d)
        e, sg = np.array([0.5, 2.0]), np.array([1.0, 2.0])
        F, _ = oracle.rbl_short_force(x, y, z, q, e, sg, L, 0.0, 3.0, 6.0, 4, np.zeros(2))
        assert abs(F[0, 0] - f0) < 1e-12 and abs(F[0, 0] + F[0, 1]) < 1e-12


def test_coulomb_limit():
    """alpha -> 0: erfc -> 1 and the Gaussian term vanishes, leaving q_i q_j / r^2."""
    L = 40.0
    for d, qi, qj in [(2.5, 1.0, -1.0), (4.0, 0.5, 2.0)]:
        x, y, z, q, e, sg = _two(d, qi, qj, eps=0.0)
        F, _ = oracle.rbl_short_force(x, y, z, q, e, sg, L, 1e-14, 3.0, 6.0, 4, np.zeros(2))
        assert abs(F[0, 0] - (-qi * qj / d ** 2)) < 1e-6 * abs(qi * qj / d ** 2)
        assert np.max(np.abs(F[1:, :])) == 0.0


@pytest.mark.parametrize("alpha", [0.06, 0.3])
def test_force_is_minus_gradient_of_energy(alpha):
    s = ri.primitive_electrolyte(300, 0.01, 21)
    g0 = np.random.default_rng(5)      # unequal LJ parameters, so the mixing rules matter
    s.eps = g0.uniform(0.5, 1.5, s.n)
    s.sig = g0.uniform(0.8, 1.6, s.n)
    rc, rs = 6.0, 12.0
    F, ns = _exact(s, alpha, rc, rs)
    g = np.random.default_rng(3)
    h = 1e-5
    for _ in range(8):
        i, d = int(g.integers(s.n)), int(g.integers(3))
        coords = [s.x.copy(), s.y.copy(), s.z.copy()]
        coords[d][i] += h
        up = oracle.short_energy(*coords, s.q, s.eps, s.sig, s.L, alpha, rs)
        coords[d][i] -= 2 * h
        dn = oracle.short_energy(*coords, s.q, s.eps, s.sig, s.L, alpha, rs)
        fd = -(up - dn) / (2 * h)
        assert abs(F[d, i] - fd) < 1e-6 * max(abs(fd), np.sqrt(np.mean(F ** 2))), (i, d, F[d, i], fd)


@pytest.mark.parametrize("p", [1, 7, 30])
def test_momentum_conserved(p):
    s = ri.primitive_electrolyte(500, 0.01, 22)
    F, ns = oracle.rbl_short_force(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, 0.06, 6.0, 12.0, p,
                                   oracle.rbl_offsets(4, 1, s.n))
    assert np.all(np.abs(F.sum(axis=1)) < 1e-12 * np.abs(F).sum(axis=1))
    assert ns.min() > p   # the batch is a proper subset here


def test_unbiased_against_exact_truncated_force():
    s = ri.primitive_electrolyte(200, 0.01, 23)
    alpha, rc, rs, p = 0.06, 6.0, 12.0, 5
    F_ex, ns = _exact(s, alpha, rc, rs)
    B = 400
    g = np.random.default_rng(9)
    acc = np.zeros((B, 3, s.n))
    for b in range(B):
        acc[b], _ = oracle.rbl_short_force(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, alpha, rc, rs, p,
                                           g.uniform(0.0, 1.0, s.n))
    mean, sd = acc.mean(axis=0), acc.std(axis=0, ddof=1) / math.sqrt(B)
    z = (mean - F_ex) / sd
    rms = math.sqrt(np.mean(z * z))
    assert 0.85 < rms < 1.15 and np.abs(z).max() < 6, (rms, np.abs(z).max())
    # a batch does differ from the exact force
    assert np.sqrt(np.mean((acc[0] - F_ex) ** 2)) > 1e-3 * np.sqrt(np.mean(F_ex ** 2))


def test_systematic_batch_inclusion():
    """Over a grid of K offsets each shell member is picked K p / N_s times (to one), seen
    through the force: the mean over the grid equals the exact truncated force."""
    s = ri.primitive_electrolyte(200, 0.01, 24)
    alpha, rc, rs, p = 0.06, 6.0, 12.0, 6
    F_ex, ns = _exact(s, alpha, rc, rs)
    K = 997   # prime, so no member lines up with the grid
    tot = np.zeros((3, s.n))
    for k in range(K):
        F, _ = oracle.rbl_short_force(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, alpha, rc, rs, p,
                                      np.full(s.n, (k + 0.5) / K))
        tot += F
    mean = tot / K
    # each member is picked floor or ceil of K p / N_s times: the error is at most
    # ~ N_s / (K p) of one pair force per member
    err = np.sqrt(np.mean((mean - F_ex) ** 2)) / np.sqrt(np.mean(F_ex ** 2))
    assert err < 0.02, err


def test_argument_checks():
    s = ri.primitive_electrolyte(50, 0.01, 25)
    with pytest.raises(ValueError):
        oracle.rbl_short_force(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, 0.06, 6.0, 0.6 * s.L, 5, np.zeros(s.n))
    with pytest.raises(ValueError):
        oracle.rbl_short_force(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, 0.06, 6.0, 5.0, 5, np.zeros(s.n))
