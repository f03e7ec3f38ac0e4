"""Pins for the oracle's k-space virial tensor (CPU only).

The virial is the negative derivative of the long-range energy term under a
symmetric affine strain of the box, at fixed fractional coordinates (the
quantity an NPT variant needs; the paper cites NPT random batch Ewald in
Sec. 2.2).  Each test checks the oracle's closed form against something else:
  * central finite differences of a separate box-matrix energy (a general,
    non-cubic strain, written here with numpy) for all six components;
  * isotropic scaling of the cubic box through the oracle's own energy path:
    -dU/d(ln L) equals the trace;
  * the RBE estimate averaged over independent batches converges to the full
    Ewald k-space virial (unbiasedness of the importance-sampled estimator).
"""
import math

import numpy as np
import pytest

import rbe_inputs as ri
from oracle import sampler

COMP = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def box_energy(h, s_frac, q, mlist, alpha):
    """Ewald k-space energy sum_m (2 pi / V) exp(-k^2/4 alpha) / k^2 |rho(k)|^2 for box
    matrix h (columns = box edges), k = 2 pi h^-T m, positions r = h s."""
    V = abs(np.linalg.det(h))
    G = 2 * np.pi * np.linalg.inv(h).T
    k = mlist.astype(np.float64) @ G.T
    r = s_frac @ h.T
    rho = np.exp(1j * (r @ k.T)).T @ q
    k2 = np.sum(k * k, axis=1)
    return float(np.sum(2 * np.pi / V * np.exp(-k2 / (4 * alpha)) / k2 * np.abs(rho) ** 2))


def test_virial_equals_strain_derivative(oracle_lib):
    rng = np.random.default_rng(11)
    n, L, alpha = 12, 6.0, 0.8
    s_frac = rng.random((n, 3))
    q = rng.choice([-1.0, 1.0], n)
    q -= q.mean()
    m = sampler.all_vectors(6)
    w = sampler.ewald_weights(m, L, alpha)
    x, y, z = (s_frac * L).T
    rho = oracle_lib.rho(x, y, z, q, m, L)
    W = oracle_lib.virial(m, w, L, alpha, rho)
    h0 = L * np.eye(3)
    # the cubic box energy of the test function equals the oracle's energy
    k2 = np.sum((2 * np.pi * m / L) ** 2, axis=1)
    U_oracle = float(np.sum(2 * np.pi / L ** 3 * w / k2 * np.abs(rho) ** 2))
    assert abs(box_energy(h0, s_frac, q, m, alpha) / U_oracle - 1) < 1e-12
    d = 1e-5
    for c, (a, b) in enumerate(COMP):
        e = np.zeros((3, 3))
        e[a, b] = e[b, a] = d
        up = box_energy((np.eye(3) + e) @ h0, s_frac, q, m, alpha)
        um = box_energy((np.eye(3) - e) @ h0, s_frac, q, m, alpha)
        fd = -(up - um) / (2 * d)
        expect = W[c] if a == b else 2 * W[c]
        assert abs(fd - expect) < 1e-7 * np.max(np.abs(W)), (c, fd, expect)


def test_virial_trace_is_isotropic_scaling_derivative(oracle_lib):
    """tr W = -dU/d ln L for the cubic box through the oracle's own energy (RBE weights)."""
    s, alpha, P = ri.c1_small()
    m, S = sampler.sample_k(31, 0, s.L, alpha, P)

    def energy(L, weights):
        f = L / s.L
        _, U, _ = oracle_lib.force_energy(s.x * f, s.y * f, s.z * f, s.q, m, weights, L)
        return U

    # the RBE estimate of the Ewald virial differentiates the Ewald kernel too, so the
    # weights follow exp(-k^2 / 4 alpha) under the scaling: w(L) = S/P * g(k(L)) / g(k(L0))
    def weights(L):
        k2 = np.sum((2 * np.pi * m / L) ** 2, axis=1)
        k20 = np.sum((2 * np.pi * m / s.L) ** 2, axis=1)
        return S / P * np.exp(-(k2 - k20) / (4 * alpha))

    rho = oracle_lib.rho(s.x, s.y, s.z, s.q, m, s.L)
    W = oracle_lib.virial(m, np.full(P, S / P), s.L, alpha, rho)
    d = 1e-6
    fd = -(energy(s.L * (1 + d), weights(s.L * (1 + d))) - energy(s.L * (1 - d), weights(s.L * (1 - d)))) / (2 * d)
    assert abs(fd - (W[0] + W[1] + W[2])) < 1e-7 * np.max(np.abs(W))


@pytest.mark.slow
def test_rbe_virial_mean_converges_to_ewald(oracle_lib):
    s, alpha, P = ri.c1_small()
    mref = sampler.all_vectors(10)
    wref = sampler.ewald_weights(mref, s.L, alpha)
    Wref = oracle_lib.virial(mref, wref, s.L, alpha, oracle_lib.rho(s.x, s.y, s.z, s.q, mref, s.L))
    B = 200
    Ws = np.zeros((B, 6))
    for b in range(B):
        m, S = sampler.sample_k(7001 + b, 0, s.L, alpha, P)
        Ws[b] = oracle_lib.virial(m, np.full(P, S / P), s.L, alpha, oracle_lib.rho(s.x, s.y, s.z, s.q, m, s.L))
    z = (Ws.mean(axis=0) - Wref) / (Ws.std(axis=0, ddof=1) / math.sqrt(B))
    assert np.max(np.abs(z)) < 4.5, z
