"""Pins for the oracle's structure factor, force and energy (CPU only).

Each test checks the oracle against something other than itself:
  * rho on gridded charges equals a numpy FFT (library routine);
  * rho for N <= 8 equals a 50-digit mpmath sum (brute force);
  * rho(-k) = conj(rho(k)); translation multiplies rho by exp(i k.c);
    periodic images leave it unchanged;
  * sum_i F_i = 0 for any wave-vector list; F = -grad U by finite differences;
  * a two-charge system against its closed form;
  * a perfect rock-salt lattice has zero RBE force for any wave-vector list;
  * the full Ewald sum (real + k-space + self) reproduces the rock-salt
    Madelung constant (textbook value, tests/golden/madelung_nacl.txt);
  * the RBE estimator averaged over many independent batches converges to
    the full Ewald k-space force and energy (unbiasedness, paper Sec. 2.2).
"""
import math
import os

import mpmath
import numpy as np
import pytest

import rbe_inputs as ri
from oracle import sampler

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name, key):
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            if line.startswith(key + " "):
                return float(line.split()[1])
    raise KeyError(key)


def test_rho_equals_fft_of_gridded_charges(oracle_lib):
    n, L = 8, 13.0
    g = np.random.default_rng(1)
    grid = g.standard_normal((n, n, n))
    idx = np.argwhere(np.ones((n, n, n), dtype=bool))
    q = grid[idx[:, 0], idx[:, 1], idx[:, 2]]
    pos = idx.astype(np.float64) * (L / n)
    m = g.integers(-20, 21, size=(64, 3)).astype(np.int32)
    m[np.all(m == 0, axis=1)] = [1, 0, 0]
    got = oracle_lib.rho(pos[:, 0], pos[:, 1], pos[:, 2], q, m, L)
    # rho(m) = sum_g q_g exp(+2 pi i m.g / n) = n^3 * ifftn(grid)[m mod n]
    ref_all = np.fft.ifftn(grid) * n ** 3
    ref = ref_all[m[:, 0] % n, m[:, 1] % n, m[:, 2] % n]
    assert np.max(np.abs(got - ref)) < 1e-11 * math.sqrt(np.sum(q * q))


def test_rho_brute_force_mpmath(oracle_lib):
    mpmath.mp.dps = 50
    s = ri.random_charges(7, 9.5, 3)
    m = np.array([[1, 0, 0], [0, -2, 3], [5, 4, -7], [-11, 2, 1]], dtype=np.int32)
    got = oracle_lib.rho(s.x, s.y, s.z, s.q, m, s.L)
    for l in range(m.shape[0]):
        acc = mpmath.mpc(0)
        for i in range(s.n):
            th = 2 * mpmath.pi * (int(m[l, 0]) * mpmath.mpf(s.x[i]) + int(m[l, 1]) * mpmath.mpf(s.y[i])
                                  + int(m[l, 2]) * mpmath.mpf(s.z[i])) / mpmath.mpf(s.L)
            acc += mpmath.mpf(s.q[i]) * mpmath.expjpi(2 * th / (2 * mpmath.pi))
        assert abs(complex(acc) - got[l]) < 1e-13


def test_rho_symmetries(oracle_lib):
    s = ri.uniform_pm1(500, 20.0, 5)
    g = np.random.default_rng(2)
    m = g.integers(-9, 10, size=(40, 3)).astype(np.int32)
    m[np.all(m == 0, axis=1)] = [0, 0, 1]
    r = oracle_lib.rho(s.x, s.y, s.z, s.q, m, s.L)
    rneg = oracle_lib.rho(s.x, s.y, s.z, s.q, -m, s.L)
    assert np.array_equal(rneg, np.conj(r))
    c = np.array([0.37, -1.21, 2.5])
    rt = oracle_lib.rho(s.x + c[0], s.y + c[1], s.z + c[2], s.q, m, s.L)
    k = 2 * np.pi * m / s.L
    assert np.max(np.abs(rt - np.exp(1j * (k @ c)) * r)) < 1e-11
    shift = np.zeros(s.n)
    shift[::3] = s.L
    rp = oracle_lib.rho(s.x + shift, s.y - shift, s.z, s.q, m, s.L)
    assert np.max(np.abs(rp - r)) < 1e-11


def test_force_sum_is_zero(oracle_lib):
    s, alpha, P = ri.c1_small()
    m, S = sampler.sample_k(2001, 0, s.L, alpha, P)
    F, U, _ = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, np.full(P, S / P), s.L)
    scale = np.sqrt(np.mean(F * F))
    assert np.max(np.abs(F.sum(axis=1))) < 1e-12 * scale * s.n
    assert U > 0


def test_force_is_minus_gradient_of_energy(oracle_lib):
    s = ri.random_charges(30, 8.0, 9)
    m, S = sampler.sample_k(5, 0, s.L, 0.4, 24)
    w = np.full(24, S / 24)
    F, U, _ = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    h = 1e-5
    pos = [s.x.copy(), s.y.copy(), s.z.copy()]
    for i in [0, 7, 29]:
        for d in range(3):
            pp = [a.copy() for a in pos]
            pm = [a.copy() for a in pos]
            pp[d][i] += h
            pm[d][i] -= h
            _, Up, _ = oracle_lib.force_energy(*pp, s.q, m, w, s.L)
            _, Um, _ = oracle_lib.force_energy(*pm, s.q, m, w, s.L)
            fd = -(Up - Um) / (2 * h)
            assert abs(fd - F[d, i]) < 1e-7 * max(1.0, abs(F[d, i]))


def test_two_charge_closed_form(oracle_lib):
    L, d = 7.0, 1.3
    x = np.array([0.0, d])
    zero = np.zeros(2)
    q = np.array([1.0, -1.0])
    m = np.array([[1, 0, 0]], dtype=np.int32)
    F, U, r = oracle_lib.force_energy(x, zero, zero, q, m, np.ones(1), L)
    k = 2 * np.pi / L
    c = 4 * np.pi / (L ** 3 * k * k)
    assert abs(U - c * (1 - math.cos(k * d))) < 1e-15
    assert abs(F[0, 0] - c * k * math.sin(k * d)) < 1e-15
    assert abs(F[0, 1] + c * k * math.sin(k * d)) < 1e-15
    assert np.all(F[1:] == 0)
    assert abs(r[0] - (1 - np.exp(1j * k * d))) < 1e-15


def test_rock_salt_lattice_has_zero_rbe_force(oracle_lib):
    s = ri.nacl_lattice(2)
    m, S = sampler.sample_k(8, 0, s.L, 1.0, 50)
    F, _, _ = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, np.full(50, S / 50), s.L)
    assert np.max(np.abs(F)) < 1e-11


def _ewald_total(oracle_lib, s, alpha, mmax, nmax):
    m = sampler.all_vectors(mmax)
    w = sampler.ewald_weights(m, s.L, alpha)
    _, Uk, _ = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, w, s.L) if m.shape[0] <= 256 else (None, None, None)
    if Uk is None:
        rho = oracle_lib.rho(s.x, s.y, s.z, s.q, m, s.L)
        k2 = np.sum((2 * np.pi * m / s.L) ** 2, axis=1)
        Uk = float(np.sum(2 * np.pi / s.L ** 3 * w / k2 * np.abs(rho) ** 2))
        # same quantity through the oracle's force/energy path (U = sum c/2 |rho|^2)
        F = np.zeros(3 * s.n)
        U = np.zeros(1)
        import ctypes
        lib = oracle_lib._load()
        rr = np.empty(2 * m.shape[0])
        rr[0::2], rr[1::2] = rho.real, rho.imag
        args = [np.ascontiguousarray(a, dtype=np.float64) for a in (s.x, s.y, s.z, s.q, w)]
        mm = np.ascontiguousarray(m)
        P = ctypes.c_void_p
        lib.oracle_force_from_rho(s.n, *[a.ctypes.data_as(P) for a in args[:4]], m.shape[0],
                                  mm.ctypes.data_as(P), args[4].ctypes.data_as(P), float(s.L),
                                  rr.ctypes.data_as(P), F.ctypes.data_as(P), U.ctypes.data_as(P))
        assert abs(U[0] - Uk) < 1e-12 * abs(Uk)
        Uk = float(U[0])
    Ur, Us = oracle_lib.ewald_real_self(s.x, s.y, s.z, s.q, s.L, alpha, nmax)
    return Ur + Uk + Us


@pytest.mark.parametrize("alpha", [1.5, 2.5, 4.0])
def test_madelung_constant_rock_salt(oracle_lib, alpha):
    M = _golden("madelung_nacl.txt", "M")
    s = ri.nacl_lattice(1)          # 8 ions, r0 = 1, L = 2
    U = _ewald_total(oracle_lib, s, alpha, mmax=12, nmax=4)
    assert abs(U / (-4.0 * M) - 1.0) < 1e-11


def test_madelung_supercell_energy_per_ion(oracle_lib):
    M = _golden("madelung_nacl.txt", "M")
    s = ri.nacl_lattice(2)          # 64 ions, L = 4
    U = _ewald_total(oracle_lib, s, 1.0, mmax=12, nmax=3)
    assert abs(U / (-(s.n / 2) * M) - 1.0) < 1e-10


@pytest.mark.slow
def test_rbe_mean_converges_to_full_ewald(oracle_lib):
    """Unbiasedness (Sec. 2.2): mean over B independent batches vs the full k-space sum."""
    s, alpha, P = ri.c1_small()
    mref = sampler.all_vectors(10)
    wref = sampler.ewald_weights(mref, s.L, alpha)
    rho_ref = oracle_lib.rho(s.x, s.y, s.z, s.q, mref, s.L)
    Fref = np.zeros((3, s.n))
    sel = np.arange(s.n)
    Fref = oracle_lib.force_subset(s.x, s.y, s.z, s.q, mref, wref, s.L, rho_ref, sel)
    k2 = np.sum((2 * np.pi * mref / s.L) ** 2, axis=1)
    Uref = float(np.sum(2 * np.pi / s.L ** 3 * wref / k2 * np.abs(rho_ref) ** 2))
    B = 150
    acc = np.zeros((B, 3, s.n))
    Us = np.zeros(B)
    for b in range(B):
        m, S = sampler.sample_k(2001 + b, 0, s.L, alpha, P)
        F, U, _ = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, np.full(P, S / P), s.L)
        acc[b] = F
        Us[b] = U
    mean = acc.mean(axis=0)
    sd = acc.std(axis=0, ddof=1) / math.sqrt(B)
    z = (mean - Fref) / sd
    rms_z = math.sqrt(np.mean(z * z))
    assert 0.85 < rms_z < 1.15, rms_z
    assert np.max(np.abs(z)) < 7
    zU = (Us.mean() - Uref) / (Us.std(ddof=1) / math.sqrt(B))
    assert abs(zU) < 4


@pytest.mark.parametrize("what", ["nan_x", "inf_y", "nan_q"])
def test_non_finite_input_gives_nan(oracle_lib, what):
    """The contract the library follows: a non-finite position or charge makes rho, every
    force and the energy NaN (the definition evaluated literally)."""
    s = ri.uniform_pm1(40, 6.0, 5)
    if what == "nan_x":
        s.x[7] = np.nan
    elif what == "inf_y":
        s.y[7] = np.inf
    else:
        s.q[7] = np.nan
    m, _ = sampler.sample_k(3, 0, s.L, 0.5, 6)
    w = np.full(6, sampler.normalization_S(s.L, 0.5) / 6)
    F, U, rho = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    assert np.all(np.isnan(rho)) and np.isnan(U) and np.all(np.isnan(F))


def test_thread_count_does_not_change_results(oracle_lib):
    s = ri.uniform_pm1(500, 8.0, 6)
    m, _ = sampler.sample_k(4, 0, s.L, 0.4, 12)
    w = np.ones(12)
    a = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    n0 = oracle_lib.num_threads()
    oracle_lib.set_num_threads(1)
    try:
        b = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    finally:
        oracle_lib.set_num_threads(n0)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2])
