"""GPU parity of the forward path (rho, F, U) against the FP64 oracle.

Plans use the tuned kernel variants ("auto", the configuration bench.py times) unless a
test names its variants; test_all_variants runs every variant.

FP64 form: every measure <= 1e-12, the per-particle force measure
max_i |dF_i| / RMS|F_ref| <= 1e-11.  FP32 forms (fixed-point phases "fp32_mixed" and
FP32 phases "fp32"): every measure <= 1e-5, the per-particle one <= 1e-4.
Cases: the 3,000-charge box, the paper's electrolyte and water shapes, the
300k water box, the 200k differentiable box and the 1M electrolyte at P = 100
and 200 in full; the 10M electrolyte on all of rho and on sampled forces;
ragged and degenerate sizes; the full Ewald sum; the Madelung constant
through the GPU k-space; the phase-cache variant.
"""
import numpy as np
import pytest
import torch

import oracle
import rbe_inputs as ri
from oracle import sampler
from paper_2407_09315_amd import Batch, Plan, rbe_sample_k
from parity_util import (FP32_TOL, FP64_TOL, MAX_TOL, dev, force_err, max_err, note, particles, rel,
                         rho_err, to_dev)

pytestmark = pytest.mark.gpu
TOL = {"fp64": FP64_TOL, "fp32_mixed": FP32_TOL, "fp32": FP32_TOL}


def _run(s, alpha, m, w, precision, phase_mode="auto", tiles="auto"):
    plan = Plan(Batch.single(s.n, m.shape[0], s.L, alpha), precision=precision,
                phase_mode=phase_mode, device=dev(), tiles=tiles)
    X = particles(s)
    F, U, rho = plan.forward(*X, to_dev(m, torch.int32), to_dev(w))
    torch.cuda.synchronize()
    return F.double().cpu().numpy(), float(U.cpu()[0]), rho.cpu().numpy()


def _check(name, s, alpha, P, seed, precision, phase_mode="auto", tiles="auto"):
    m, w, S = rbe_sample_k(seed, 0, s.L, alpha, P)
    note(f"case {name} n={s.n} P={P} {precision} {phase_mode} tiles={tiles}")
    F, U, rho = _run(s, alpha, m, w, precision, phase_mode, tiles)
    F_ref, U_ref, rho_ref = oracle.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    ef, eu, er = force_err(F, F_ref), rel(U, U_ref), rho_err(rho, rho_ref, s.q)
    em = max_err(F, F_ref)
    note(f"  force {ef:.2e} (max per particle {em:.2e})  U {eu:.2e}  rho {er:.2e}")
    tol = TOL[precision]
    assert ef <= tol and eu <= tol and er <= tol and em <= MAX_TOL[precision]
    return ef, eu, er


SMALL = {
    "c1_3000": ri.c1_small,
    "e3_electrolyte": ri.e3_electrolyte,
    "e4_water": ri.e4_water,
}


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
@pytest.mark.parametrize("case", sorted(SMALL))
def test_small_parity(case, precision):
    s, alpha, P = SMALL[case]()
    _check(case, s, alpha, P, 2001, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1023, 1025, 5000])
def test_ragged_sizes(n, precision):
    s = ri.random_charges(n, 9.0, 40 + n)
    # positions partly outside the box: results are periodic in each coordinate
    s.x[::3] += 2 * s.L
    s.y[1::4] -= 3 * s.L
    if n == 1:
        # a lone charge feels no force from its own periodic images; its energy is q^2 sum c/2
        s.q[:] = 1.3
        m, w, _ = rbe_sample_k(18, 0, s.L, 0.3, 7)
        F, U, _ = _run(s, 0.3, m, w, precision)
        _, U_ref, _ = oracle.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
        assert rel(U, U_ref) < TOL[precision] and np.max(np.abs(F)) < TOL[precision] * U_ref
        return
    for P in (1, 7, 100):
        _check(f"ragged n={n}", s, 0.3, P, 17 + P, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_all_variants(precision):
    s, alpha, P = ri.c1_small()
    plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=precision, device=dev())
    nr, nf = plan.num_variants()
    for rv in range(nr):
        for fv in range(nf):
            _check("c1 variants", s, alpha, P, 2001, precision, tiles=(rv, fv))


# the k-lane rho layouts (5 wave vectors on each of 3 x 21 lanes, one (tile, k-range) item
# per block, at most 105 wave vectors per item): FP32 variants 9 (512-particle tiles), 10
# (256) and 11 (492), FP64 variants 8 (512) and 9 (492)
KLANE = 9
KLANE_256 = 10
KLANE_492 = 11
KLANE_COMP = 12      # 492-particle tiles, compensated FP32 sums in the forward pass
KLANE_F64 = 8
KLANE_F64_492 = 9
KLANE_CASES = [("fp32_mixed", KLANE), ("fp32_mixed", KLANE_256), ("fp32_mixed", KLANE_492),
               ("fp32_mixed", KLANE_COMP), ("fp32", KLANE), ("fp32", KLANE_256), ("fp32", KLANE_492),
               ("fp32", KLANE_COMP), ("fp64", KLANE_F64), ("fp64", KLANE_F64_492)]


@pytest.mark.parametrize("precision,rv", KLANE_CASES)
@pytest.mark.parametrize("n,P", [(1300, 250), (511, 105), (2049, 106), (64, 3)])
def test_klane_layout(n, P, rv, precision):
    """Several k-ranges per tile, a short last range, ragged and single tiles."""
    plan = Plan(Batch.single(n, P, 11.0, 0.35), precision=precision, device=dev())
    assert plan.rho_variant_info(rv)["waves_per_block"] == 1
    s = ri.random_charges(n, 11.0, 70 + n)
    _check(f"k-lane{rv} n={n}", s, 0.35, P, 300 + P, precision, tiles=(rv, 0))


@pytest.mark.parametrize("rv", [KLANE, KLANE_256, KLANE_492, KLANE_COMP])
def test_klane_layout_phase_cache(rv):
    """The phase cache with a k-lane variant selected runs the per-wave kernel on its items."""
    s = ri.random_charges(1300, 11.0, 71)
    _check(f"k-lane{rv} cached", s, 0.35, 250, 551, "fp32_mixed", phase_mode="cached", tiles=(rv, 0))


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_degenerate(precision):
    # P = 0: zero force, zero energy; n = 0: empty force, zero energy
    s = ri.random_charges(100, 5.0, 1)
    F, U, rho = _run(s, 0.5, np.zeros((0, 3), np.int32), np.zeros(0), precision)
    assert np.all(F == 0) and U == 0.0 and rho.size == 0
    plan = Plan(Batch.single(0, 10, 5.0, 0.5), precision=precision, device=dev())
    e = torch.empty(0, dtype=torch.float64, device=dev())
    m, w, _ = rbe_sample_k(3, 0, 5.0, 0.5, 10)
    F, U, rho = plan.forward(e, e, e, e, to_dev(m, torch.int32), to_dev(w))
    torch.cuda.synchronize()
    assert F.numel() == 0 and float(U[0]) == 0.0 and np.all(rho.cpu().numpy() == 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_two_charge_closed_form(precision):
    L, d = 7.0, 1.3
    s = ri.System(np.array([0.0, d]), np.zeros(2), np.zeros(2), np.array([1.0, -1.0]), L)
    m = np.array([[1, 0, 0]], dtype=np.int32)
    F, U, _ = _run(s, 1.0, m, np.ones(1), precision)
    k = 2 * np.pi / L
    c = 4 * np.pi / (L ** 3 * k * k)
    tol = TOL[precision]
    assert rel(U, c * (1 - np.cos(k * d))) < tol
    assert rel(F[0, 0], c * k * np.sin(k * d)) < tol and rel(F[0, 1], -c * k * np.sin(k * d)) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_full_ewald_kspace(precision):
    """Deterministic Ewald k-space sum over |m_d| <= 10 (Eq. long) through the same kernels."""
    s, alpha, _ = ri.c1_small()
    m = sampler.all_vectors(10)
    w = sampler.ewald_weights(m, s.L, alpha)
    note(f"case full-ewald {precision} K={m.shape[0]}")
    F, U, rho = _run(s, alpha, m, w, precision)
    F_ref, U_ref, rho_ref = oracle.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    tol = TOL[precision]
    assert force_err(F, F_ref) < tol and rel(U, U_ref) < tol and rho_err(rho, rho_ref, s.q) < tol
    assert max_err(F, F_ref) < MAX_TOL[precision]


def test_madelung_through_gpu_kspace():
    M = 1.7475645946331822
    s = ri.nacl_lattice(1)
    alpha = 2.5
    m = sampler.all_vectors(12)
    w = sampler.ewald_weights(m, s.L, alpha)
    _, Uk, _ = _run(s, alpha, m, w, "fp64")
    Ur, Us = oracle.ewald_real_self(s.x, s.y, s.z, s.q, s.L, alpha, 4)
    assert abs((Ur + Uk + Us) / (-4 * M) - 1) < 1e-11


LARGE = {
    "c2_water_300k": ri.c2_water,
    "c4_pm1_200k": ri.c4_differentiable,
}


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
@pytest.mark.parametrize("case", sorted(LARGE))
def test_large_parity(case, precision):
    s, alpha, P = LARGE[case]()
    _check(case, s, alpha, P, 2002, precision)


@pytest.fixture(scope="module")
def c3a():
    return ri.c3a_electrolyte()


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
@pytest.mark.parametrize("P", [100, 200])
def test_c3a_1M_parity(c3a, P, precision):
    s, alpha, _ = c3a
    _check("c3a_1M", s, alpha, P, 2003, precision)


def test_c3a_1M_cached_phase(c3a):
    s, alpha, _ = c3a
    _check("c3a_1M cached", s, alpha, 100, 2003, "fp32_mixed", phase_mode="cached")


# RBE_FP32 phases are refused for this box (sampled |m| spread 25.8 > 16)
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_c3b_10M_sampled(precision):
    s, alpha, P = ri.c3b_electrolyte()
    m, w, _ = rbe_sample_k(2004, 0, s.L, alpha, P)
    note(f"case c3b_10M {precision}")
    F, U, rho = _run(s, alpha, m, w, precision)
    rho_ref = oracle.rho(s.x, s.y, s.z, s.q, m, s.L)
    sel = np.random.default_rng(7).choice(s.n, 4000, replace=False)
    F_ref = oracle.force_subset(s.x, s.y, s.z, s.q, m, w, s.L, rho_ref, sel)
    k2 = np.sum((2 * np.pi * m / s.L) ** 2, axis=1)
    U_ref = float(np.sum(2 * np.pi / s.L ** 3 * w / k2 * np.abs(rho_ref) ** 2))
    tol = TOL[precision]
    ef, er, eu = force_err(F[:, sel], F_ref), rho_err(rho, rho_ref, s.q), rel(U, U_ref)
    em = max_err(F[:, sel], F_ref)
    note(f"  force(sampled) {ef:.2e} (max per particle {em:.2e})  U {eu:.2e}  rho {er:.2e}")
    assert ef < tol and er < tol and eu < tol and em < MAX_TOL[precision]
    # zero net force holds at any size
    assert np.max(np.abs(F.sum(axis=1))) < (1e-9 if precision == "fp64" else 1e-2) * np.sqrt(np.mean(F ** 2)) * s.n ** 0.5


def test_fp32_truncation_rotation_is_removed(c3a):
    """Mean phase offset of rho (FP32-mixed) against the oracle stays far below pi 2^-23."""
    s, alpha, _ = c3a
    m, w, _ = rbe_sample_k(2003, 0, s.L, alpha, 200)
    _, _, rho = _run(s, alpha, m, w, "fp32_mixed")
    rho_ref = oracle.rho(s.x, s.y, s.z, s.q, m, s.L)
    rc = rho[:, 0] + 1j * rho[:, 1]
    phase = np.angle(rc / rho_ref)
    wts = np.abs(rho_ref) ** 2
    mean = float(np.sum(phase * wts) / np.sum(wts))
    note(f"  mean phase offset {mean:.2e} rad (uncorrected would be {np.pi * 2 ** -23:.2e})")
    assert abs(mean) < 0.25 * np.pi * 2 ** -23


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_bitwise_deterministic(c3a, precision):
    s, alpha, _ = c3a
    m, w, _ = rbe_sample_k(2003, 0, s.L, alpha, 100)
    a = _run(s, alpha, m, w, precision)
    b = _run(s, alpha, m, w, precision)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2])
