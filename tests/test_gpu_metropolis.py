"""GPU checks of the Metropolis sampler (the paper's procedure for Alg. 1 step 1).

  * the device chains equal the oracle's chains and the library's host chains bit for
    bit, for a batch of uneven systems (key seed + b per system);
  * whole evaluations and graph replays with the Metropolis sampler draw the oracle's
    wave vectors for every step of the device counter, and their forces match the oracle;
  * unbiasedness: the mean RBE force over 2,000 batches of Metropolis draws against the
    full Ewald k-space force (z-test, as for the exact sampler).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import rbe_inputs as ri
from oracle import sampler
from paper_2407_09315_amd import Batch, Plan, rbe_sample_k_metropolis
from parity_util import MAX_TOL, dev, force_err, max_err, note, particles, rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("burn_in", [0, 1, 64])
def test_device_metropolis_bit_exact(burn_in):
    reps = ri.c5_replicas(B=12)
    systems = reps.systems
    batch = Batch.from_sizes([x.n for x in systems], [reps.P] * 12, [x.L for x in systems], reps.alphas)
    plan = Plan(batch, precision="fp32_mixed", device=dev())
    plan.set_sampler("metropolis", burn_in)
    note(f"case metropolis device burn_in={burn_in}")
    m, w = plan.sample_k_device(6000, 3)
    m, w = m.cpu().numpy(), w.cpu().numpy()
    for b, x in enumerate(systems):
        ks = slice(reps.P * b, reps.P * (b + 1))
        m_ref, S_ref = sampler.metropolis_k(6000 + b, 3, x.L, reps.alphas[b], reps.P, burn_in)
        m_lib, w_lib, _ = rbe_sample_k_metropolis(6000 + b, 3, x.L, reps.alphas[b], reps.P, burn_in)
        assert np.array_equal(m[ks], m_ref) and np.array_equal(m[ks], m_lib), b
        assert np.all(w[ks] == w_lib)


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_evaluate_and_graph_with_metropolis(precision):
    s, alpha, P = ri.c1_small()
    plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=precision, device=dev())
    plan.set_sampler("metropolis", 48)
    X = particles(s)
    counter = torch.zeros(1, dtype=torch.int64, device=dev())
    tol = 1e-12 if precision == "fp64" else 1e-5
    for step in range(3):
        note(f"case metropolis evaluate {precision} step {step}")
        m, w, rho, F, U = plan.evaluate(*X, seed=17, stream_base=100, step_counter=counter)
        torch.cuda.synchronize()
        m_ref, _ = sampler.metropolis_k(17, 100 + step, s.L, alpha, P, 48)
        mh = m.cpu().numpy()
        assert np.array_equal(mh, m_ref)
        F_ref, U_ref, _ = oracle.force_energy(s.x, s.y, s.z, s.q, mh, w.cpu().numpy(), s.L)
        Fh = F.double().cpu().numpy()
        assert force_err(Fh, F_ref) < tol and max_err(Fh, F_ref) < MAX_TOL[precision]
        assert rel(float(U.cpu()[0]), U_ref) < tol
    # graph replays continue the same counter
    g = plan.graph(*X, seed=17, stream_base=100, step_counter=counter)
    for step in range(3, 5):
        g.launch()
        torch.cuda.synchronize()
        m_ref, _ = sampler.metropolis_k(17, 100 + step, s.L, alpha, P, 48)
        assert np.array_equal(g.m.cpu().numpy(), m_ref)
    g.close()


def test_metropolis_unbiased_against_full_ewald():
    """Mean of B = 2000 RBE batches with Metropolis draws vs the full Ewald k-space force."""
    s, alpha, P = ri.c1_small()
    B = 2000
    mref = sampler.all_vectors(10)
    wref = sampler.ewald_weights(mref, s.L, alpha)
    Fe, Ue, _ = oracle.force_energy(s.x, s.y, s.z, s.q, mref, wref, s.L)
    plan = Plan(Batch.from_sizes([s.n] * B, [P] * B, [s.L] * B, [alpha] * B), precision="fp64", device=dev())
    plan.set_sampler("metropolis")
    m, w = plan.sample_k_device(2001, 0)
    cat = [t.repeat(B) for t in particles(s)]
    F, U, _ = plan.forward(*cat, m, w)
    F = F.cpu().numpy().reshape(3, B, s.n)
    U = U.cpu().numpy()
    mean, sd = F.mean(axis=1), F.std(axis=1, ddof=1) / math.sqrt(B)
    z = (mean - Fe) / sd
    rms = math.sqrt(np.mean(z * z))
    zU = (U.mean() - Ue) / (U.std(ddof=1) / math.sqrt(B))
    note(f"  RMS z {rms:.3f}, max |z| {np.abs(z).max():.2f}, z_U {zU:.2f}")
    assert 0.9 < rms < 1.1 and np.abs(z).max() < 6 and abs(zU) < 4
