"""GPU parity at the full sizes of the benchmark workloads, with the tuned kernel variants
(the configuration bench.py times).

  * 128 uneven replicas (9.38M charges, P = 100 each, one batch): every replica's rho in
    full, its energy, and 256 sampled forces per replica against the FP64 oracle, in
    FP32-mixed and FP64;
  * the 10M-atom electrolyte at P = 200: all of rho, the energy and 4,000 sampled forces,
    in FP32-mixed and FP64.
The oracle computes sampled forces one particle at a time from its own rho.
"""
import numpy as np
import pytest
import torch

import oracle
import rbe_inputs as ri
from paper_2407_09315_amd import Batch, Plan, rbe_sample_k
from parity_util import MAX_TOL, dev, force_err, max_err, note, rel, rho_err, to_dev

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32_mixed": 1e-5}


def _energy(m, w, L, rho_ref):
    k2 = np.sum((2 * np.pi * m / L) ** 2, axis=1)
    return float(np.sum(2 * np.pi / L ** 3 * w / k2 * np.abs(rho_ref) ** 2))


@pytest.fixture(scope="module")
def c5():
    reps = ri.c5_replicas(B=128)
    systems = reps.systems
    batch = Batch.from_sizes([x.n for x in systems], [reps.P] * 128, [x.L for x in systems], reps.alphas)
    return reps, batch


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_c5_128_replicas(c5, precision):
    reps, batch = c5
    systems = reps.systems
    plan = Plan(batch, precision=precision, device=dev())
    note(f"case c5 128 replicas {precision} N={plan.n_total} tiles={plan.tiles()}")
    m, w = plan.sample_k_device(6000, 0)
    cat = [to_dev(np.concatenate([getattr(x, a) for x in systems])) for a in ("x", "y", "z", "q")]
    F, U, rho = plan.forward(*cat, m, w)
    torch.cuda.synchronize()
    F, U, rho = F.double().cpu().numpy(), U.cpu().numpy(), rho.cpu().numpy()
    mh, wh = m.cpu().numpy(), w.cpu().numpy()
    del cat
    tol = TOL[precision]
    g = np.random.default_rng(11)
    worst = [0.0, 0.0, 0.0, 0.0]
    no = 0
    for b, x in enumerate(systems):
        ks = slice(reps.P * b, reps.P * (b + 1))
        rho_ref = oracle.rho(x.x, x.y, x.z, x.q, mh[ks], x.L)
        sel = np.sort(g.choice(x.n, 256, replace=False))
        F_ref = oracle.force_subset(x.x, x.y, x.z, x.q, mh[ks], wh[ks], x.L, rho_ref, sel)
        Fb = F[:, no + sel]
        errs = (force_err(Fb, F_ref), max_err(Fb, F_ref), rel(U[b], _energy(mh[ks], wh[ks], x.L, rho_ref)),
                rho_err(rho[ks], rho_ref, x.q))
        worst = [max(a, e) for a, e in zip(worst, errs)]
        assert errs[0] < tol and errs[2] < tol and errs[3] < tol and errs[1] < MAX_TOL[precision], (b, errs)
        no += x.n
    note(f"  worst over replicas: force {worst[0]:.2e} (max {worst[1]:.2e})  U {worst[2]:.2e}  rho {worst[3]:.2e}")


@pytest.fixture(scope="module")
def c3b_p200():
    s, alpha, _ = ri.c3b_electrolyte()
    m, w, _ = rbe_sample_k(2004, 0, s.L, alpha, 200)
    rho_ref = oracle.rho(s.x, s.y, s.z, s.q, m, s.L)
    return s, alpha, m, w, rho_ref


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_c3b_10M_P200(c3b_p200, precision):
    s, alpha, m, w, rho_ref = c3b_p200
    plan = Plan(Batch.single(s.n, 200, s.L, alpha), precision=precision, device=dev())
    note(f"case c3b 10M P=200 {precision} tiles={plan.tiles()}")
    X = [to_dev(a) for a in (s.x, s.y, s.z, s.q)]
    F, U, rho = plan.forward(*X, to_dev(m, torch.int32), to_dev(w))
    torch.cuda.synchronize()
    F, U, rho = F.double().cpu().numpy(), float(U.cpu()[0]), rho.cpu().numpy()
    del X
    sel = np.sort(np.random.default_rng(8).choice(s.n, 4000, replace=False))
    F_ref = oracle.force_subset(s.x, s.y, s.z, s.q, m, w, s.L, rho_ref, sel)
    ef, em = force_err(F[:, sel], F_ref), max_err(F[:, sel], F_ref)
    eu, er = rel(U, _energy(m, w, s.L, rho_ref)), rho_err(rho, rho_ref, s.q)
    note(f"  force(sampled) {ef:.2e} (max {em:.2e})  U {eu:.2e}  rho {er:.2e}")
    tol = TOL[precision]
    assert ef < tol and eu < tol and er < tol and em < MAX_TOL[precision]
