"""GPU checks of the autotuner (rbe_plan_tune) and of the plans it leaves behind.

  * the variants it reports are in range and are the plan's variants afterwards;
  * the tuned plan (uploaded again by the tuner) still matches the FP64 oracle,
    for a single small system, a small batch and the 1M-atom electrolyte;
  * the cache round trip of tune.autotune keeps the winners under the shape's key.
"""
import numpy as np
import pytest
import torch

import oracle
import rbe_inputs as ri
from paper_2407_09315_amd import Batch, Plan, rbe_sample_k
from paper_2407_09315_amd.tune import autotune, load_cache, shape_key
from parity_util import MAX_TOL, dev, force_err, max_err, note, particles, rel, rho_err, to_dev

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32_mixed": 1e-5, "fp32": 1e-5}


def _tune_and_check(s, alpha, P, precision, seed):
    m, w, _ = rbe_sample_k(seed, 0, s.L, alpha, P)
    plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=precision, device=dev(), tiles=None)
    X = particles(s)
    mt, wt = to_dev(m, torch.int32), to_dev(w)
    res = plan.tune(*X, mt, wt, reps=3)
    nr, nf = plan.num_variants()
    note(f"case tune n={s.n} P={P} {precision}: {res}")
    assert 0 <= res["rho_variant"] < nr and 0 <= res["force_variant"] < nf
    assert res["rho_ms"] > 0 and res["force_ms"] > 0
    assert plan.tiles()[:2] == (res["rho_variant"], res["force_variant"])
    F, U, rho = plan.forward(*X, mt, wt)
    torch.cuda.synchronize()
    F, U, rho = F.double().cpu().numpy(), float(U.cpu()[0]), rho.cpu().numpy()
    F_ref, U_ref, rho_ref = oracle.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    tol = TOL[precision]
    ef, em, eu, er = force_err(F, F_ref), max_err(F, F_ref), rel(U, U_ref), rho_err(rho, rho_ref, s.q)
    note(f"  tuned: force {ef:.2e} (max {em:.2e})  U {eu:.2e}  rho {er:.2e}")
    assert ef < tol and eu < tol and er < tol and em < MAX_TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_tune_small_single(precision):
    s, alpha, P = ri.c1_small()
    _tune_and_check(s, alpha, P, precision, 2001)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_tune_1M(precision):
    s, alpha, P = ri.c3a_electrolyte()
    _tune_and_check(s, alpha, P, precision, 2003)


def test_tune_small_batch_and_cache(tmp_path):
    reps = ri.c5_replicas(B=6)
    systems = reps.systems
    batch = Batch.from_sizes([x.n for x in systems], [100] * 6, [x.L for x in systems], reps.alphas)
    plan = Plan(batch, precision="fp32_mixed", device=dev(), tiles=None)
    m, w = plan.sample_k_device(6000, 0)
    cat = [to_dev(np.concatenate([getattr(x, a) for x in systems])) for a in ("x", "y", "z", "q")]
    path = str(tmp_path / "cache.json")
    res = autotune(plan, *cat, m, w, reps=3, path=path)
    key = shape_key("fp32_mixed", "auto", 6, plan.n_total, plan.p_total)
    assert load_cache(path)[key]["rho_variant"] == res["rho_variant"] == plan.tiles()[0]
    F, U, rho = plan.forward(*cat, m, w)
    torch.cuda.synchronize()
    F, U, rho = F.double().cpu().numpy(), U.cpu().numpy(), rho.cpu().numpy()
    mh, wh = m.cpu().numpy(), w.cpu().numpy()
    no = 0
    for b, x in enumerate(systems):
        ks = slice(100 * b, 100 * (b + 1))
        F_ref, U_ref, rho_ref = oracle.force_energy(x.x, x.y, x.z, x.q, mh[ks], wh[ks], x.L)
        Fb = F[:, no:no + x.n]
        assert force_err(Fb, F_ref) < 1e-5 and max_err(Fb, F_ref) < MAX_TOL["fp32_mixed"]
        assert rel(U[b], U_ref) < 1e-5 and rho_err(rho[ks], rho_ref, x.q) < 1e-5
        no += x.n
