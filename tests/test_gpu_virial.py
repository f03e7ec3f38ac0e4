"""GPU parity of the k-space virial tensor (rbe_kspace_virial) against the FP64 oracle.

The oracle's virial is pinned on the CPU by strain finite differences, isotropic
scaling and RBE unbiasedness (test_oracle_virial.py).  Here the GPU tensor, from the
GPU's own rho, must match the oracle's tensor from the oracle's rho:
max |dW| / max |W_ref| <= 1e-12 (FP64) or 1e-5 (FP32 forms).
"""
import numpy as np
import pytest
import torch

import oracle
import rbe_inputs as ri
from oracle import sampler
from paper_2407_09315_amd import Batch, Plan, rbe_sample_k
from parity_util import FP32_TOL, FP64_TOL, dev, note, particles, to_dev

pytestmark = pytest.mark.gpu
TOL = {"fp64": FP64_TOL, "fp32_mixed": FP32_TOL, "fp32": FP32_TOL}


def _gpu_virial(s, alpha, m, w, precision):
    plan = Plan(Batch.single(s.n, m.shape[0], s.L, alpha), precision=precision, device=dev())
    mt, wt = to_dev(m, torch.int32), to_dev(w)
    _, _, rho = plan.forward(*particles(s), mt, wt)
    W = plan.kspace_virial(mt, wt, rho)
    torch.cuda.synchronize()
    return W.cpu().numpy()[0]


def _err(W, Wref):
    return float(np.max(np.abs(W - Wref)) / np.max(np.abs(Wref)))


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
@pytest.mark.parametrize("case", ["c1_3000", "c2_water_300k", "c3a_1M"])
def test_virial_parity(case, precision):
    s, alpha, P = {"c1_3000": ri.c1_small, "c2_water_300k": ri.c2_water, "c3a_1M": ri.c3a_electrolyte}[case]()
    m, w, _ = rbe_sample_k(2101, 0, s.L, alpha, P)
    W = _gpu_virial(s, alpha, m, w, precision)
    Wref = oracle.virial(m, w, s.L, alpha, oracle.rho(s.x, s.y, s.z, s.q, m, s.L))
    e = _err(W, Wref)
    note(f"case {case} {precision} virial err {e:.2e}")
    assert e <= TOL[precision]


def test_virial_full_ewald():
    s, alpha, _ = ri.c1_small()
    m = sampler.all_vectors(10)
    w = sampler.ewald_weights(m, s.L, alpha)
    W = _gpu_virial(s, alpha, m, w, "fp64")
    Wref = oracle.virial(m, w, s.L, alpha, oracle.rho(s.x, s.y, s.z, s.q, m, s.L))
    assert _err(W, Wref) <= FP64_TOL


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_virial_batched(precision):
    reps = ri.c5_replicas(B=5)
    systems = reps.systems
    ps = [100, 37, 1, 64, 100]
    batch = Batch.from_sizes([x.n for x in systems], ps, [x.L for x in systems], reps.alphas)
    plan = Plan(batch, precision=precision, device=dev())
    cat = [to_dev(np.concatenate([getattr(x, a) for x in systems])) for a in ("x", "y", "z", "q")]
    ms, ws = [], []
    for b, x in enumerate(systems):
        m, w, _ = rbe_sample_k(600 + b, 2, x.L, reps.alphas[b], ps[b])
        ms.append(m)
        ws.append(w)
    mt, wt = to_dev(np.concatenate(ms), torch.int32), to_dev(np.concatenate(ws))
    _, _, rho = plan.forward(*cat, mt, wt)
    W = plan.kspace_virial(mt, wt, rho).cpu().numpy()
    for b, x in enumerate(systems):
        Wref = oracle.virial(ms[b], ws[b], x.L, reps.alphas[b], oracle.rho(x.x, x.y, x.z, x.q, ms[b], x.L))
        assert _err(W[b], Wref) <= TOL[precision], b
