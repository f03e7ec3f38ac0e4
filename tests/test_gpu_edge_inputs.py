"""GPU checks of inputs at the edge of the contract in include/rbe.h.

  * a caller-supplied wave-vector list with zero rows m = (0, 0, 0): rho of those rows is
    sum q, and they add nothing to F, U, the virial or the VJP (the oracle's k = 0 weight
    is zero too), in every precision and in both rho layouts;
  * a NaN or infinite coordinate, or a NaN charge, makes rho, every force, the energy and
    the VJP outputs NaN in every precision (the fixed-point fraction of a non-finite
    coordinate is finite, so the FP32-mixed passes must carry it as a NaN charge).
"""
import numpy as np
import pytest
import torch

import oracle
import rbe_inputs as ri
from paper_2407_09315_amd import Batch, Plan, rbe_sample_k
from parity_util import MAX_TOL, dev, force_err, max_err, note, particles, rel, rho_err, to_dev

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32_mixed": 1e-5, "fp32": 1e-5}
# the k-lane rho layout of each precision, and the per-wave layout
LAYOUTS = {"fp64": (8, 0), "fp32_mixed": (9, 0), "fp32": (9, 0)}


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_zero_wave_vectors(precision, layout):
    s = ri.random_charges(2000, 12.0, 91)
    s.q -= s.q.mean() - 0.37 / s.n    # slightly non-neutral, so rho(0) = sum q is not zero
    m, w, _ = rbe_sample_k(92, 0, s.L, 0.3, 40)
    for row in (0, 17, 39):
        m[row] = 0
    rv = LAYOUTS[precision][layout]
    plan = Plan(Batch.single(s.n, 40, s.L, 0.3), precision=precision, device=dev(), tiles=(rv, 1))
    X = particles(s)
    mt, wt = to_dev(m, torch.int32), to_dev(w)
    F, U, rho = plan.forward(*X, mt, wt)
    W = plan.kspace_virial(mt, wt, rho)
    gF = to_dev(ri.gaussian_vectors(s.n, 93)).to(plan.force_dtype).contiguous()
    gU = torch.full((1,), 0.7, dtype=torch.float64, device=dev())
    gr, gq = plan.kspace_vjp(*X, mt, wt, rho, gU, gF)
    torch.cuda.synchronize()
    note(f"case zero wave vectors {precision} rho variant {rv}")
    F, U, rho = F.double().cpu().numpy(), float(U.cpu()[0]), rho.cpu().numpy()
    F_ref, U_ref, rho_ref = oracle.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    tol = TOL[precision]
    assert abs(rho_ref[17] - s.q.sum()) < 1e-12
    assert force_err(F, F_ref) < tol and max_err(F, F_ref) < MAX_TOL[precision]
    assert rel(U, U_ref) < tol and rho_err(rho, rho_ref, s.q) < tol
    W_ref = oracle.virial(m, w, s.L, 0.3, rho_ref)
    assert np.max(np.abs(W.cpu().numpy()[0] - W_ref)) < tol * np.max(np.abs(W_ref))
    gr_ref, gq_ref = oracle.vjp(s.x, s.y, s.z, s.q, m, w, s.L, 0.7, gF.double().cpu().numpy())
    gr, gq = gr.cpu().numpy(), gq.cpu().numpy()
    assert gr.dtype == np.float64 and gq.dtype == np.float64
    assert force_err(gr, gr_ref) < tol and force_err(gq, gq_ref) < tol
    # the zero rows alone: only rho(0) = sum q, no force and no energy
    z = np.zeros((3, 3), np.int32)
    F0, U0, rho0 = plan_forward_only(s, z, precision)
    assert np.all(F0 == 0) and U0 == 0.0
    assert np.max(np.abs(rho0[:, 0] - s.q.sum())) < tol * np.sqrt(np.sum(s.q ** 2))


def plan_forward_only(s, m, precision):
    plan = Plan(Batch.single(s.n, m.shape[0], s.L, 0.3), precision=precision, device=dev())
    F, U, rho = plan.forward(*particles(s), to_dev(m, torch.int32), to_dev(np.ones(m.shape[0])))
    torch.cuda.synchronize()
    return F.double().cpu().numpy(), float(U.cpu()[0]), rho.cpu().numpy()


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("what", ["nan_x", "inf_y", "ninf_z", "nan_q"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_non_finite_input_propagates(precision, what, layout):
    s = ri.uniform_pm1(3000, 14.0, 94)
    i = 1234
    if what == "nan_x":
        s.x[i] = np.nan
    elif what == "inf_y":
        s.y[i] = np.inf
    elif what == "ninf_z":
        s.z[i] = -np.inf
    else:
        s.q[i] = np.nan
    m, w, _ = rbe_sample_k(95, 0, s.L, 0.3, 30)
    rv = LAYOUTS[precision][layout]
    plan = Plan(Batch.single(s.n, 30, s.L, 0.3), precision=precision, device=dev(), tiles=(rv, 1))
    X = particles(s)
    mt, wt = to_dev(m, torch.int32), to_dev(w)
    F, U, rho = plan.forward(*X, mt, wt)
    gF = torch.ones((3, s.n), dtype=plan.force_dtype, device=dev())
    gU = torch.ones(1, dtype=torch.float64, device=dev())
    gr, gq = plan.kspace_vjp(*X, mt, wt, rho, gU, gF)
    torch.cuda.synchronize()
    note(f"case non-finite {what} {precision} rho variant {rv}")
    assert torch.isnan(rho).all() and torch.isnan(U).all()
    assert torch.isnan(F).all()
    assert torch.isnan(gr).all() and torch.isnan(gq).all()
