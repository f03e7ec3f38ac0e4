"""rbe_evaluate_static: the evaluation entry point that allocates nothing.

It runs the kernels of rbe_evaluate on a library-owned device scratch array instead of
a caller workspace, so its outputs must equal rbe_evaluate's bit for bit.  The GPU
cases call both through the C ABI on two calls in a row, the second with a smaller
system (so the scratch holds the first call's tables and partials when the second
starts), in FP32-mixed and FP64, and also check the static outputs against the FP64
oracle.  The host case checks the size limit, which is enforced before any launch.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import rbe_inputs as ri
from paper_2407_09315_amd import Batch, Plan, _lib, rbe
from parity_util import MAX_TOL, force_err, max_err, rel, rho_err

TOL = {"fp64": 1e-12, "fp32_mixed": 1e-5}


def _plan_handle(n, p, L, alpha, precision, mode):
    lib = _lib.load()
    arrs = [np.array(v) for v in ([0, n], [0, p])] + [np.array([L]), np.array([alpha])]
    arrs = [np.ascontiguousarray(a, dtype=t) for a, t in zip(arrs, (np.int64, np.int64, np.float64, np.float64))]
    desc = _lib.BatchDesc(1, *[rbe._ptr(a) for a in arrs])
    h = ctypes.c_void_p()
    assert lib.rbe_plan_create(ctypes.byref(desc), precision, mode, ctypes.byref(h)) == 0
    return h


def test_static_scratch_limit_is_checked_on_the_host():
    lib = _lib.load()
    # the phase cache of 200,000 charges x 100 wave vectors (160 MB) does not fit 64 MiB
    h = _plan_handle(200_000, 100, 126.0, 0.08, _lib.RBE_FP32_MIXED, _lib.RBE_PHASE_CACHED)
    st = lib.rbe_evaluate_static(h, 1, 0, *([None] * 11))
    assert st == _lib.RBE_EWORKSPACE
    assert b"rbe_evaluate_static" in lib.rbe_last_error()
    lib.rbe_plan_destroy(h)
    # a plan that fits passes the size check and reaches the device check
    h = _plan_handle(3000, 100, 31.0, 0.1, _lib.RBE_FP64, _lib.RBE_PHASE_AUTO)
    st = lib.rbe_evaluate_static(h, 1, 0, *([None] * 11))
    if not torch.cuda.is_available():
        assert st == _lib.RBE_ENODEV
    else:
        assert st == _lib.RBE_EINVAL   # NULL arrays
    lib.rbe_plan_destroy(h)


def _system(n, L, seed):
    g = np.random.default_rng(seed)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    g.shuffle(q)
    pos = g.uniform(0.0, L, size=(3, n))
    return pos[0], pos[1], pos[2], q


def _buffers(plan, dev):
    return (torch.full((plan.p_total, 3), -7, dtype=torch.int32, device=dev),
            torch.full((plan.p_total,), np.nan, dtype=torch.float64, device=dev),
            torch.full((plan.p_total, 2), np.nan, dtype=torch.float64, device=dev),
            torch.full((3, plan.n_total), np.nan, dtype=plan.force_dtype, device=dev),
            torch.full((1,), np.nan, dtype=torch.float64, device=dev))


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_static_equals_workspace_entry_point(precision):
    dev = torch.device("cuda:0")
    # first a 1M-atom-class tile count (several hundred tiles, ragged last tile), then a
    # smaller system with fewer wave vectors
    cases = [(150_001, 100, 115.0, 0.06, 7001), (3_000, 60, 31.0, 0.1, 7002)]
    for n, P, L, alpha, seed in cases:
        print(f"case static n={n} P={P} {precision}", flush=True)
        plan = Plan(Batch.single(n, P, L, alpha), precision=precision, device=dev)
        x, y, z, q = _system(n, L, seed)
        X = [torch.tensor(a, dtype=torch.float64, device=dev) for a in (x, y, z, q)]
        ref = _buffers(plan, dev)
        out = _buffers(plan, dev)
        rbe.rbe_evaluate(plan.handle, 11, 5, None, *X, *ref, plan.ws)
        rbe.rbe_evaluate_static(plan.handle, 11, 5, None, *X, *out)
        torch.cuda.synchronize()
        for a, b, name in zip(ref, out, ("m", "w", "rho", "F", "U")):
            assert torch.equal(a, b), (name, n, precision)
        # the static outputs against the FP64 oracle on the same wave vectors
        m, w = out[0].cpu().numpy(), out[1].cpu().numpy()
        F_ref, U_ref, rho_ref = oracle.force_energy(x, y, z, q, m, w, L)
        F = out[3].double().cpu().numpy()
        rho_c = out[2].cpu().numpy()
        tol = TOL[precision]
        assert force_err(F, F_ref) < tol and max_err(F, F_ref) < MAX_TOL[precision]
        assert rel(float(out[4].cpu()[0]), U_ref) < tol
        assert rho_err(rho_c, rho_ref, q) < tol
        plan.close()


@pytest.mark.gpu
def test_static_after_layout_change_and_with_step_counter():
    """A changed layout (other tile variants) is uploaded again; the step counter advances
    the same way as with rbe_evaluate."""
    dev = torch.device("cuda:0")
    s, alpha, P = ri.c1_small()
    plan = Plan(Batch.single(s.n, P, s.L, alpha), precision="fp32_mixed", device=dev, tiles=None)
    X = [torch.tensor(a, dtype=torch.float64, device=dev) for a in (s.x, s.y, s.z, s.q)]
    nr, nf = plan.num_variants()
    for rv, fv in ((0, 0), (nr - 1, nf - 1)):
        print(f"case static layout rv={rv} fv={fv}", flush=True)
        plan.set_tiles(rv, fv)
        c_ref = torch.zeros(1, dtype=torch.int64, device=dev)
        c_out = torch.zeros(1, dtype=torch.int64, device=dev)
        for _ in range(2):
            ref = _buffers(plan, dev)
            out = _buffers(plan, dev)
            rbe.rbe_evaluate(plan.handle, 3, 0, c_ref, *X, *ref, plan.ws)
            rbe.rbe_evaluate_static(plan.handle, 3, 0, c_out, *X, *out)
            torch.cuda.synchronize()
            for a, b in zip(ref, out):
                assert torch.equal(a, b)
        assert int(c_ref.item()) == int(c_out.item()) == 2
    plan.close()
