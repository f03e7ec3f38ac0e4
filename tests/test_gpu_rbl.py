"""GPU parity of the random batch list (RBL) short-range force against the FP64 oracle.

  * whole systems (every force, every N_s) on the same batch offsets: the primitive
    electrolyte at the paper's density with p = 30 and 100, unequal LJ parameters, a
    particle count off the block size, a box whose stencil wraps, a batch larger than
    every shell (the exact truncated force), alpha = 0 and sqrt(alpha) r_s = 17 (the ends of
    the erfcx table), a dense box whose cells hold more than one group of targets and whose
    stencil is streamed in windows, r_c = r_s (no shell), 50 particles with p = 1, pairs at
    r_c and r_s to within 1e-10 (the FP64 decisions inside the selection's bands), a packed cluster whose particles have more pairs than the fast
    path's slots, and systems of 1, 2 and 7 particles (one in a box of mostly empty cells);
  * the 1M-particle benchmark system and a 10M one: N_s exact and the raw force differences F_i - F_0 of
    sampled particles (the momentum correction is one vector for all) against the oracle's
    brute-force raw forces of those particles, and sum_i F_i = 0;
  * repeated calls are bitwise equal, and a new step gives a new batch.
Bounds: FP64 element-wise, max_i |dF_i| / RMS |F| < 1e-11 and relative RMS < 1e-12; N_s
bit-exact (it is integer work).
"""
import numpy as np
import pytest
import torch

import oracle
import rbe_inputs as ri
from paper_2407_09315_amd import RBLPlan
from parity_util import dev, force_err, max_err, note, to_dev

pytestmark = pytest.mark.gpu


def _run(s, alpha, rc, rs, p, seed, step):
    plan = RBLPlan(s.n, s.L, alpha, rc, rs, p, device=dev())
    X = [to_dev(a) for a in (s.x, s.y, s.z, s.q, s.eps, s.sig)]
    F, ns = plan.short_force(*X, seed=seed, step=step)
    torch.cuda.synchronize()
    return plan, X, F.cpu().numpy(), ns.cpu().numpy()


CASES = [
    # (n, density, alpha, rc, rs, p, unequal LJ)
    (2000, 0.01, 0.06, 6.0, 12.0, 30, False),
    (2000, 0.01, 0.06, 6.0, 12.0, 100, False),
    (4099, 0.01, 0.1, 5.0, 11.0, 17, True),
    (250, 0.01, 0.06, 6.0, 12.0, 30, False),     # L = 29.2: 4 cells per axis, the stencil wraps
    (1500, 0.01, 0.06, 6.0, 12.0, 4000, False),  # batch larger than every shell: exact force
    (2500, 0.3, 0.3, 2.5, 5.0, 10, True),        # denser: about 5 particles per cell
    (2000, 1.0, 0.3, 2.5, 5.0, 20, True),        # 16 per cell, stencils of 2000 positions
    (2000, 0.01, 0.06, 8.0, 8.0, 30, False),     # r_c = r_s: the two bands coincide, no shell
    (50, 0.01, 0.1, 3.0, 8.0, 1, True),          # 50 particles, p = 1, the stencil wraps
    (2000, 0.01, 0.0, 6.0, 12.0, 30, True),      # alpha = 0: erfc = 1, the erfcx table is one interval
    (2000, 0.01, 2.0, 6.0, 12.0, 30, True),      # sqrt(alpha) r_s = 17: 170 table intervals
]


@pytest.mark.parametrize("n,density,alpha,rc,rs,p,unequal", CASES)
def test_rbl_parity(n, density, alpha, rc, rs, p, unequal):
    s = ri.primitive_electrolyte(n, density, 300 + n)
    if unequal:
        g = np.random.default_rng(n)
        s.eps = g.uniform(0.5, 1.5, n)
        s.sig = g.uniform(0.8, 1.3, n)
    seed, step = 77, 3
    note(f"case rbl n={n} L={s.L:.2f} rc={rc} rs={rs} p={p}")
    plan, X, F, ns = _run(s, alpha, rc, rs, p, seed, step)
    note(f"  grid {plan.grid()}")
    F_ref, ns_ref = oracle.rbl_short_force(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, alpha, rc, rs, p,
                                           oracle.rbl_offsets(seed, step, n))
    assert np.array_equal(ns, ns_ref)
    ef, em = force_err(F, F_ref), max_err(F, F_ref)
    note(f"  force rel RMS {ef:.2e}, max {em:.2e}, mean N_s {ns.mean():.1f}")
    assert ef < 1e-12 and em < 1e-11
    assert np.all(np.abs(F.sum(axis=1)) < 1e-11 * np.abs(F).sum(axis=1))
    plan.close()


@pytest.mark.parametrize("n,L,spread", [(1, 30.0, None), (2, 30.0, 2.5), (7, 30.0, None), (7, 60.0, 5.0),
                                         (7, 60.0, None)])
def test_rbl_parity_tiny(n, L, spread):
    """A handful of particles with random charges: one particle alone (no pairs, zero force),
    a close pair, 7 scattered particles, and 7 particles in a box of 1,728 cells, almost all
    of them empty, either clustered (core and shell pairs) or scattered (no pairs at all)."""
    g = np.random.default_rng(900 + n)
    if spread is None:
        x, y, z = (g.uniform(0.0, L, n) for _ in range(3))
    else:
        x, y, z = (g.uniform(0.0, L) + g.uniform(-spread, spread, n) for _ in range(3))
    q = g.choice([-1.0, 1.0], n)
    eps, sig = g.uniform(0.5, 1.5, n), g.uniform(0.8, 1.3, n)
    alpha, rc, rs, p, seed, step = 0.1, 5.0, 10.0, 3, 5, 2
    note(f"case rbl tiny n={n} L={L} spread={spread}")
    plan = RBLPlan(n, L, alpha, rc, rs, p, device=dev())
    X = [to_dev(a) for a in (x, y, z, q, eps, sig)]
    F, ns = plan.short_force(*X, seed=seed, step=step)
    torch.cuda.synchronize()
    F, ns = F.cpu().numpy(), ns.cpu().numpy()
    F_ref, ns_ref = oracle.rbl_short_force(x, y, z, q, eps, sig, L, alpha, rc, rs, p, oracle.rbl_offsets(seed, step, n))
    note(f"  grid {plan.grid()}, N_s {ns.tolist()}")
    assert np.array_equal(ns, ns_ref)
    if not np.any(F_ref != 0.0):
        assert np.all(F == 0.0)
    else:
        assert force_err(F, F_ref) < 1e-12 and max_err(F, F_ref) < 1e-11
    plan.close()


def _cutoff_band_system():
    """The electrolyte of 2,000 particles with 8 centres (L/2 apart, so that their groups do not
    meet), each with 5 particles at r_c (1 + d) and 5 at r_s (1 + d), d in {-1e-10, -1e-14, 0,
    1e-14, 1e-10}, along the directions of an icosahedron's vertices: squared distances
    inside the bands of the fixed-point estimate, which the FP64 distance decides.  The
    grid is offset by L/8 so that half of the groups straddle the periodic boundary.
    Background particles within 1.5 of any placed one are dropped."""
    s = ri.primitive_electrolyte(2000, 0.01, 777)
    rc, rs, L = 6.0, 12.0, s.L
    t = (1.0 + 5.0 ** 0.5) / 2.0
    ico = np.array([(0, 1, t), (0, -1, t), (0, 1, -t), (0, -1, -t), (1, t, 0), (-1, t, 0), (1, -t, 0), (-1, -t, 0),
                    (t, 0, 1), (t, 0, -1)], float)
    ico /= np.linalg.norm(ico, axis=1, keepdims=True)
    deltas = [-1e-10, -1e-14, 0.0, 1e-14, 1e-10]
    placed = []
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                c = np.array([cx, cy, cz]) * (L / 2) + L / 8 + (L / 2 - L / 8) * (cx == 0)
                c = np.mod(c - (L / 4 if cx == cy else 0.0), L)
                placed.append(c)
                for k, d in enumerate(deltas):
                    placed.append(c + rc * (1.0 + d) * ico[k])
                    placed.append(c + rs * (1.0 + d) * ico[5 + k])
    placed = np.array(placed)
    base = np.stack([s.x, s.y, s.z], 1)
    diff = base[:, None, :] - placed[None, :, :]
    diff -= L * np.rint(diff / L)
    keep = np.min(np.linalg.norm(diff, axis=2), axis=1) > 1.5
    pos = np.concatenate([placed, base[keep]])
    g = np.random.default_rng(5)
    q = np.concatenate([g.choice([-1.0, 1.0], len(placed)), s.q[keep]])
    eps = np.concatenate([g.uniform(0.5, 1.5, len(placed)), s.eps[keep]])
    sig = np.concatenate([g.uniform(0.8, 1.3, len(placed)), s.sig[keep]])
    return pos, q, eps, sig, L, len(placed)


@pytest.mark.parametrize("p", [30, 100])
def test_rbl_parity_cutoff_band(p):
    """Pairs at r_c and r_s to within 1e-10 relative: N_s bit-exact and the forces against the
    oracle, through the selection's FP64 decisions for the lanes inside its bands."""
    pos, q, eps, sig, L, npl = _cutoff_band_system()
    n = len(q)
    alpha, rc, rs, seed, step = 0.06, 6.0, 12.0, 13, 4
    note(f"case rbl cutoff band n={n} placed={npl} p={p}")
    plan = RBLPlan(n, L, alpha, rc, rs, p, device=dev())
    X = [to_dev(a) for a in (pos[:, 0], pos[:, 1], pos[:, 2], q, eps, sig)]
    F, ns = plan.short_force(*X, seed=seed, step=step)
    torch.cuda.synchronize()
    F, ns = F.cpu().numpy(), ns.cpu().numpy()
    F_ref, ns_ref = oracle.rbl_short_force(pos[:, 0], pos[:, 1], pos[:, 2], q, eps, sig, L, alpha, rc, rs, p,
                                           oracle.rbl_offsets(seed, step, n))
    assert np.array_equal(ns, ns_ref)
    ef, em = force_err(F, F_ref), max_err(F, F_ref)
    note(f"  force rel RMS {ef:.2e}, max {em:.2e}, N_s of the centres {ns[:npl:11].tolist()}")
    assert ef < 1e-12 and em < 1e-11
    plan.close()


def test_rbl_parity_crowded():
    """80 particles packed into a ball (density about 0.2 inside a box at 0.01): each has more
    core pairs than the plan's pair slots hold, so they take the slower path."""
    n, alpha, rc, rs, p = 2000, 0.06, 6.0, 12.0, 30
    s = ri.primitive_electrolyte(n, 0.01, 4242)
    g = np.random.default_rng(7)
    pts = np.array([(i, j, k) for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)], float) * 1.6
    pts = pts[np.argsort(np.linalg.norm(pts, axis=1), kind="stable")][:80]
    pts += g.uniform(-0.2, 0.2, pts.shape) + s.L / 2
    s.x[:80], s.y[:80], s.z[:80] = pts[:, 0], pts[:, 1], pts[:, 2]
    seed, step = 31, 2
    plan, X, F, ns = _run(s, alpha, rc, rs, p, seed, step)
    slots, _ = plan.capacity()
    note(f"case rbl crowded: pair slots {slots}")
    assert slots < 79
    F_ref, ns_ref = oracle.rbl_short_force(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, alpha, rc, rs, p,
                                           oracle.rbl_offsets(seed, step, n))
    assert np.array_equal(ns, ns_ref)
    ef, em = force_err(F, F_ref), max_err(F, F_ref)
    note(f"  force rel RMS {ef:.2e}, max {em:.2e}")
    assert ef < 1e-12 and em < 1e-11
    plan.close()


def test_rbl_non_finite_position():
    """A NaN or infinite coordinate is placed in cell 0 and gives NaN forces, which the
    momentum correction carries to every particle; positions outside [0, L) are wrapped."""
    s = ri.primitive_electrolyte(1500, 0.01, 77)
    for bad in (float("nan"), float("inf")):
        x = s.x.copy()
        x[5] = bad
        plan = RBLPlan(s.n, s.L, 0.06, 6.0, 12.0, 30, device=dev())
        X = [to_dev(a) for a in (x, s.y, s.z, s.q, s.eps, s.sig)]
        F, ns = plan.short_force(*X, seed=1, step=0)
        torch.cuda.synchronize()
        assert torch.isnan(F).all()
        plan.close()
    # shifted by whole periods: the same forces up to rounding
    plan = RBLPlan(s.n, s.L, 0.06, 6.0, 12.0, 30, device=dev())
    F0, n0 = plan.short_force(*[to_dev(a) for a in (s.x, s.y, s.z, s.q, s.eps, s.sig)], seed=1, step=0)
    F1, n1 = plan.short_force(*[to_dev(a) for a in (s.x + 3 * s.L, s.y - 2 * s.L, s.z, s.q, s.eps, s.sig)],
                              seed=1, step=0)
    torch.cuda.synchronize()
    assert torch.equal(n0, n1)
    assert force_err(F1.cpu().numpy(), F0.cpu().numpy()) < 1e-12
    plan.close()


def test_rbl_repeatable_and_step_dependent():
    s = ri.primitive_electrolyte(3000, 0.01, 12)
    plan = RBLPlan(s.n, s.L, 0.06, 6.0, 12.0, 30, device=dev())
    X = [to_dev(a) for a in (s.x, s.y, s.z, s.q, s.eps, s.sig)]
    F1, n1 = plan.short_force(*X, seed=5, step=0)
    F2, n2 = plan.short_force(*X, seed=5, step=0)
    F3, _ = plan.short_force(*X, seed=5, step=1)
    torch.cuda.synchronize()
    assert torch.equal(F1, F2) and torch.equal(n1, n2)
    assert not torch.equal(F1, F3)
    plan.close()


@pytest.mark.parametrize("n,seed_in", [(1_000_000, 1006), (10_000_000, 1007)])
def test_rbl_large_sampled(n, seed_in):
    """The benchmark system (1M particles, rc = 6, rs = 12, p = 30) and ten times it (10M,
    166^3 cells, a 4 GB workspace): N_s and raw force differences of 200 sampled particles
    against the oracle, and zero total force."""
    s = ri.primitive_electrolyte(n, 0.01, seed_in)
    alpha, rc, rs, p, seed, step = 0.06, 6.0, 12.0, 30, 9, 4
    note(f"case rbl n={n} L={s.L:.2f}")
    plan, X, F, ns = _run(s, alpha, rc, rs, p, seed, step)
    sel = np.concatenate([[0], np.sort(np.random.default_rng(2).choice(np.arange(1, s.n), 199, replace=False))])
    raw, ns_ref = oracle.rbl_raw_subset(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, alpha, rc, rs, p, sel,
                                        oracle.rbl_offsets(seed, step, sel))
    assert np.array_equal(ns[sel], ns_ref)
    d_gpu = F[:, sel] - F[:, sel[:1]]
    d_ref = raw - raw[:, :1]
    rms = np.sqrt(np.mean(np.sum(raw ** 2, axis=0)))
    err = np.max(np.sqrt(np.sum((d_gpu - d_ref) ** 2, axis=0))) / rms
    note(f"  max |d(F_i - F_0)| / RMS {err:.2e}, mean N_s {ns.mean():.1f}")
    assert err < 1e-11
    assert np.all(np.abs(F.sum(axis=1)) < 1e-10 * np.abs(F).sum(axis=1))
    plan.close()
