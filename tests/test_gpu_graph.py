"""GPU checks of the captured evaluation graph and persistent grids.

  * every replay of rbe_graph equals the eager calls with the same wave vectors,
    bit for bit, with eager work and synchronisations between the replays, and
    the device step counter advances once per replay;
  * capped (persistent) grids give bitwise the results of one block per item.
"""
import numpy as np
import pytest
import torch

import rbe_inputs as ri
from paper_2407_09315_amd import Batch, Plan, rbe_sample_k
from parity_util import note, particles, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_graph_replays_match_eager(precision):
    reps = ri.c5_replicas(B=4)
    systems = reps.systems
    batch = Batch.from_sizes([s.n for s in systems], [100] * 4, [s.L for s in systems], reps.alphas)
    plan = Plan(batch, precision=precision)
    cat = [to_dev(np.concatenate([getattr(s, a) for s in systems])) for a in ("x", "y", "z", "q")]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        counter = torch.zeros(1, dtype=torch.int64, device=cat[0].device)
        g = plan.graph(*cat, seed=900, stream_base=5, step_counter=counter)
        for r in range(3):
            g.launch()
            torch.cuda.synchronize()
            note(f"replay {r} {precision}")
            # eager evaluation with the same wave vectors, run between replays
            m, w = plan.sample_k_device(900, 5 + r)
            F, U, rho = plan.forward(*cat, m, w)
            torch.cuda.synchronize()
            assert torch.equal(g.m, m) and torch.equal(g.w, w)
            assert torch.equal(g.rho, rho) and torch.equal(g.F, F) and torch.equal(g.U, U)
            mh, _, _ = rbe_sample_k(900 + 1, 5 + r, systems[1].L, reps.alphas[1], 100)
            assert np.array_equal(g.m[100:200].cpu().numpy(), mh)
            assert int(counter.item()) == r + 1


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_evaluate_matches_graph_replays(precision):
    """rbe_evaluate enqueues the graph's sequence: back-to-back calls equal the replays bitwise."""
    reps = ri.c5_replicas(B=3)
    systems = reps.systems
    batch = Batch.from_sizes([s.n for s in systems], [64] * 3, [s.L for s in systems], reps.alphas)
    plan = Plan(batch, precision=precision)
    cat = [to_dev(np.concatenate([getattr(s, a) for s in systems])) for a in ("x", "y", "z", "q")]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        c_graph = torch.zeros(1, dtype=torch.int64, device=cat[0].device)
        c_eval = torch.zeros(1, dtype=torch.int64, device=cat[0].device)
        g = plan.graph(*cat, seed=77, stream_base=3, step_counter=c_graph)
        out = None
        for r in range(4):
            g.launch()
            out = plan.evaluate(*cat, seed=77, stream_base=3, step_counter=c_eval, out=out)
            torch.cuda.synchronize()
            for a, b in zip((g.m, g.w, g.rho, g.F, g.U), out):
                assert torch.equal(a, b), r
        assert int(c_graph.item()) == 4 and int(c_eval.item()) == 4


# rho variants with the same (particles per lane, chunk) under both schedules:
# 16-wave blocks sharing single-chunk items, and one item per wave
SCHEDULES = {"fp64": (7, 5), "fp32_mixed": (7, 0), "fp32": (7, 0)}


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
@pytest.mark.parametrize("schedule", [0, 1])
def test_persistent_grid_caps_bitwise(precision, schedule):
    s, alpha, P = ri.c4_differentiable()
    m, w, _ = rbe_sample_k(5, 0, s.L, alpha, P)
    X = particles(s)
    mt, wt = to_dev(m, torch.int32), to_dev(w)
    plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=precision, tiles=(SCHEDULES[precision][schedule], 0))
    F0, U0, r0 = plan.forward(*X, mt, wt)
    for caps in [(37, 5), (1024, 256), (1, 1)]:
        plan.set_grid_caps(*caps)
        F1, U1, r1 = plan.forward(*X, mt, wt)
        torch.cuda.synchronize()
        assert torch.equal(F0, F1) and torch.equal(U0, U1) and torch.equal(r0, r1), caps


@pytest.mark.parametrize("precision,rv", [("fp32_mixed", 9), ("fp32_mixed", 10), ("fp32_mixed", 11), ("fp32", 9),
                                          ("fp32", 10), ("fp64", 8), ("fp64", 9)])
def test_klane_grid_caps_bitwise(precision, rv):
    """The k-lane rho layouts under persistent grids (blocks striding over the items)."""
    s, alpha, _ = ri.c4_differentiable()
    P = 230                                   # three k-ranges per tile
    m, w, _ = rbe_sample_k(8, 0, s.L, alpha, P)
    X = particles(s)
    mt, wt = to_dev(m, torch.int32), to_dev(w)
    plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=precision, tiles=(rv, 0))
    F0, U0, r0 = plan.forward(*X, mt, wt)
    for caps in [(37, 5), (1024, 256), (1, 1)]:
        plan.set_grid_caps(*caps)
        F1, U1, r1 = plan.forward(*X, mt, wt)
        torch.cuda.synchronize()
        assert torch.equal(F0, F1) and torch.equal(U0, U1) and torch.equal(r0, r1), caps


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32"])
def test_schedules_agree_bitwise(precision):
    """The per-(k, tile) partial sums do not depend on the schedule that computed them."""
    s, alpha, P = ri.c2_water()
    m, w, _ = rbe_sample_k(6, 0, s.L, alpha, P)
    X = particles(s)
    mt, wt = to_dev(m, torch.int32), to_dev(w)
    out = []
    for rv in SCHEDULES[precision]:
        plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=precision, tiles=(rv, 0))
        out.append(plan.forward(*X, mt, wt))
    torch.cuda.synchronize()
    (F0, U0, r0), (F1, U1, r1) = out
    assert torch.equal(F0, F1) and torch.equal(U0, U1) and torch.equal(r0, r1)
