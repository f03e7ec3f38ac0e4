"""Autotune the benchmark workloads and write the tuning cache.

Usage: python -m paper_2407_09315_amd.tune_workloads [--out PATH] [--precisions fp64,...]
       [--only NAME,...] [--phase-modes auto,cached]
Shapes: 3,000 charges (P=100), 300k water, 1M electrolyte (P=100, 200),
10M electrolyte (P=100), 200k charges (P=100), 128 uneven replicas; each in
FP64, FP32-mixed and FP32 (where the plan accepts FP32 phases).  With --phase-modes
cached, the phase-cache form (FP32-mixed only) of the named shapes.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import rbe_inputs as ri  # noqa: E402

from .rbe import Batch, Plan, RBEError  # noqa: E402
from .tune import autotune, cache_path  # noqa: E402


def _single(name, s, alpha, P):
    return name, Batch.single(s.n, P, s.L, alpha), [s]


def workloads():
    out = []
    s, a, P = ri.c1_small()
    out.append(_single("c1", s, a, P))
    s, a, P = ri.c2_water()
    out.append(_single("c2", s, a, P))
    s, a, _ = ri.c3a_electrolyte()
    out.append(_single("c3a_P100", s, a, 100))
    out.append(_single("c3a_P200", s, a, 200))
    s, a, P = ri.c4_differentiable()
    out.append(_single("c4", s, a, P))
    s, a, P = ri.c3b_electrolyte()
    out.append(_single("c3b_P100", s, a, P))
    reps = ri.c5_replicas(B=128)
    out.append(("c5", Batch.from_sizes([x.n for x in reps.systems], [reps.P] * 128,
                                       [x.L for x in reps.systems], reps.alphas), reps.systems))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=cache_path())
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--precisions", default="fp32,fp32_mixed,fp64",
                    help="comma-separated precisions to tune; the cache keeps the other entries")
    ap.add_argument("--only", default="", help="comma-separated workload names (default: all)")
    ap.add_argument("--phase-modes", default="auto", help="comma-separated phase modes: auto, cached")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    only = set(filter(None, args.only.split(",")))
    for name, batch, systems in workloads():
        if only and name not in only:
            continue
        X = [torch.tensor(np.concatenate([getattr(s, a) for s in systems]), dtype=torch.float64, device=dev)
             for a in ("x", "y", "z", "q")]
        for prec in args.precisions.split(","):
            for mode in args.phase_modes.split(","):
                if mode == "cached" and prec != "fp32_mixed":
                    continue
                try:
                    plan = Plan(batch, precision=prec, phase_mode=mode, tiles=None)
                except RBEError as e:   # FP32 phases are refused for large boxes
                    print(f"{name} {prec} {mode}: skipped ({e})", flush=True)
                    continue
                m, w = plan.sample_k_device(7, 0)
                res = autotune(plan, *X, m, w, reps=args.reps, path=args.out)
                print(f"{name} {prec} {mode}: {res}", flush=True)
                plan.close()
        del X
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
