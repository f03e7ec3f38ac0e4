"""Benchmark of the RBE k-space force on one MI355X.

A step is one whole evaluation of the hot path on the 1,000,000-atom
water + 1 mol/L NaCl box (alpha = 0.06 / A^2, P = 100 wave vectors):
  draw P wave vectors on the device -> rho(k) pass -> cross-tile reduction ->
  force/energy pass.
Inputs are resident in HBM before timing starts; nothing is skipped inside
the timed region.  The headline value is the FP32-mixed form in
G(particle*k)/s (N * P terms per evaluation).  Timed beside it and reported in
the same JSON line: the FP64 form, FP32 phases, the rho variant with
compensated FP32 sums, the phase-cache variant, P = 200, the adjoint, the
batched 128-replica form and the virial.

roofline: FP32 vector arithmetic.  Peak = 256 CU x 128 FMA lanes x 2 FLOP x
2.4 GHz = 157.3 TFLOP/s.  Algorithmic work per (particle, k) term in FP32 FMA
issue-equivalents (measured rates: FP32 FMA/mul/add 1, sin or cos 4): rho pass
phase 3 + sin + cos + 2 FMAs = 13; force pass phase 3 + sin + cos + 5 = 16;
two FLOP each.  achieved = FLOP-eq x N * P / kernel time (HIP events around
the dominant pass's kernel on its launch stream).

cpu_baseline: the FP64 oracle (plain C, OpenMP over independent outputs) on
the same box, the same system and the same wave vectors, median of 3 full
evaluations on all host threads and on one; it also gives the stated error of
each GPU form (relative RMS force error and the largest per-particle error
over the RMS force, energy and rho errors), and on the 10M-atom electrolyte
(all of rho, 4,000 sampled forces) the errors of FP32-mixed with plain and
with compensated rho sums and of FP64.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 vector peak of MI355X: 256 CUs x 128 FMA lanes x 2 FLOP x 2.4 GHz = 157.3 TFLOP/s.
PEAK_FLOP = 256 * 128 * 2 * 2.4e9
# Algorithmic work per (particle, wave vector) term in FP32 FMA issue-equivalents: an FP32
# FMA/mul/add is 1, sin or cos 4 (quarter rate, measured).  rho: phase 3 + sin + cos +
# 2 accumulating FMAs = 13; force: phase 3 + sin + cos + Im' 2 + 3 FMAs = 16.  x 2 FLOP each.
FLOP_RHO = 2 * (3 + 4 + 4 + 2)
FLOP_FORCE = 2 * (3 + 4 + 4 + 2 + 3)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="skip the extra forms and the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: 5 eager evaluations per form plus a 256 MiB device copy "
                         "(the reference kernel of known size for HBM counter scaling); prints no JSON")
    ap.add_argument("--profile-rbl", action="store_true",
                    help="short run for rocprofv3: 5 RBL evaluations of the 1M electrolyte at p = 30, then 5 "
                         "at p = 100, then a 256 MiB device copy (for HBM counter scaling); prints no JSON")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_form(torch, plan_cls, batch_cls, X, L, alpha, P, precision, phase_mode, steps, warmup, seed=2003,
             rho_variant=None):
    """Time whole evaluations replayed from one captured HIP graph, then time the two
    passes' kernels with HIP events placed around them on the launch stream.
    rho_variant: replace the tuned rho variant (the tuned force variant is kept)."""
    n = X[0].numel()
    dev = X[0].device
    plan = plan_cls(batch_cls.single(n, P, L, alpha), precision=precision, phase_mode=phase_mode)
    if rho_variant is not None:
        plan.set_tiles(rho_variant, plan.tiles()[1])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        counter = torch.zeros(1, dtype=torch.int64, device=dev)
        g = plan.graph(*X, seed=seed, stream_base=0, step_counter=counter)
        for _ in range(warmup):
            g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch()
        torch.cuda.synchronize()
        wall_graph = (time.perf_counter() - t0) / steps
        # the same evaluation enqueued by rbe_evaluate, back to back (no graph launch cost)
        counter2 = torch.zeros(1, dtype=torch.int64, device=dev)
        ev = None
        for _ in range(warmup):
            ev = plan.evaluate(*X, seed=seed, stream_base=0, step_counter=counter2, out=ev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ev = plan.evaluate(*X, seed=seed, stream_base=0, step_counter=counter2, out=ev)
        torch.cuda.synchronize()
        wall_eval = (time.perf_counter() - t0) / steps
        out = {"wall_s": min(wall_graph, wall_eval), "wall_graph_s": wall_graph, "wall_evaluate_s": wall_eval,
               "m": g.m.cpu().numpy(), "w": g.w.cpu().numpy(), "F": g.F.double().cpu().numpy(),
               "U": float(g.U.cpu()[0]), "rho": g.rho.cpu().numpy(), "tiles": plan.tiles(),
               "rho_kernel": rho_kernel_name(plan)}
        # kernel timing: the same step as eager calls, events around each pass's kernel
        m = torch.empty_like(g.m)
        w = torch.empty_like(g.w)
        rho = torch.empty_like(g.rho)
        F = torch.empty_like(g.F)
        U = torch.empty_like(g.U)
        evs = []
        for k in range(steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            for e in ev:
                e.record()
            plan.set_timing_events(*ev)
            plan.sample_k_device(seed, k, m, w)
            plan.structure_factor(*X, m, rho)
            plan.kspace_force(*X, m, w, rho, F, U)
            evs.append(ev)
        plan.set_timing_events()
        torch.cuda.synchronize()
    out["t_rho_s"] = float(np.mean([e[0].elapsed_time(e[1]) for e in evs])) * 1e-3
    out["t_force_s"] = float(np.mean([e[2].elapsed_time(e[3]) for e in evs])) * 1e-3
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)
    import torch

    import rbe_inputs as ri
    from paper_2407_09315_amd import Batch, Plan

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_rbl:
        profile_rbl(torch, ri, dev)
        return
    t_gen = time.perf_counter()
    s, alpha, P = ri.c3a_electrolyte()
    log(f"generated {s.name} (N={s.n}, L={s.L:.4f}) in {time.perf_counter() - t_gen:.1f}s")
    X = [torch.tensor(a, dtype=torch.float64, device=dev) for a in (s.x, s.y, s.z, s.q)]
    terms = s.n * P

    if args.profile:
        profile_run(torch, Plan, Batch, X, s, alpha, P, dev)
        return
    res = {}
    res["fp32"] = run_form(torch, Plan, Batch, X, s.L, alpha, P, "fp32_mixed", "recompute", args.steps, args.warmup)
    log(f"fp32_mixed: {res['fp32']['wall_s'] * 1e3:.3f} ms/step")
    res["fp64"] = run_form(torch, Plan, Batch, X, s.L, alpha, P, "fp64", "recompute", args.steps, args.warmup)
    log(f"fp64: {res['fp64']['wall_s'] * 1e3:.3f} ms/step")
    res["fp32_phase"] = run_form(torch, Plan, Batch, X, s.L, alpha, P, "fp32", "recompute", args.steps, args.warmup)
    log(f"fp32 (FP32 phases): {res['fp32_phase']['wall_s'] * 1e3:.3f} ms/step")
    r = res["fp32_phase"]
    extra = {"fp32_phase_P100": {"ms_per_step": round(r["wall_s"] * 1e3, 4),
                                 "G_terms_per_s": round(terms / r["wall_s"] / 1e9, 3),
                                 "rho_kernel_ms": round(r["t_rho_s"] * 1e3, 4),
                                 "force_kernel_ms": round(r["t_force_s"] * 1e3, 4), "tiles": r["tiles"]}}
    if not args.quick:
        comp = compensated_variant(Plan, Batch)
        res["fp32_comp"] = r = run_form(torch, Plan, Batch, X, s.L, alpha, P, "fp32_mixed", "recompute", args.steps,
                                        args.warmup, rho_variant=comp)
        extra["fp32_mixed_compensated_P100"] = {"ms_per_step": round(r["wall_s"] * 1e3, 4),
                                                "G_terms_per_s": round(terms / r["wall_s"] / 1e9, 3),
                                                "rho_kernel_ms": round(r["t_rho_s"] * 1e3, 4),
                                                "force_kernel_ms": round(r["t_force_s"] * 1e3, 4), "tiles": r["tiles"]}
        log("compensated done")
        r = run_form(torch, Plan, Batch, X, s.L, alpha, P, "fp32_mixed", "cached", max(5, args.steps // 5), 3)
        extra["fp32_mixed_cached_phase_P100"] = {"ms_per_step": r["wall_s"] * 1e3, "G_terms_per_s": terms / r["wall_s"] / 1e9,
                                                 "rho_kernel_ms": r["t_rho_s"] * 1e3, "force_kernel_ms": r["t_force_s"] * 1e3}
        log("cached done")
        for prec, key in (("fp32_mixed", "fp32_mixed_P200"), ("fp64", "fp64_P200")):
            r = run_form(torch, Plan, Batch, X, s.L, alpha, 200, prec, "recompute", max(5, args.steps // 5), 3)
            extra[key] = {"ms_per_step": r["wall_s"] * 1e3, "G_terms_per_s": s.n * 200 / r["wall_s"] / 1e9}
        log("P200 done")
        extra.update(bench_vjp(torch, ri, Plan, Batch, dev, max(5, args.steps // 5)))
        log("vjp done")
        extra.update(bench_batched(torch, ri, Plan, Batch, dev, max(5, args.steps // 5)))
        log("batched done")
        extra.update(bench_virial(torch, Plan, Batch, X, s, alpha, P, args.steps))
        log("virial done")
        extra.update(bench_rbl(torch, ri, dev, max(5, args.steps // 5), with_cpu=not args.no_cpu))
        log("rbl done")

    f32, f64 = res["fp32"], res["fp64"]
    value = terms / f32["wall_s"] / 1e9
    dom = "rho" if f32["t_rho_s"] >= f32["t_force_s"] else "force"
    rho_name = f32["rho_kernel"]
    t_dom = f32["t_rho_s"] if dom == "rho" else f32["t_force_s"]
    flop = FLOP_RHO if dom == "rho" else FLOP_FORCE
    achieved = flop * terms / t_dom / 1e12
    peak = PEAK_FLOP / 1e12
    out = {
        "metric": "RBE force G(particle·k)/s & ms/eval at 1M, FP32-mixed vs FP64 at stated err",
        "value": round(value, 3),
        "unit": "G(particle·k)/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["wall_s"] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "water+1M NaCl electrolyte, N=1,000,000, L=217.0535 A, alpha=0.06, P=100",
                   "N": s.n, "P": P, "L": s.L, "alpha": alpha, "precision": "fp32_mixed",
                   "phase_mode": "recompute",
                   "step": "device sampling + rho pass + reduction + force pass (one evaluation; the faster of "
                           "back-to-back rbe_evaluate calls and HIP graph replays)",
                   "ms_graph_replay": round(f32["wall_graph_s"] * 1e3, 4),
                   "ms_evaluate_calls": round(f32["wall_evaluate_s"] * 1e3, 4)},
        "fp64": {"ms_per_step": round(f64["wall_s"] * 1e3, 4), "G_terms_per_s": round(terms / f64["wall_s"] / 1e9, 3),
                 "ms_graph_replay": round(f64["wall_graph_s"] * 1e3, 4),
                 "ms_evaluate_calls": round(f64["wall_evaluate_s"] * 1e3, 4),
                 "rho_kernel_ms": round(f64["t_rho_s"] * 1e3, 4), "force_kernel_ms": round(f64["t_force_s"] * 1e3, 4),
                 "tiles": f64["tiles"]},
        "fp32_over_fp64_speedup": round(f64["wall_s"] / f32["wall_s"], 3),
        "fp32_kernels_ms": {"rho_kernel": round(f32["t_rho_s"] * 1e3, 4), "force_kernel": round(f32["t_force_s"] * 1e3, 4),
                            "tiles": f32["tiles"]},
        "roofline": {"bound": "alu", "kernel": rho_name if dom == "rho" else "force_f32_kernel",
                     "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4),
                     "traffic": traffic_from_profile(rho_name if dom == "rho" else "force_f32_kernel"),
                     "flop_equivalents_per_term": flop, "terms_per_launch": terms,
                     "other_pass": {"kernel": "force_f32_kernel" if dom == "rho" else rho_name,
                                    "frac": round((FLOP_FORCE if dom == "rho" else FLOP_RHO) * terms /
                                                  (f32["t_force_s"] if dom == "rho" else f32["t_rho_s"]) / PEAK_FLOP, 4)},
                     "whole_evaluation_frac": round((FLOP_RHO + FLOP_FORCE) * terms / f32["wall_s"] / PEAK_FLOP, 4)},
        "extra": extra,
    }
    if not args.quick and not args.no_cpu:
        out["cpu_baseline"], out["error_vs_oracle"] = cpu_baseline(s, P, res)
        del X
        out["error_vs_oracle"]["electrolyte_10M_P100"] = errors_10M(torch, ri, Plan, Batch, dev)
    print(json.dumps(out), flush=True)


def profile_run(torch, Plan, Batch, X, s, alpha, P, dev):
    for prec in ("fp32_mixed", "fp64"):
        plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=prec, phase_mode="recompute")
        m, w = plan.sample_k_device(2003, 0)
        for k in range(7):
            plan.sample_k_device(2003, k, m, w)
            plan.forward(*X, m, w)
        torch.cuda.synchronize()
        log(f"profile {prec}: tiles {plan.tiles()}")
    src = torch.ones(256 * 2 ** 20 // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("profile copy: 3 x 256 MiB")


def profile_rbl(torch, ri, dev):
    from paper_2407_09315_amd import RBLPlan
    s = ri.primitive_electrolyte(1_000_000, 0.01, 1006)
    X = [torch.tensor(a, dtype=torch.float64, device=dev) for a in (s.x, s.y, s.z, s.q, s.eps, s.sig)]
    for p in (30, 100):
        plan = RBLPlan(s.n, s.L, 0.06, 6.0, 12.0, p, device=dev)
        F, ns = plan.short_force(*X, seed=1, step=0)
        for k in range(1, 5):
            plan.short_force(*X, seed=1, step=k, F=F, ns=ns)
        torch.cuda.synchronize()
        log(f"profile rbl p={p}: 5 evaluations")
    src = torch.ones(256 * 2 ** 20 // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("profile copy: 3 x 256 MiB")


def rho_kernel_name(plan):
    """Name of the rho kernel the plan's selected variant launches (as rocprofv3 reports it)."""
    klane = plan.rho_variant_info(plan.tiles()[0])["waves_per_block"] == 1
    if plan.precision == "fp64":
        return "rho_klane_f64_kernel" if klane else "rho_f64_kernel"
    return "rho_klane_kernel" if klane else "rho_f32_kernel"


def traffic_from_profile(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when the
    summary is missing or was taken on a different kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_1M.md")
    src = os.path.join(ROOT, "paper_2407_09315_amd", "csrc", "rbe_kernels.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel source sha256") != digest:
        return None
    try:
        return float(fields["hbm bytes per launch"])
    except (KeyError, ValueError):
        return None


def rbl_traffic_from_profile(kernel: str, p: int):
    """HBM bytes per launch of the RBL `kernel` at batch size p (30 or 100) from the committed
    counter summary, or None when it is missing or was taken on a different kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "counters_rbl_electrolyte_1M.md")
    src = os.path.join(ROOT, "paper_2407_09315_amd", "csrc", "rbl_kernels.hip")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    text = open(path).read()
    if f"kernel source sha256 (rbl_kernels.hip): {digest}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] == f"`{kernel}`" and cells[1] == str(p):
            try:
                return float(cells[4].replace(",", "")) * 1e6
            except ValueError:
                return None
    return None


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline(s, P, res):
    """The FP64 oracle on the host: one full evaluation (rho + F + U) of the benchmark
    system with the GPU run's wave vectors, median of 3 timed runs after a warm-up, on all
    the threads OpenMP gives it and on one thread.  Its result also gives each GPU form's
    error."""
    import oracle
    m, w = res["fp32"]["m"], res["fp32"]["w"]

    def timed(reps):
        ts, out = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            out = oracle.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), out

    threads = oracle.num_threads()
    timed(1)                                    # warm-up
    t_all, (F_ref, U_ref, rho_ref) = timed(3)
    oracle.set_num_threads(1)
    try:
        t_one, _ = timed(3)
    finally:
        oracle.set_num_threads(threads)
    model, ncpu, navail = cpu_info()
    terms = s.n * P
    base = {"value": round(terms / t_all / 1e9, 5), "unit": "G(particle·k)/s", "cores": threads,
            "kind": "oracle",
            "sample": f"full evaluation (rho + F + U) of the same 1M-atom system and P={P} wave vectors, "
                      f"median of 3 runs after a warm-up: {t_all:.3f} s on {threads} threads",
            "single_core": {"value": round(terms / t_one / 1e9, 5), "unit": "G(particle·k)/s", "cores": 1,
                            "s_per_evaluation": round(t_one, 3), "sample": "the same evaluation, median of 3 runs"},
            "s_per_evaluation": round(t_all, 3), "cpu_model": model, "nproc": ncpu, "cpus_available": navail}
    errs = {}
    for key, prec in (("fp32", "fp32_mixed"), ("fp64", "fp64"), ("fp32_phase", "fp32"),
                      ("fp32_comp", "fp32_mixed_compensated")):
        if key not in res:
            continue
        r = res[key]
        if not np.array_equal(r["m"], m):
            F_ref2, U_ref2, rho_ref2 = oracle.force_energy(s.x, s.y, s.z, s.q, r["m"], r["w"], s.L)
        else:
            F_ref2, U_ref2, rho_ref2 = F_ref, U_ref, rho_ref
        F = r["F"]
        rc = r["rho"][:, 0] + 1j * r["rho"][:, 1]
        dF = np.sqrt(np.sum((F - F_ref2) ** 2, axis=0))
        errs[prec] = {"force_rel_rms": float(np.sqrt(np.sum((F - F_ref2) ** 2) / np.sum(F_ref2 ** 2))),
                      "force_max_particle_over_rms": float(dF.max() / np.sqrt(np.mean(np.sum(F_ref2 ** 2, axis=0)))),
                      "energy_rel": float(abs(r["U"] - U_ref2) / abs(U_ref2)),
                      "rho_max_over_qnorm": float(np.max(np.abs(rc - rho_ref2)) / np.sqrt(np.sum(s.q ** 2)))}
    return base, errs


def compensated_variant(Plan, Batch):
    """Index of the FP32 rho variant with compensated sums."""
    plan = Plan(Batch.single(1000, 8, 10.0, 0.5), precision="fp32_mixed", tiles=None)
    nr, _ = plan.num_variants()
    return next(v for v in range(nr) if plan.rho_variant_info(v)["compensated"] == 1)


def errors_10M(torch, ri, Plan, Batch, dev):
    """Errors of the FP32-mixed form (tuned rho variant and the compensated one) and of FP64 on
    the 10M-atom electrolyte, P = 100, against the oracle: all of rho, the energy, and the
    forces of 4,000 sampled particles (relative RMS and largest per-particle error over the
    sample's RMS force)."""
    import oracle
    s, alpha, _ = ri.c3b_electrolyte()
    P = 100
    X = [torch.tensor(a, dtype=torch.float64, device=dev) for a in (s.x, s.y, s.z, s.q)]
    comp = compensated_variant(Plan, Batch)
    out, ref = {}, None
    for name, prec, rv in (("fp32_mixed", "fp32_mixed", None), ("fp32_mixed_compensated", "fp32_mixed", comp),
                           ("fp64", "fp64", None)):
        plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=prec)
        if rv is not None:
            plan.set_tiles(rv, plan.tiles()[1])
        m, w = plan.sample_k_device(2004, 0)
        F, U, rho = plan.forward(*X, m, w)
        torch.cuda.synchronize()
        mh, wh = m.cpu().numpy(), w.cpu().numpy()
        if ref is None:
            sel = np.sort(np.random.default_rng(8).choice(s.n, 4000, replace=False))
            rho_ref = oracle.rho(s.x, s.y, s.z, s.q, mh, s.L)
            F_ref = oracle.force_subset(s.x, s.y, s.z, s.q, mh, wh, s.L, rho_ref, sel)
            k2 = np.sum((2 * np.pi * mh / s.L) ** 2, axis=1)
            U_ref = float(np.sum(2 * np.pi / s.L ** 3 * wh / k2 * np.abs(rho_ref) ** 2))
            ref = (mh, sel, rho_ref, F_ref, U_ref)
        assert np.array_equal(mh, ref[0])   # the same device-drawn wave vectors in every form
        _, sel, rho_ref, F_ref, U_ref = ref
        Fs = F[:, torch.tensor(sel, device=dev)].double().cpu().numpy()
        rc = rho[:, 0].cpu().numpy() + 1j * rho[:, 1].cpu().numpy()
        dF = np.sqrt(np.sum((Fs - F_ref) ** 2, axis=0))
        out[name] = {"tiles": plan.tiles(),
                     "force_rel_rms_sampled": float(np.sqrt(np.sum((Fs - F_ref) ** 2) / np.sum(F_ref ** 2))),
                     "force_max_particle_over_rms_sampled": float(dF.max() / np.sqrt(np.mean(np.sum(F_ref ** 2, axis=0)))),
                     "energy_rel": float(abs(float(U.cpu()[0]) - U_ref) / abs(U_ref)),
                     "rho_max_over_qnorm": float(np.max(np.abs(rc - rho_ref)) / np.sqrt(np.sum(s.q ** 2)))}
        plan.close()
        del F, U, rho
    return out


def bench_rbl(torch, ri, dev, steps, with_cpu=True):
    """RBL short-range force (cell list, core sum, shell batch, momentum correction) on the
    paper's primitive electrolyte at 0.01 particles / sigma^3, 1M particles, r_c = 6, r_s = 12,
    alpha = 0.06, p = 30 and 100: whole evaluations back to back.  With with_cpu, the FP64
    oracle's brute-force raw forces of 2,000 sampled particles (p = 30, median of 3) are timed
    beside it and compared with the GPU's (raw-force differences F_i - F_0, which the momentum
    correction leaves unchanged, and N_s).  The selection and pair kernels are timed with events
    the library records around them; each gets a roofline line against the FP64 vector peak (the
    rate of unpacked FP32 too), its work counted from the definition: the stencil population
    from the cell counts, the core and shell sizes from a periodic k-d tree."""
    from paper_2407_09315_amd import RBLPlan
    s = ri.primitive_electrolyte(1_000_000, 0.01, 1006)
    X = [torch.tensor(a, dtype=torch.float64, device=dev) for a in (s.x, s.y, s.z, s.q, s.eps, s.sig)]
    out = {}
    counts = None
    for p in (30, 100):
        plan = RBLPlan(s.n, s.L, 0.06, 6.0, 12.0, p, device=dev)
        F, ns = plan.short_force(*X, seed=1, step=0)
        for k in range(3):
            plan.short_force(*X, seed=1, step=k, F=F, ns=ns)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            plan.short_force(*X, seed=1, step=k, F=F, ns=ns)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        # the selection and pair kernels, with events recorded around them by the library
        evs = []
        for k in range(steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            for e in ev:
                e.record()
            plan.set_timing_events(*ev)
            plan.short_force(*X, seed=1, step=k, F=F, ns=ns)
            evs.append(ev)
        plan.set_timing_events()
        torch.cuda.synchronize()
        t_sel = float(np.mean([e[0].elapsed_time(e[1]) for e in evs])) * 1e-3
        t_pair = float(np.mean([e[2].elapsed_time(e[3]) for e in evs])) * 1e-3
        nc, R, span = plan.grid()
        if counts is None:
            counts = (stencil_population(s, nc, span),) + neighbour_counts(s, 6.0, 12.0)
        T, core, shell = counts
        pairs = float(core.sum() + np.minimum(shell, p).sum())
        lines = {
            "rbl_select_kernel": (t_sel, 8.0 * T * s.n,
                                  "8 FP64 FLOP per (particle, stencil candidate) distance test; "
                                  f"{T:.2f} candidates per particle"),
            "rbl_pair_kernel": (t_pair, 42.0 * pairs,
                                "42 FP64 FLOP per core or batch pair (distance 8, 1/r^2, r, 1/r 3, "
                                "Lennard-Jones with the mixing rules 13, real-space Coulomb 12, "
                                f"sum 6; erfc, exp, sqrt, divide as one each); {pairs / s.n:.2f} pairs per particle")}
        roof = {k: {"bound": "alu", "kernel": k, "achieved": round(f / t / 1e12, 3), "peak": 78.6,
                    "unit": "TFLOP/s", "frac": round(f / t / 78.6e12, 4),
                    "traffic": rbl_traffic_from_profile(k, p), "work": w, "kernel_ms": round(t * 1e3, 4)}
                for k, (t, f, w) in lines.items()}
        dom = max(roof, key=lambda k: roof[k]["kernel_ms"])
        key = f"rbl_short_force_electrolyte_1M_p{p}"
        out[key] = {
            "ms_per_evaluation": round(dt * 1e3, 4), "particles_per_s": round(s.n / dt, 1), "N": s.n,
            "L": round(s.L, 4), "r_c": 6.0, "r_s": 12.0, "p": p,
            "mean_shell_size": round(float(ns.double().mean()), 2), "grid": [nc, R, span],
            "pair_slots_per_particle": plan.capacity()[0],
            "select_kernel_ms": round(t_sel * 1e3, 4), "pair_kernel_ms": round(t_pair * 1e3, 4),
            "roofline": roof[dom], "roofline_other": [roof[k] for k in roof if k != dom]}
        if with_cpu and p == 30:
            import oracle
            seed, step = 1, steps - 1   # the last timed evaluation's batch
            sel = np.concatenate([[0], np.sort(np.random.default_rng(11).choice(np.arange(1, s.n), 1999,
                                                                                 replace=False))])
            u = oracle.rbl_offsets(seed, step, sel)
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                raw, ns_ref = oracle.rbl_raw_subset(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, 0.06, 6.0, 12.0, p, sel, u)
                ts.append(time.perf_counter() - t0)
            # one core on the first 250 of them
            threads = oracle.num_threads()
            oracle.set_num_threads(1)
            try:
                ts1 = []
                for _ in range(3):
                    t0 = time.perf_counter()
                    oracle.rbl_raw_subset(s.x, s.y, s.z, s.q, s.eps, s.sig, s.L, 0.06, 6.0, 12.0, p, sel[:250], u[:250])
                    ts1.append(time.perf_counter() - t0)
            finally:
                oracle.set_num_threads(threads)
            t_one = float(np.median(ts1))
            Fg = F.cpu().numpy()[:, sel]
            d_gpu, d_ref = Fg - Fg[:, :1], raw - raw[:, :1]
            rms = float(np.sqrt(np.mean(np.sum(raw ** 2, axis=0))))
            t_cpu = float(np.median(ts))
            out[key]["cpu_baseline"] = {
                "value": round(len(sel) / t_cpu, 1), "unit": "particles/s", "cores": threads,
                "kind": "oracle",
                "sample": f"raw RBL forces of {len(sel)} sampled particles of the same system (brute force over "
                          f"all N in the oracle), median of 3: {t_cpu:.3f} s",
                "single_core": {"value": round(250 / t_one, 1), "unit": "particles/s", "cores": 1,
                                "sample": f"the first 250 of those particles, median of 3: {t_one:.3f} s"}}
            out[key]["error_vs_oracle_sample"] = {
                "n_s_equal": bool(np.array_equal(ns.cpu().numpy()[sel], ns_ref)),
                "raw_force_difference_max_over_rms": float(np.max(np.sqrt(np.sum((d_gpu - d_ref) ** 2, axis=0))) / rms)}
        plan.close()
    return out


def stencil_population(s, nc, span):
    """Mean over particles of the number of particles in their cell stencil (span^3 cells,
    periodic), from the cell counts: sum over cells of n_c times its stencil's count, / N."""
    cell = [np.minimum(np.floor((v / s.L - np.floor(v / s.L)) * nc).astype(np.int64), nc - 1) for v in (s.x, s.y, s.z)]
    counts = np.bincount((cell[0] * nc + cell[1]) * nc + cell[2], minlength=nc ** 3).reshape(nc, nc, nc).astype(np.float64)
    acc = counts
    for axis in range(3):
        offs = range(span) if span == nc else range(-(span // 2), span // 2 + 1)
        acc = sum(np.roll(acc, o, axis=axis) for o in offs)
    return float((counts * acc).sum() / s.n)


def neighbour_counts(s, rc, rs):
    """(core, shell) neighbour counts per particle, r < r_c and r_c <= r <= r_s under the minimum
    image, from a periodic k-d tree (the work the pair kernel's definition implies)."""
    from scipy.spatial import cKDTree
    P = np.stack([s.x, s.y, s.z], 1)
    P = P - np.floor(P / s.L) * s.L
    P[P >= s.L] = 0.0
    tree = cKDTree(P, boxsize=s.L)
    c = tree.query_ball_point(P, rc, return_length=True, workers=8)
    a = tree.query_ball_point(P, rs, return_length=True, workers=8)
    return c - 1, a - c


def bench_virial(torch, Plan, Batch, X, s, alpha, P, steps):
    """Virial tensor (rbe_kspace_virial) after an FP32-mixed evaluation: mean kernel time."""
    plan = Plan(Batch.single(s.n, P, s.L, alpha), precision="fp32_mixed")
    m, w = plan.sample_k_device(2003, 0)
    F, U, rho = plan.forward(*X, m, w)
    W = plan.kspace_virial(m, w, rho)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.kspace_virial(m, w, rho, W)
    e1.record()
    torch.cuda.synchronize()
    return {"virial_tensor_fp32_mixed_P100": {"us_per_call": round(e0.elapsed_time(e1) * 1e3 / steps, 2),
                                              "W_xx_yy_zz_xy_xz_yz": [round(v, 6) for v in W[0].tolist()]}}


def bench_vjp(torch, ri, Plan, Batch, dev, steps):
    s, alpha, P = ri.c4_differentiable()
    X = [torch.tensor(a, dtype=torch.float64, device=dev) for a in (s.x, s.y, s.z, s.q)]
    out = {}
    for prec in ("fp32_mixed", "fp64"):
        plan = Plan(Batch.single(s.n, P, s.L, alpha), precision=prec)
        m, w = plan.sample_k_device(2005, 0)
        F, U, rho = plan.forward(*X, m, w)
        gF = torch.randn((3, s.n), device=dev, dtype=torch.float64).to(plan.force_dtype)
        gU = torch.ones(1, dtype=torch.float64, device=dev)
        gr, gq = plan.kspace_vjp(*X, m, w, rho, gU, gF)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            F, U, rho = plan.forward(*X, m, w)
            plan.kspace_vjp(*X, m, w, rho, gU, gF, gr, gq)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[f"vjp_{prec}_N200k_P100"] = {"ms_forward_plus_backward": dt * 1e3,
                                         "G_terms_per_s_4passes": 4 * s.n * P / dt / 1e9}
    return out


def bench_batched(torch, ri, Plan, Batch, dev, steps):
    reps = ri.c5_replicas(B=128)
    systems = reps.systems
    batch = Batch.from_sizes([x.n for x in systems], [reps.P] * len(systems), [x.L for x in systems], reps.alphas)
    plan = Plan(batch, precision="fp32_mixed")
    cat = [torch.tensor(np.concatenate([getattr(x, a) for x in systems]), dtype=torch.float64, device=dev)
           for a in ("x", "y", "z", "q")]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        counter = torch.zeros(1, dtype=torch.int64, device=dev)
        g = plan.graph(*cat, seed=6000, stream_base=0, step_counter=counter)
        for k in range(3):
            g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            g.launch()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
    terms = sum(x.n for x in systems) * reps.P
    return {"batched_128_replicas_fp32_mixed_graph": {"ms_per_step": dt * 1e3, "G_terms_per_s": terms / dt / 1e9,
                                                      "N_total": int(sum(x.n for x in systems)), "tiles": plan.tiles()}}


if __name__ == "__main__":
    main()
