"""Kernel-variant autotuner driver and its JSON cache.

The timing itself is native (rbe_plan_tune: HIP events around every rho-pass
and force-pass variant on the caller's inputs).  This module keeps the
winners in a JSON file keyed by shape, so later plans of the same shape start
with the measured best variants:

  key = "<precision>|<phase_mode>|B=<systems>|N=<particles>|P=<wave vectors>"

Lookup falls back to the entry of the same precision, phase mode and system
count whose particle count is nearest on a log scale, then to the built-in
defaults.  The cache path is $RBE_TUNE_CACHE, else tune_cache.json next to
this file (measured on MI355X and kept with the sources).
"""
from __future__ import annotations

import json
import math
import os

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def cache_path() -> str:
    return os.environ.get("RBE_TUNE_CACHE", DEFAULT_CACHE)


def shape_key(precision: str, phase_mode: str, B: int, n_total: int, p_total: int) -> str:
    mode = "cached" if phase_mode == "cached" else "recompute"     # "auto" recomputes
    return f"{precision}|{mode}|B={B}|N={n_total}|P={p_total}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(precision: str, phase_mode: str, B: int, n_total: int, p_total: int, cache: dict | None = None):
    """(rho_variant, force_variant, rho_grid_cap, occupancy_clamp) for this shape, or None (defaults)."""
    cache = load_cache() if cache is None else cache
    key = shape_key(precision, phase_mode, B, n_total, p_total)
    if key in cache:
        e = cache[key]
        return e["rho_variant"], e["force_variant"], e.get("rho_grid_cap", 0), e.get("occupancy_clamp", 1)
    want_mode = key.split("|")[1]
    best, best_d = None, None
    for k, e in cache.items():
        prec, mode, b, n, p = k.split("|")
        if prec != precision or mode != want_mode or int(b[2:]) != B:
            continue
        if int(p[2:]) // B != p_total // max(B, 1):
            continue
        d = abs(math.log(max(int(n[2:]), 1)) - math.log(max(n_total, 1)))
        if best_d is None or d < best_d:
            best, best_d = (e["rho_variant"], e["force_variant"], e.get("rho_grid_cap", 0),
                            e.get("occupancy_clamp", 1)), d
    return best


def autotune(plan, x, y, z, q, m, w, reps: int = 10, path: str | None = None) -> dict:
    """Run the native tuner on these inputs, keep the winners in the plan and the cache."""
    res = plan.tune(x, y, z, q, m, w, reps=reps)
    cache = load_cache(path)
    key = shape_key(plan.precision, plan.phase_mode, plan.batch.B, plan.n_total, plan.p_total)
    cache[key] = res
    save_cache(cache, path)
    return res
