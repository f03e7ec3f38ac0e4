"""Python binding of the RBE C ABI (argument marshalling only).

Functions with the C names take torch tensors (device memory) or numpy arrays
(host memory) and pass raw pointers; every computation happens in librbe.so.
``Plan`` bundles a plan, its device workspace and the current torch stream.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import (RBE_FP32, RBE_FP32_MIXED, RBE_FP64, RBE_PHASE_AUTO, RBE_PHASE_CACHED,  # noqa: F401
                   RBE_PHASE_RECOMPUTE, RBEError, check, load)

PRECISIONS = {"fp64": RBE_FP64, "fp32_mixed": RBE_FP32_MIXED, "fp32": RBE_FP32}

# Library handles still alive.  At interpreter exit they are released by an atexit hook
# (graphs first, then plans), which runs before the HIP runtime unloads; finalisers that
# run later find the handles already released and do nothing.
_live_graphs: "weakref.WeakSet" = weakref.WeakSet()
_live_plans: "weakref.WeakSet" = weakref.WeakSet()
_released_all = False


def _release_all():
    global _released_all
    for g in list(_live_graphs):
        g.close()
    for p in list(_live_plans):
        p.close()
    _released_all = True


atexit.register(_release_all)
PHASE_MODES = {"auto": RBE_PHASE_AUTO, "recompute": RBE_PHASE_RECOMPUTE, "cached": RBE_PHASE_CACHED}


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if isinstance(t, torch.Tensor):
        return ctypes.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(ctypes.c_void_p)
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    raise TypeError(f"cannot pass {type(t)} as a pointer")


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor (got {t.dtype})")
    return t


# ---------------------------------------------------------------------- host calls

def rbe_sample_k(seed: int, stream_id: int, L: float, alpha: float, P: int):
    """(m (P, 3) int32, w (P,) float64 = S/P, S) from the library's host sampler."""
    m = np.zeros((P, 3), dtype=np.int32)
    w = np.zeros(P, dtype=np.float64)
    S = np.zeros(1, dtype=np.float64)
    check(load().rbe_sample_k(seed, stream_id, L, alpha, P, _ptr(m), _ptr(w), _ptr(S)), "rbe_sample_k")
    return m, w, float(S[0])


def rbe_sample_k_metropolis(seed: int, stream_id: int, L: float, alpha: float, P: int, burn_in: int = 64):
    """(m (P, 3) int32, w (P,) float64 = S/P, S) from the library's Metropolis chains."""
    m = np.zeros((P, 3), dtype=np.int32)
    w = np.zeros(P, dtype=np.float64)
    S = np.zeros(1, dtype=np.float64)
    check(load().rbe_sample_k_metropolis(seed, stream_id, L, alpha, P, burn_in, _ptr(m), _ptr(w), _ptr(S)),
          "rbe_sample_k_metropolis")
    return m, w, float(S[0])


def rbe_normalization(L: float, alpha: float) -> float:
    S = np.zeros(1, dtype=np.float64)
    check(load().rbe_normalization(L, alpha, _ptr(S)), "rbe_normalization")
    return float(S[0])


def rbe_ewald_weights(L: float, alpha: float, m: np.ndarray) -> np.ndarray:
    m = np.ascontiguousarray(m, dtype=np.int32)
    w = np.zeros(m.shape[0], dtype=np.float64)
    check(load().rbe_ewald_weights(L, alpha, m.shape[0], _ptr(m), _ptr(w)), "rbe_ewald_weights")
    return w


# ---------------------------------------------------------------------- device calls (C names)

def rbe_plan_upload(plan, ws, stream=None):
    check(load().rbe_plan_upload(plan, _ptr(ws), _stream(stream)), "rbe_plan_upload")


def rbe_structure_factor(plan, x, y, z, q, m, rho, ws, stream=None):
    check(load().rbe_structure_factor(plan, _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(m), _ptr(rho),
                                      _ptr(ws), _stream(stream)), "rbe_structure_factor")


def rbe_kspace_force(plan, x, y, z, q, m, w, rho, F, U, ws, stream=None):
    check(load().rbe_kspace_force(plan, _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(m), _ptr(w), _ptr(rho),
                                  _ptr(F), _ptr(U), _ptr(ws), _stream(stream)), "rbe_kspace_force")


def rbe_evaluate(plan, seed, stream_base, step_counter, x, y, z, q, m, w, rho, F, U, ws, stream=None):
    check(load().rbe_evaluate(plan, seed, stream_base, _ptr(step_counter), _ptr(x), _ptr(y), _ptr(z), _ptr(q),
                              _ptr(m), _ptr(w), _ptr(rho), _ptr(F), _ptr(U), _ptr(ws), _stream(stream)),
          "rbe_evaluate")


def rbe_evaluate_static(plan, seed, stream_base, step_counter, x, y, z, q, m, w, rho, F, U, stream=None):
    check(load().rbe_evaluate_static(plan, seed, stream_base, _ptr(step_counter), _ptr(x), _ptr(y), _ptr(z),
                                     _ptr(q), _ptr(m), _ptr(w), _ptr(rho), _ptr(F), _ptr(U), _stream(stream)),
          "rbe_evaluate_static")


def rbe_kspace_virial(plan, m, w, rho, W, ws, stream=None):
    check(load().rbe_kspace_virial(plan, _ptr(m), _ptr(w), _ptr(rho), _ptr(W), _ptr(ws), _stream(stream)),
          "rbe_kspace_virial")


def rbe_kspace_vjp(plan, x, y, z, q, m, w, rho, gU, gF, gr, gq, ws, stream=None):
    check(load().rbe_kspace_vjp(plan, _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(m), _ptr(w), _ptr(rho),
                                _ptr(gU), _ptr(gF), _ptr(gr), _ptr(gq), _ptr(ws), _stream(stream)),
          "rbe_kspace_vjp")


def rbe_sample_k_device(plan, seed, stream_id, m, w, ws, stream=None):
    check(load().rbe_sample_k_device(plan, seed, stream_id, _ptr(m), _ptr(w), _ptr(ws), _stream(stream)),
          "rbe_sample_k_device")


# ---------------------------------------------------------------------- plan object

@dataclass
class Batch:
    sys_off: np.ndarray   # (B+1,) int64
    k_off: np.ndarray     # (B+1,) int64
    L: np.ndarray         # (B,) float64
    alpha: np.ndarray     # (B,) float64

    @staticmethod
    def single(n: int, p: int, L: float, alpha: float) -> "Batch":
        return Batch(np.array([0, n], dtype=np.int64), np.array([0, p], dtype=np.int64),
                     np.array([L], dtype=np.float64), np.array([alpha], dtype=np.float64))

    @staticmethod
    def from_sizes(ns, ps, Ls, alphas) -> "Batch":
        so = np.concatenate([[0], np.cumsum(np.asarray(ns, dtype=np.int64))]).astype(np.int64)
        ko = np.concatenate([[0], np.cumsum(np.asarray(ps, dtype=np.int64))]).astype(np.int64)
        return Batch(so, ko, np.asarray(Ls, dtype=np.float64), np.asarray(alphas, dtype=np.float64))

    @property
    def B(self) -> int:
        return int(self.L.shape[0])


class Plan:
    """A plan for a batch of systems plus its device workspace (a torch uint8 tensor)."""

    def __init__(self, batch: Batch, precision: str = "fp32_mixed", phase_mode: str = "auto",
                 device=None, tiles="auto"):
        """precision: "fp64", "fp32_mixed" (exact fixed-point phases, FP32 sin/cos) or
        "fp32" (FP32 phases, fewer operations, phase error growing with |m|).
        tiles: (rho_variant, force_variant[, rho_grid_cap[, occupancy_clamp]]), "auto"
        (the tuning cache, else the library defaults) or None (library defaults)."""
        self.lib = load()
        self.batch = batch
        self.precision = precision
        self.phase_mode = phase_mode
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.n_total = int(batch.sys_off[-1])
        self.p_total = int(batch.k_off[-1])
        self._arrays = [np.ascontiguousarray(a, dtype=t) for a, t in
                        ((batch.sys_off, np.int64), (batch.k_off, np.int64), (batch.L, np.float64),
                         (batch.alpha, np.float64))]
        desc = _lib.BatchDesc(batch.B, *[_ptr(a) for a in self._arrays])
        handle = ctypes.c_void_p()
        check(self.lib.rbe_plan_create(ctypes.byref(desc), PRECISIONS[precision], PHASE_MODES[phase_mode],
                                       ctypes.byref(handle)), "rbe_plan_create")
        self.handle = handle
        self._events = ()
        _live_plans.add(self)
        if isinstance(tiles, str) and tiles == "auto":
            from .tune import lookup
            tiles = lookup(precision, phase_mode, batch.B, self.n_total, self.p_total)
        if tiles is not None:
            check(self.lib.rbe_plan_set_tiles(self.handle, int(tiles[0]), int(tiles[1])), "rbe_plan_set_tiles")
            if len(tiles) > 2:
                check(self.lib.rbe_plan_set_grid_caps(self.handle, int(tiles[2]), 0), "rbe_plan_set_grid_caps")
            if len(tiles) > 3:
                check(self.lib.rbe_plan_set_occupancy_clamp(self.handle, int(tiles[3])), "rbe_plan_set_occupancy_clamp")
        self._alloc()

    def _alloc(self):
        nbytes = int(self.lib.rbe_plan_workspace_bytes(self.handle))
        # over-allocate by 256 bytes and slice to a 256-byte boundary
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + nbytes]
        rbe_plan_upload(self.handle, self.ws)

    def set_sampler(self, sampler: str = "exact", burn_in: int = 64):
        """Device sampler: "exact" (i.i.d. draws) or "metropolis" (the paper's procedure)."""
        code = {"exact": _lib.RBE_SAMPLER_EXACT, "metropolis": _lib.RBE_SAMPLER_METROPOLIS}[sampler]
        check(self.lib.rbe_plan_set_sampler(self.handle, code, int(burn_in)), "rbe_plan_set_sampler")

    def set_tiles(self, rho_variant: int, force_variant: int):
        check(self.lib.rbe_plan_set_tiles(self.handle, rho_variant, force_variant), "rbe_plan_set_tiles")
        rbe_plan_upload(self.handle, self.ws)

    def tune(self, x, y, z, q, m, w, reps: int = 5, stream=None):
        """Time every kernel variant on these inputs and keep the fastest (rbe_plan_tune)."""
        self._check_particles(x, y, z, q)
        self._check_k(m, w)
        rho = torch.empty((self.p_total, 2), dtype=torch.float64, device=self.device)
        F = torch.empty((3, self.n_total), dtype=self.force_dtype, device=self.device)
        U = torch.empty(self.batch.B, dtype=torch.float64, device=self.device)
        rv, fv, cap = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        rms, fms = ctypes.c_double(), ctypes.c_double()
        check(self.lib.rbe_plan_tune(self.handle, _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(m), _ptr(w),
                                     _ptr(rho), _ptr(F), _ptr(U), _ptr(self.ws), _stream(stream), reps,
                                     ctypes.byref(rv), ctypes.byref(fv), ctypes.byref(cap), ctypes.byref(rms),
                                     ctypes.byref(fms)),
              "rbe_plan_tune")
        return {"rho_variant": rv.value, "force_variant": fv.value, "rho_grid_cap": cap.value,
                "occupancy_clamp": self.tiles()[3], "rho_ms": rms.value, "force_ms": fms.value}

    def tiles(self):
        """(rho_variant, force_variant, rho_grid_cap, occupancy_clamp)."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.rbe_plan_get_tiles(self.handle, ctypes.byref(a), ctypes.byref(b)), "rbe_plan_get_tiles")
        c, d = ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.rbe_plan_get_grid_caps(self.handle, ctypes.byref(c), ctypes.byref(d)), "rbe_plan_get_grid_caps")
        e = ctypes.c_int32()
        check(self.lib.rbe_plan_get_occupancy_clamp(self.handle, ctypes.byref(e)), "rbe_plan_get_occupancy_clamp")
        return a.value, b.value, c.value, e.value

    def set_occupancy_clamp(self, on: bool):
        check(self.lib.rbe_plan_set_occupancy_clamp(self.handle, 1 if on else 0), "rbe_plan_set_occupancy_clamp")

    def num_variants(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.rbe_plan_num_variants(self.handle, ctypes.byref(a), ctypes.byref(b)), "rbe_plan_num_variants")
        return a.value, b.value

    def rho_variant_info(self, variant: int) -> dict:
        """Layout of a rho variant (rbe_plan_rho_variant_info); waves_per_block 1 is the k-lane layout."""
        v = [ctypes.c_int32() for _ in range(6)]
        check(self.lib.rbe_plan_rho_variant_info(self.handle, int(variant), *[ctypes.byref(x) for x in v]),
              "rbe_plan_rho_variant_info")
        return dict(zip(("particles_per_lane", "vectors_per_chunk", "vectors_per_item", "waves_per_block",
                         "particles_per_tile", "compensated"), (x.value for x in v)))

    @property
    def force_dtype(self):
        return torch.float64 if self.precision == "fp64" else torch.float32

    def close(self):
        """Release the plan (host memory) and drop the workspace; the plan is unusable afterwards."""
        h = getattr(self, "handle", None)
        if h is not None and h.value and not _released_all:
            self.lib.rbe_plan_destroy(h)
        self.handle = None
        self._events = ()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()

    # -- device calls (inputs: float64 x, y, z, q; int32 m (P_total, 3); float64 w)
    def _check_particles(self, x, y, z, q):
        for name, t in (("x", x), ("y", y), ("z", z), ("q", q)):
            _dev(t, torch.float64, name)
            if t.numel() != self.n_total:
                raise ValueError(f"{name} has {t.numel()} elements, plan expects {self.n_total}")

    def _check_k(self, m, w=None):
        _dev(m, torch.int32, "m")
        if m.numel() != 3 * self.p_total:
            raise ValueError(f"m has {m.numel()} elements, plan expects {3 * self.p_total}")
        if w is not None:
            _dev(w, torch.float64, "w")
            if w.numel() != self.p_total:
                raise ValueError(f"w has {w.numel()} elements, plan expects {self.p_total}")

    def structure_factor(self, x, y, z, q, m, rho=None, stream=None):
        self._check_particles(x, y, z, q)
        self._check_k(m)
        if rho is None:
            rho = torch.empty((self.p_total, 2), dtype=torch.float64, device=self.device)
        rbe_structure_factor(self.handle, x, y, z, q, m, rho, self.ws, stream)
        return rho

    def kspace_force(self, x, y, z, q, m, w, rho, F=None, U=None, stream=None):
        self._check_particles(x, y, z, q)
        self._check_k(m, w)
        if F is None:
            F = torch.empty((3, self.n_total), dtype=self.force_dtype, device=self.device)
        if U is None:
            U = torch.empty(self.batch.B, dtype=torch.float64, device=self.device)
        rbe_kspace_force(self.handle, x, y, z, q, m, w, rho, F, U, self.ws, stream)
        return F, U

    def forward(self, x, y, z, q, m, w, stream=None):
        rho = self.structure_factor(x, y, z, q, m, stream=stream)
        F, U = self.kspace_force(x, y, z, q, m, w, rho, stream=stream)
        return F, U, rho

    def kspace_virial(self, m, w, rho, W=None, stream=None):
        """Virial tensor per system, (B, 6) FP64: xx, yy, zz, xy, xz, yz."""
        self._check_k(m, w)
        _dev(rho, torch.float64, "rho")
        if W is None:
            W = torch.empty((self.batch.B, 6), dtype=torch.float64, device=self.device)
        _dev(W, torch.float64, "W")
        rbe_kspace_virial(self.handle, m, w, rho, W, self.ws, stream)
        return W

    def kspace_vjp(self, x, y, z, q, m, w, rho, gU, gF, gr=None, gq=None, stream=None):
        self._check_particles(x, y, z, q)
        self._check_k(m, w)
        _dev(gU, torch.float64, "gU")
        _dev(gF, self.force_dtype, "gF")
        if gr is None:
            gr = torch.empty((3, self.n_total), dtype=torch.float64, device=self.device)
        if gq is None:
            gq = torch.empty(self.n_total, dtype=torch.float64, device=self.device)
        _dev(gr, torch.float64, "gr")
        _dev(gq, torch.float64, "gq")
        rbe_kspace_vjp(self.handle, x, y, z, q, m, w, rho, gU, gF, gr, gq, self.ws, stream)
        return gr, gq

    def set_timing_events(self, rho_begin=None, rho_end=None, force_begin=None, force_end=None):
        """Record torch.cuda.Events (already recorded once, so their handles exist) around the kernels."""
        evs = (rho_begin, rho_end, force_begin, force_end)
        h = [ctypes.c_void_p(e.cuda_event) if e is not None else ctypes.c_void_p(0) for e in evs]
        check(self.lib.rbe_plan_set_timing_events(self.handle, *h), "rbe_plan_set_timing_events")
        # the plan records into these events on later calls: keep them alive while set
        self._events = tuple(e for e in evs if e is not None)

    def set_grid_caps(self, rho_cap: int, force_cap: int):
        check(self.lib.rbe_plan_set_grid_caps(self.handle, rho_cap, force_cap), "rbe_plan_set_grid_caps")

    def evaluate(self, x, y, z, q, seed: int, stream_base: int = 0, step_counter=None, out=None, stream=None):
        """One whole evaluation (device sampling, rho, force and energy) enqueued without
        synchronisation.  out: (m, w, rho, F, U) buffers to reuse, else new ones.
        Returns (m, w, rho, F, U)."""
        self._check_particles(x, y, z, q)
        if out is None:
            dev = self.device
            out = (torch.empty((self.p_total, 3), dtype=torch.int32, device=dev),
                   torch.empty(self.p_total, dtype=torch.float64, device=dev),
                   torch.empty((self.p_total, 2), dtype=torch.float64, device=dev),
                   torch.empty((3, self.n_total), dtype=self.force_dtype, device=dev),
                   torch.empty(self.batch.B, dtype=torch.float64, device=dev))
        m, w, rho, F, U = out
        _dev(m, torch.int32, "m")
        _dev(w, torch.float64, "w")
        _dev(rho, torch.float64, "rho")
        _dev(F, self.force_dtype, "F")
        _dev(U, torch.float64, "U")
        if step_counter is not None:
            _dev(step_counter, torch.int64, "step_counter")
        rbe_evaluate(self.handle, seed, stream_base, step_counter, x, y, z, q, m, w, rho, F, U, self.ws, stream)
        return out

    def graph(self, x, y, z, q, seed: int, stream_base: int = 0, step_counter=None):
        """A captured evaluation (sample -> rho -> force) of this plan; see EvalGraph."""
        return EvalGraph(self, x, y, z, q, seed, stream_base, step_counter)

    def sample_k_device(self, seed: int, stream_id: int, m=None, w=None, stream=None):
        if m is None:
            m = torch.empty((self.p_total, 3), dtype=torch.int32, device=self.device)
        if w is None:
            w = torch.empty(self.p_total, dtype=torch.float64, device=self.device)
        rbe_sample_k_device(self.handle, seed, stream_id, m, w, self.ws, stream)
        return m, w


class EvalGraph:
    """One RBE evaluation captured into a HIP graph (rbe_graph_create / rbe_graph_launch).

    Owns its output buffers: m, w, rho, F, U.  With a step counter (a one-element
    uint64 device tensor) every replay draws new wave vectors.
    """

    def __init__(self, plan: Plan, x, y, z, q, seed, stream_base=0, step_counter=None):
        plan._check_particles(x, y, z, q)
        self.plan = plan
        dev = plan.device
        self.inputs = (x, y, z, q)
        self.m = torch.zeros((plan.p_total, 3), dtype=torch.int32, device=dev)
        self.w = torch.zeros(plan.p_total, dtype=torch.float64, device=dev)
        self.rho = torch.zeros((plan.p_total, 2), dtype=torch.float64, device=dev)
        self.F = torch.zeros((3, plan.n_total), dtype=plan.force_dtype, device=dev)
        self.U = torch.zeros(plan.batch.B, dtype=torch.float64, device=dev)
        self.counter = step_counter
        torch.cuda.synchronize()
        handle = ctypes.c_void_p()
        check(plan.lib.rbe_graph_create(plan.handle, seed, stream_base, _ptr(step_counter), _ptr(x), _ptr(y),
                                        _ptr(z), _ptr(q), _ptr(self.m), _ptr(self.w), _ptr(self.rho),
                                        _ptr(self.F), _ptr(self.U), _ptr(plan.ws), ctypes.byref(handle)),
              "rbe_graph_create")
        self.handle = handle
        _live_graphs.add(self)

    def launch(self, stream=None):
        if self.handle is None:
            raise RuntimeError("the graph was closed")
        check(self.plan.lib.rbe_graph_launch(self.handle, _stream(stream)), "rbe_graph_launch")

    def close(self):
        """Destroy the HIP graph; waits for the device first, since a replay may still run."""
        h = getattr(self, "handle", None)
        if h is not None and h.value and not _released_all:
            torch.cuda.synchronize(self.plan.device)
            self.plan.lib.rbe_graph_destroy(h)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------- RBL short-range force

def rbl_short_force(plan, x, y, z, q, eps, sig, seed, step, F, ns, ws, stream=None):
    check(load().rbl_short_force(plan, _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(eps), _ptr(sig), int(seed),
                                 int(step), _ptr(F), _ptr(ns), _ptr(ws), _stream(stream)), "rbl_short_force")


class RBLPlan:
    """A random batch list plan (rbl_plan_create) and its device workspace."""

    def __init__(self, n: int, L: float, alpha: float, r_c: float, r_s: float, p: int, device=None):
        self.lib = load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.n = int(n)
        prm = _lib.RBLParams(int(n), float(L), float(alpha), float(r_c), float(r_s), int(p))
        handle = ctypes.c_void_p()
        check(self.lib.rbl_plan_create(ctypes.byref(prm), ctypes.byref(handle)), "rbl_plan_create")
        self.handle = handle
        _live_plans.add(self)
        nbytes = int(self.lib.rbl_plan_workspace_bytes(self.handle))
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + nbytes]

    def grid(self):
        v = [ctypes.c_int32() for _ in range(3)]
        check(self.lib.rbl_plan_grid(self.handle, *[ctypes.byref(a) for a in v]), "rbl_plan_grid")
        return tuple(a.value for a in v)

    def set_timing_events(self, select_begin=None, select_end=None, pair_begin=None, pair_end=None):
        """Record torch.cuda.Events (already recorded once, so their handles exist) around the
        selection and pair kernels of later short_force calls."""
        evs = (select_begin, select_end, pair_begin, pair_end)
        h = [ctypes.c_void_p(e.cuda_event) if e is not None else ctypes.c_void_p(0) for e in evs]
        check(self.lib.rbl_plan_set_timing_events(self.handle, *h), "rbl_plan_set_timing_events")
        self._events = tuple(e for e in evs if e is not None)

    def capacity(self):
        """(pair slots per particle, stencil positions per cell) of the fast path."""
        v = [ctypes.c_int32() for _ in range(2)]
        check(self.lib.rbl_plan_capacity(self.handle, *[ctypes.byref(a) for a in v]), "rbl_plan_capacity")
        return tuple(a.value for a in v)

    def short_force(self, x, y, z, q, eps, sig, seed: int, step: int, F=None, ns=None, stream=None):
        """(F (3, N) FP64, N_s (N,) int32) for one evaluation; enqueued without synchronisation."""
        for name, t in (("x", x), ("y", y), ("z", z), ("q", q), ("eps", eps), ("sig", sig)):
            _dev(t, torch.float64, name)
            if t.numel() != self.n:
                raise ValueError(f"{name} has {t.numel()} elements, the plan {self.n}")
        if F is None:
            F = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        if ns is None:
            ns = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _dev(F, torch.float64, "F")
        _dev(ns, torch.int32, "ns")
        rbl_short_force(self.handle, x, y, z, q, eps, sig, seed, step, F, ns, self.ws, stream)
        return F, ns

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and not _released_all:
            self.lib.rbl_plan_destroy(h)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
