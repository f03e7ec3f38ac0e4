"""ctypes loader for librbe.so (the gfx950 HIP library).

torch is imported first so that the HIP runtime torch ships is the one the
library binds to (both carry the soname libamdhip64.so.7); torch tensors and
streams can then be passed straight through.  There is no fallback: if the
library is missing the import fails with instructions to build it.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before librbe.so, see module docstring)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librbe.so")

RBE_OK, RBE_EINVAL, RBE_ENODEV, RBE_EHIP, RBE_EWORKSPACE, RBE_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RBE_FP64, RBE_FP32_MIXED, RBE_FP32 = 0, 1, 2
RBE_PHASE_AUTO, RBE_PHASE_RECOMPUTE, RBE_PHASE_CACHED = 0, 1, 2
RBE_SAMPLER_EXACT, RBE_SAMPLER_METROPOLIS = 0, 1

# name -> (restype, argtypes); every symbol that include/rbe.h and include/rbl.h declare
_VP, _I32, _U64, _D, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
_ST = ctypes.c_int
SIGNATURES = {
    "rbe_sample_k": (_ST, [_U64, _U64, _D, _D, _I32, _VP, _VP, _VP]),
    "rbe_sample_k_metropolis": (_ST, [_U64, _U64, _D, _D, _I32, _I32, _VP, _VP, _VP]),
    "rbe_plan_set_sampler": (_ST, [_VP, _I32, _I32]),
    "rbe_normalization": (_ST, [_D, _D, _VP]),
    "rbe_ewald_weights": (_ST, [_D, _D, _I32, _VP, _VP]),
    "rbe_plan_create": (_ST, [_VP, _I32, _I32, _VP]),
    "rbe_plan_workspace_bytes": (_SZ, [_VP]),
    "rbe_plan_set_tiles": (_ST, [_VP, _I32, _I32]),
    "rbe_plan_num_variants": (_ST, [_VP, _VP, _VP]),
    "rbe_plan_rho_variant_info": (_ST, [_VP, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP, _VP]),
    "rbe_plan_get_tiles": (_ST, [_VP, _VP, _VP]),
    "rbe_plan_destroy": (None, [_VP]),
    "rbe_plan_upload": (_ST, [_VP, _VP, _VP]),
    "rbe_structure_factor": (_ST, [_VP] * 9),
    "rbe_kspace_force": (_ST, [_VP] * 12),
    "rbe_kspace_vjp": (_ST, [_VP] * 14),
    "rbe_sample_k_device": (_ST, [_VP, _U64, _U64, _VP, _VP, _VP, _VP]),
    "rbe_plan_tune": (_ST, [_VP] * 12 + [_I32, _VP, _VP, _VP, _VP, _VP]),
    "rbe_plan_get_grid_caps": (_ST, [_VP, _VP, _VP]),
    "rbe_plan_set_occupancy_clamp": (_ST, [_VP, _I32]),
    "rbe_plan_get_occupancy_clamp": (_ST, [_VP, _VP]),
    "rbe_plan_set_grid_caps": (_ST, [_VP, _I32, _I32]),
    "rbe_plan_set_timing_events": (_ST, [_VP] * 5),
    "rbe_evaluate": (_ST, [_VP, _U64, _U64] + [_VP] * 12),
    "rbe_kspace_virial": (_ST, [_VP] * 7),
    "rbe_evaluate_static": (_ST, [_VP, _U64, _U64] + [_VP] * 11),
    "rbe_graph_create": (_ST, [_VP, _U64, _U64] + [_VP] * 12),
    "rbe_graph_launch": (_ST, [_VP, _VP]),
    "rbe_graph_destroy": (None, [_VP]),
    "rbl_plan_create": (_ST, [_VP, _VP]),
    "rbl_plan_workspace_bytes": (_SZ, [_VP]),
    "rbl_plan_grid": (_ST, [_VP, _VP, _VP, _VP]),
    "rbl_plan_capacity": (_ST, [_VP, _VP, _VP]),
    "rbl_plan_set_timing_events": (_ST, [_VP] * 5),
    "rbl_plan_destroy": (None, [_VP]),
    "rbl_short_force": (_ST, [_VP] * 7 + [_U64, _U64] + [_VP] * 4),
    "rbe_status_string": (ctypes.c_char_p, [_ST]),
    "rbe_last_error": (ctypes.c_char_p, []),
    "rbe_abi_version": (_I32, []),
}



class RBLParams(ctypes.Structure):
    """rbl_params: N, L, alpha, r_c, r_s, p."""
    _fields_ = [("N", ctypes.c_int64), ("L", ctypes.c_double), ("alpha", ctypes.c_double),
                ("r_c", ctypes.c_double), ("r_s", ctypes.c_double), ("p", ctypes.c_int32)]


class BatchDesc(ctypes.Structure):
    """rbe_batch_desc: B and pointers to the host offset / box arrays."""
    _fields_ = [("B", ctypes.c_int32), ("sys_off", _VP), ("k_off", _VP), ("L", _VP), ("alpha", _VP)]


_lib = None


class RBEError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where} failed with status {status}: {detail}")
        self.status = status


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2407_09315_amd.build` "
                              "(or __graft_entry__.build()) first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str) -> None:
    if status != RBE_OK:
        lib = load()
        detail = lib.rbe_last_error().decode(errors="replace")
        raise RBEError(status, where, detail or lib.rbe_status_string(status).decode())
