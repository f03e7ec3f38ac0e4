"""Shared helpers for the GPU parity tests: error measures and device transfer.

Error measures (the targets do not define them; these are the readings used):
  force  : relative RMS over all particles, sqrt(sum |dF|^2 / sum |F_ref|^2), and the
           per-particle measure max_i |dF_i| / RMS_i |F_ref_i| (3-vector norms), which
           catches a few wrong particles that the global norm would average away
  rho    : max_l |d rho_l| / sqrt(sum_i q_i^2)
  energy : |dU| / |U_ref|
  VJP    : the same two measures for dL/dr (3-vectors) and dL/dq (scalars)
"""
import numpy as np
import torch

FP64_TOL = 1e-12
FP32_TOL = 1e-5
# bounds of the per-particle measure: a particle wrong by 1e-3 of its own force (FP32) or
# 1e-9 (FP64) fails them at any system size
FP64_MAX_TOL = 1e-11
FP32_MAX_TOL = 1e-4
MAX_TOL = {"fp64": FP64_MAX_TOL, "fp32_mixed": FP32_MAX_TOL, "fp32": FP32_MAX_TOL}


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev())


def particles(s):
    return [to_dev(a) for a in (s.x, s.y, s.z, s.q)]


def force_err(F, F_ref):
    F = np.asarray(F, dtype=np.float64)
    return float(np.sqrt(np.sum((F - F_ref) ** 2) / np.sum(F_ref ** 2)))


def max_err(F, F_ref):
    """max_i |dF_i| / RMS_i |F_ref_i|: columns of (3, N) arrays are particles' vectors,
    elements of 1-D arrays are scalars."""
    F = np.asarray(F, dtype=np.float64)
    F_ref = np.asarray(F_ref, dtype=np.float64)
    if F_ref.ndim == 1:
        F, F_ref = F[None, :], F_ref[None, :]
    d = np.sqrt(np.sum((F - F_ref) ** 2, axis=0))
    rms = np.sqrt(np.mean(np.sum(F_ref ** 2, axis=0)))
    return float(d.max() / rms) if d.size else 0.0


def rho_err(rho, rho_ref, q):
    r = np.asarray(rho, dtype=np.float64)
    rc = r[:, 0] + 1j * r[:, 1]
    return float(np.max(np.abs(rc - rho_ref)) / np.sqrt(np.sum(np.asarray(q) ** 2)))


def rel(a, b):
    return abs(a - b) / abs(b)


def note(msg):
    print(msg, flush=True)
