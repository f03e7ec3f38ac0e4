"""Shared helpers for the GPU parity tests: error measures and device transfer.

Error measures (the targets do not define them; these are the readings used):
  force  : relative RMS over all particles, sqrt(sum |dF|^2 / sum |F_ref|^2)
  rho    : max_l |d rho_l| / sqrt(sum_i q_i^2)
  energy : |dU| / |U_ref|
"""
import numpy as np
import torch

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev())


def particles(s):
    return [to_dev(a) for a in (s.x, s.y, s.z, s.q)]


def force_err(F, F_ref):
    F = np.asarray(F, dtype=np.float64)
    return float(np.sqrt(np.sum((F - F_ref) ** 2) / np.sum(F_ref ** 2)))


def rho_err(rho, rho_ref, q):
    r = np.asarray(rho, dtype=np.float64)
    rc = r[:, 0] + 1j * r[:, 1]
    return float(np.max(np.abs(rc - rho_ref)) / np.sqrt(np.sum(np.asarray(q) ** 2)))


def rel(a, b):
    return abs(a - b) / abs(b)


def note(msg):
    print(msg, flush=True)
