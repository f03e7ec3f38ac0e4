"""CPU oracle for the RBE k-space path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never links,
loads or calls it, and it imports nothing from the product package.

Contents:
  * ``rbe_oracle.c`` -- plain FP64 definitions of rho(k), the RBE / Ewald
    k-space force, energy and virial tensor, their vector-Jacobian product,
    and the real-space + self Ewald energy;
  * ``rbl_oracle.c`` -- the random batch list (RBL) short-range force (core
    sum, shell batch, momentum correction) by brute force over all pairs, and
    the truncated short-range energy; both compiled with gcc into
    ``liboracle.so``;
  * ``sampler.py`` -- the exact i.i.d. wave-vector sampler, Philox4x64-10 and
    the normalisation S, in plain Python;
  * this module -- numpy wrappers.

Parity status: every function here is pinned by the ``-m "not gpu"`` tests
against values that the paper or the mathematics fixes (closed forms,
invariants, the rock-salt Madelung constant, an FFT of gridded charges,
finite differences, independent autograd, a library Philox, a chi-square
test against the exact pmf; the virial against strain finite differences of
a separate box-matrix energy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import sampler  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "rbe_oracle.c"), os.path.join(_HERE, "rbl_oracle.c")]
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, *_SRCS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
        P = ctypes.c_void_p
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_rho.argtypes = [i64, P, P, P, P, i64, P, d, P]
        lib.oracle_force_from_rho.argtypes = [i64, P, P, P, P, i64, P, P, d, P, P, P]
        lib.oracle_force_energy.argtypes = [i64, P, P, P, P, i64, P, P, d, P, P, P]
        lib.oracle_force_subset.argtypes = [i64, P, P, P, P, i64, P, P, d, P, i64, P, P]
        lib.oracle_vjp.argtypes = [i64, P, P, P, P, i64, P, P, d, d, P, P, P, P]
        lib.oracle_ewald_real_self.argtypes = [i64, P, P, P, P, d, d, i32, P, P]
        lib.oracle_virial.argtypes = [i64, P, P, d, d, P, P]
        lib.oracle_rbl_short_force.restype = ctypes.c_int
        lib.oracle_rbl_short_force.argtypes = [i64, P, P, P, P, P, P, d, d, d, d, i32, P, P, P]
        lib.oracle_rbl_raw_subset.restype = ctypes.c_int
        lib.oracle_rbl_raw_subset.argtypes = [i64, P, P, P, P, P, P, d, d, d, d, i32, i64, P, P, P, P]
        lib.oracle_short_energy.restype = d
        lib.oracle_short_energy.argtypes = [i64, P, P, P, P, P, P, d, d, d]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Run later oracle calls on n OpenMP threads (timing only; results do not change)."""
    _load().oracle_set_num_threads(int(n))


def rho(x, y, z, q, m, L):
    """Structure factor rho(k_l) for every row of m; returns complex128 (P,)."""
    x, y, z, q = map(_f64, (x, y, z, q))
    m = np.ascontiguousarray(m, dtype=np.int32)
    out = np.zeros(2 * m.shape[0])
    _load().oracle_rho(q.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(q), m.shape[0], _ptr(m),
                       float(L), _ptr(out))
    return out[0::2] + 1j * out[1::2]


def force_energy(x, y, z, q, m, w, L):
    """(F (3, N), U, rho (P,) complex) for weights w (S/P for RBE, exp(-k^2/4a) for Ewald)."""
    x, y, z, q, w = map(_f64, (x, y, z, q, w))
    m = np.ascontiguousarray(m, dtype=np.int32)
    n, p = q.shape[0], m.shape[0]
    F = np.zeros(3 * n)
    U = np.zeros(1)
    r = np.zeros(2 * p)
    _load().oracle_force_energy(n, _ptr(x), _ptr(y), _ptr(z), _ptr(q), p, _ptr(m), _ptr(w),
                                float(L), _ptr(r), _ptr(F), _ptr(U))
    return F.reshape(3, n), float(U[0]), r[0::2] + 1j * r[1::2]


def force_subset(x, y, z, q, m, w, L, rho_c, sel):
    """Forces (3, len(sel)) of the selected particles, from a given complex rho."""
    x, y, z, q, w = map(_f64, (x, y, z, q, w))
    m = np.ascontiguousarray(m, dtype=np.int32)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    r = np.empty(2 * m.shape[0])
    r[0::2], r[1::2] = np.real(rho_c), np.imag(rho_c)
    out = np.zeros(3 * sel.shape[0])
    _load().oracle_force_subset(q.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(q), m.shape[0],
                                _ptr(m), _ptr(w), float(L), _ptr(r), sel.shape[0], _ptr(sel),
                                _ptr(out))
    return out.reshape(3, sel.shape[0])


def vjp(x, y, z, q, m, w, L, gU, GF):
    """(dL/dr (3, N), dL/dq (N,)) for upstream gU (scalar) on U and GF (3, N) on F."""
    x, y, z, q, w = map(_f64, (x, y, z, q, w))
    GF = _f64(GF).reshape(-1)
    m = np.ascontiguousarray(m, dtype=np.int32)
    n, p = q.shape[0], m.shape[0]
    gr = np.zeros(3 * n)
    gq = np.zeros(n)
    work = np.zeros(6 * p)
    _load().oracle_vjp(n, _ptr(x), _ptr(y), _ptr(z), _ptr(q), p, _ptr(m), _ptr(w), float(L),
                       float(gU), _ptr(GF), _ptr(gr), _ptr(gq), _ptr(work))
    return gr.reshape(3, n), gq


def ewald_real_self(x, y, z, q, L, alpha, nmax):
    """(U_real, U_self) of the Ewald split energy."""
    x, y, z, q = map(_f64, (x, y, z, q))
    ur, us = np.zeros(1), np.zeros(1)
    _load().oracle_ewald_real_self(q.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(q), float(L),
                                   float(alpha), int(nmax), _ptr(ur), _ptr(us))
    return float(ur[0]), float(us[0])


def virial(m, w, L, alpha, rho_c):
    """k-space virial tensor (xx, yy, zz, xy, xz, yz) from a complex rho (P,)."""
    m = np.ascontiguousarray(m, dtype=np.int32)
    w = _f64(w)
    rc = np.asarray(rho_c)
    rho = np.ascontiguousarray(np.stack([rc.real, rc.imag], axis=1).reshape(-1), dtype=np.float64)
    W = np.zeros(6)
    _load().oracle_virial(m.shape[0], _ptr(m), _ptr(w), float(L), float(alpha), _ptr(rho), _ptr(W))
    return W


def rbl_offsets(seed: int, step: int, n, ) -> np.ndarray:
    """Batch offsets u_i in [0, 1) of the RBL shell batches: word 0 of Philox4x64-10 with
    key (seed, step) and counter (i, 0, 3, 0), top 53 bits.  n: a count (particles 0..n-1)
    or an array of particle indices."""
    idx = range(n) if isinstance(n, (int, np.integer)) else [int(i) for i in n]
    return np.array([(sampler.philox4x64_10((i, 0, 3, 0), (seed, step))[0] >> 11) * 2.0 ** -53 for i in idx],
                    dtype=np.float64)


def rbl_raw_subset(x, y, z, q, eps, sig, L, alpha, rc, rs, p, sel, u_sel):
    """Raw RBL forces (before the momentum correction) of the particles sel: ((3, m), N_s (m,))."""
    x, y, z, q, eps, sig, u_sel = map(_f64, (x, y, z, q, eps, sig, u_sel))
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    m = sel.shape[0]
    out = np.zeros(3 * m)
    ns = np.zeros(m, dtype=np.int64)
    st = _load().oracle_rbl_raw_subset(q.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(eps), _ptr(sig),
                                       float(L), float(alpha), float(rc), float(rs), int(p), m, _ptr(sel),
                                       _ptr(u_sel), _ptr(out), _ptr(ns))
    if st != 0:
        raise ValueError(f"oracle_rbl_raw_subset failed ({st})")
    return out.reshape(3, m), ns


def rbl_short_force(x, y, z, q, eps, sig, L, alpha, rc, rs, p, u):
    """RBL short-range force (F (3, N), N_s (N,)) with batch offsets u (N,)."""
    x, y, z, q, eps, sig, u = map(_f64, (x, y, z, q, eps, sig, u))
    n = q.shape[0]
    F = np.zeros(3 * n)
    ns = np.zeros(n, dtype=np.int64)
    st = _load().oracle_rbl_short_force(n, _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(eps), _ptr(sig), float(L),
                                        float(alpha), float(rc), float(rs), int(p), _ptr(u), _ptr(F), _ptr(ns))
    if st != 0:
        raise ValueError(f"oracle_rbl_short_force failed ({st}): need 0 < rc <= rs < L/2 and p >= 1")
    return F.reshape(3, n), ns


def short_energy(x, y, z, q, eps, sig, L, alpha, rs):
    """Short-range energy (LJ + real-space Coulomb) of every pair inside rs."""
    x, y, z, q, eps, sig = map(_f64, (x, y, z, q, eps, sig))
    return float(_load().oracle_short_energy(q.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(q), _ptr(eps),
                                             _ptr(sig), float(L), float(alpha), float(rs)))
