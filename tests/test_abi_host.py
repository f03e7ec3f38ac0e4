"""Host-side checks of the C ABI (no GPU needed).

  * librbe.so loads and exports every function include/rbe.h declares;
  * the host wave-vector sampler equals the oracle's sampler bit for bit
    (both implement Philox4x64-10 and the FP64 inverse CDF independently);
  * S and the Ewald weights agree with the oracle;
  * argument validation returns RBE_EINVAL / RBE_EUNSUPPORTED before any launch;
  * without a GPU, device calls report RBE_ENODEV.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest
import torch

import oracle
from paper_2407_09315_amd import _lib, rbe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _headers():
    return "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("rbe.h", "rbl.h"))


def _declared_functions():
    src = _headers()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rb[el]_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"
    assert lib.rbe_abi_version() == 3


_CTYPE_OF = {"int32_t": ctypes.c_int32, "uint64_t": ctypes.c_uint64, "double": ctypes.c_double,
             "size_t": ctypes.c_size_t, "rbe_status": ctypes.c_int}


def _prototypes():
    """name -> (return C type, [parameter C types]) of every function rbe.h and rbl.h declare."""
    src = _headers()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for ret, name, params in re.findall(r"([A-Za-z_][\w \*]*?)\b(rb[el]_[a-z0-9_]+)\s*\(([^)]*)\)\s*;", src):
        ps = [p.strip() for p in params.split(",") if p.strip() and p.strip() != "void"]
        out[name] = (ret.strip(), ps)
    return out


def _ctype(decl: str, is_return: bool = False):
    if "*" in decl:
        return ctypes.c_char_p if (is_return and "char" in decl) else ctypes.c_void_p
    base = decl.replace("const", "").split()[0]
    if base == "void":
        return None
    return _CTYPE_OF[base]


def test_binding_signatures_match_header():
    """Every ctypes signature of the binding has the header's parameter count and kinds."""
    protos = _prototypes()
    assert set(protos) == set(_lib.SIGNATURES), set(protos) ^ set(_lib.SIGNATURES)
    for name, (ret, params) in protos.items():
        res, args = _lib.SIGNATURES[name]
        assert _ctype(ret, True) == res, (name, ret, res)
        assert len(args) == len(params), (name, params, args)
        for p, a in zip(params, args):
            assert _ctype(p) == a, (name, p, a)
    # the VJP writes FP64 gradients in every precision
    assert protos["rbe_kspace_vjp"][1][10].startswith("double") and protos["rbe_kspace_vjp"][1][11].startswith("double")
    assert protos["rbe_plan_create"][1][0].startswith("const rbe_batch_desc")


@pytest.mark.parametrize("seed,stream,L,alpha,P", [
    (2001, 0, 31.0, 0.1, 100),
    (2002, 5, 144.1289, 0.08, 100),
    (2003, 1, 217.0535, 0.06, 200),
    (2004, 0, 467.6275, 0.06, 100),
    (7, 2 ** 63 + 3, 2.0, 1.5, 300),        # tiny box: many rejections of m = 0
    (2 ** 64 - 1, 0, 10.0, 0.362, 100),
])
def test_host_sampler_bit_exact_vs_oracle(seed, stream, L, alpha, P):
    m, w, S = rbe.rbe_sample_k(seed, stream, L, alpha, P)
    m_ref, S_ref = oracle.sampler.sample_k(seed, stream, L, alpha, P)
    assert np.array_equal(m, m_ref)
    assert abs(S / S_ref - 1) < 1e-14
    assert np.all(w == S / P)


def test_normalization_and_ewald_weights():
    for L, alpha in [(31.0, 0.1), (2.0, 1.5), (66.9, 0.048)]:
        assert abs(rbe.rbe_normalization(L, alpha) / oracle.sampler.normalization_S(L, alpha) - 1) < 1e-14
    m = oracle.sampler.all_vectors(4)
    w = rbe.rbe_ewald_weights(10.0, 0.362, m)
    assert np.allclose(w, oracle.sampler.ewald_weights(m, 10.0, 0.362), rtol=1e-14, atol=0)


def _create(B, so, ko, L, a, prec=0, mode=0):
    lib = _lib.load()
    h = ctypes.c_void_p()
    arrs = [np.ascontiguousarray(v) for v in (np.asarray(so, np.int64), np.asarray(ko, np.int64),
                                              np.asarray(L, np.float64), np.asarray(a, np.float64))]
    desc = _lib.BatchDesc(B, *[rbe._ptr(v) for v in arrs])
    st = lib.rbe_plan_create(ctypes.byref(desc), prec, mode, ctypes.byref(h))
    if st != 0:
        assert not h.value   # *out is NULL on failure
    return st, h


def test_plan_validation():
    lib = _lib.load()
    ok, h = _create(1, [0, 10], [0, 5], [3.0], [1.0])
    assert ok == 0 and h.value
    assert lib.rbe_plan_workspace_bytes(h) % 256 == 0
    lib.rbe_plan_destroy(h)
    bad = [
        (0, [0], [0], [], []),
        (1, [0, 10], [0, 5], [-3.0], [1.0]),
        (1, [0, 10], [0, 5], [3.0], [0.0]),
        (1, [0, 10], [0, 5], [float("nan")], [1.0]),
        (2, [0, 10, 5], [0, 5, 6], [3.0, 3.0], [1.0, 1.0]),
        (1, [1, 10], [0, 5], [3.0], [1.0]),
    ]
    for args in bad:
        st, _ = _create(*args)
        assert st == _lib.RBE_EINVAL, args
    st, _ = _create(1, [0, 10], [0, 5], [3.0], [1.0], prec=7)
    assert st == _lib.RBE_EINVAL
    h = ctypes.c_void_p()
    assert lib.rbe_plan_create(None, 0, 0, ctypes.byref(h)) == _lib.RBE_EINVAL and not h.value
    null_arrays = _lib.BatchDesc(1, None, None, None, None)
    assert lib.rbe_plan_create(ctypes.byref(null_arrays), 0, 0, ctypes.byref(h)) == _lib.RBE_EINVAL
    st, _ = _create(1, [0, 10], [0, 5], [3.0], [1.0], prec=0, mode=2)
    assert st == _lib.RBE_EUNSUPPORTED
    # the phase cache exists for the fixed-point FP32 phases only
    st, _ = _create(1, [0, 10], [0, 5], [3.0], [1.0], prec=_lib.RBE_FP32, mode=2)
    assert st == _lib.RBE_EUNSUPPORTED
    for prec in (_lib.RBE_FP64, _lib.RBE_FP32_MIXED, _lib.RBE_FP32):
        st, h = _create(1, [0, 10], [0, 5], [3.0], [1.0], prec=prec)
        assert st == 0
        lib.rbe_plan_destroy(h)


def test_rho_variant_info():
    """Every rho variant reports a layout the kernels implement; out-of-range indices are refused."""
    lib = _lib.load()
    for prec in (_lib.RBE_FP64, _lib.RBE_FP32_MIXED):
        st, h = _create(1, [0, 10], [0, 5], [3.0], [1.0], prec=prec)
        assert st == 0
        nr, nf = ctypes.c_int32(), ctypes.c_int32()
        assert lib.rbe_plan_num_variants(h, ctypes.byref(nr), ctypes.byref(nf)) == 0
        v = [ctypes.c_int32() for _ in range(6)]
        n_comp = 0
        for r in range(nr.value):
            assert lib.rbe_plan_rho_variant_info(h, r, *[ctypes.byref(x) for x in v]) == 0
            npl, kc, krange, wpb, tile, comp = (x.value for x in v)
            assert comp in (0, 1) and (comp == 0 or wpb == 1)
            n_comp += comp
            assert wpb in (1, 4, 16) and npl in (4, 8, 16) and 1 <= kc <= krange
            if wpb == 1:
                assert krange == 21 * kc   # 3 x 21 lanes, kc vectors each
                # 4 waves, each a whole number of steps over its 3 particle groups
                assert tile % 12 == 0 or tile == 64 * npl
                assert tile <= 64 * npl
            else:
                assert tile == 64 * npl
        # one compensated variant in the FP32 forms; FP64 sums need none
        assert n_comp == (0 if prec == _lib.RBE_FP64 else 1)
        for bad in (-1, nr.value):
            assert lib.rbe_plan_rho_variant_info(h, bad, *[ctypes.byref(x) for x in v]) == _lib.RBE_EINVAL
        assert lib.rbe_plan_rho_variant_info(h, 0, None, None, None, None, None, None) == _lib.RBE_EINVAL
        lib.rbe_plan_destroy(h)


def test_fp32_phase_box_guard():
    """RBE_FP32 phases are refused once the spread of sampled m, L sqrt(2 alpha) / (2 pi), exceeds 16."""
    lib = _lib.load()
    ok = [(217.0534689782871, 0.06), (144.1289350602584, 0.08)]     # 1M electrolyte, 300k water
    bad = [(467.627523158581, 0.06), (2 * np.pi * 16.01 / np.sqrt(0.2), 0.1)]
    for L, a in ok:
        st, h = _create(1, [0, 10], [0, 5], [L], [a], prec=_lib.RBE_FP32)
        assert st == 0, (L, a)
        lib.rbe_plan_destroy(h)
    for L, a in bad:
        st, _ = _create(1, [0, 10], [0, 5], [L], [a], prec=_lib.RBE_FP32)
        assert st == _lib.RBE_EUNSUPPORTED, (L, a)
        assert b"RBE_FP32_MIXED" in lib.rbe_last_error()
        st, h = _create(1, [0, 10], [0, 5], [L], [a], prec=_lib.RBE_FP32_MIXED)
        assert st == 0
        lib.rbe_plan_destroy(h)
    assert lib.rbe_sample_k(1, 0, -1.0, 0.1, 4, None, None, None) == _lib.RBE_EINVAL
    assert b"L and alpha" in lib.rbe_last_error()


def test_workspace_checks_and_nodev():
    lib = _lib.load()
    st, h = _create(1, [0, 10], [0, 5], [3.0], [1.0])
    assert st == 0
    assert lib.rbe_structure_factor(h, None, None, None, None, None, None, None, None) == _lib.RBE_EWORKSPACE
    assert lib.rbe_plan_upload(h, ctypes.c_void_p(1024 + 8), None) == _lib.RBE_EWORKSPACE
    if not torch.cuda.is_available():
        assert lib.rbe_plan_upload(h, ctypes.c_void_p(1024), None) == _lib.RBE_ENODEV
    lib.rbe_plan_destroy(h)


@pytest.mark.parametrize("seed,stream,L,alpha,P,burn_in", [
    (2001, 0, 31.0, 0.1, 100, 64),
    (2003, 7, 217.0535, 0.06, 50, 64),
    (2004, 1, 467.6275, 0.06, 30, 40),
    (7, 2 ** 63 + 3, 2.0, 1.5, 60, 64),      # tiny box: most proposals rejected
    (2 ** 64 - 1, 5, 10.0, 0.362, 40, 0),   # no step: every chain at its start
])
def test_host_metropolis_bit_exact_vs_oracle(seed, stream, L, alpha, P, burn_in):
    m, w, S = rbe.rbe_sample_k_metropolis(seed, stream, L, alpha, P, burn_in)
    m_ref, S_ref = oracle.sampler.metropolis_k(seed, stream, L, alpha, P, burn_in)
    assert np.array_equal(m, m_ref)
    assert not np.any(np.all(m == 0, axis=1))
    assert abs(S / S_ref - 1) < 1e-14 and np.all(w == S / P)


def test_metropolis_argument_checks():
    lib = _lib.load()
    assert lib.rbe_sample_k_metropolis(1, 0, 10.0, 0.3, 4, -1, None, None, None) == _lib.RBE_EINVAL
    assert lib.rbe_sample_k_metropolis(1, 0, -1.0, 0.3, 4, 8, None, None, None) == _lib.RBE_EINVAL
    st, h = _create(1, [0, 10], [0, 5], [3.0], [1.0])
    assert st == 0
    assert lib.rbe_plan_set_sampler(h, 2, 10) == _lib.RBE_EINVAL
    assert lib.rbe_plan_set_sampler(h, _lib.RBE_SAMPLER_METROPOLIS, -3) == _lib.RBE_EINVAL
    assert lib.rbe_plan_set_sampler(h, _lib.RBE_SAMPLER_METROPOLIS, 16) == 0
    assert lib.rbe_plan_set_sampler(None, 0, 0) == _lib.RBE_EINVAL
    lib.rbe_plan_destroy(h)


def _rbl(N=1000, L=40.0, alpha=0.1, rc=5.0, rs=10.0, p=10):
    lib = _lib.load()
    h = ctypes.c_void_p()
    prm = _lib.RBLParams(N, L, alpha, rc, rs, p)
    return lib.rbl_plan_create(ctypes.byref(prm), ctypes.byref(h)), h


def test_rbl_plan_validation_and_grid():
    lib = _lib.load()
    st, h = _rbl()
    assert st == 0 and h.value
    v = [ctypes.c_int32() for _ in range(3)]
    assert lib.rbl_plan_grid(h, *[ctypes.byref(a) for a in v]) == 0
    nc, R, span = (a.value for a in v)
    assert (nc, R, span) == (8, 2, 5)                    # h = 5 = r_c, reach ceil(10 / 5)
    assert lib.rbl_plan_workspace_bytes(h) % 256 == 0
    # pair slots: mean core and min(p, mean shell) counts of the uniform density, each with
    # the allowance m + 6 sqrt(m) + 16
    c = [ctypes.c_int32() for _ in range(2)]
    assert lib.rbl_plan_capacity(h, *[ctypes.byref(a) for a in c]) == 0
    dens = 1000 / 40.0 ** 3
    mc, ms = dens * 4 / 3 * math.pi * 5.0 ** 3, dens * 4 / 3 * math.pi * (10.0 ** 3 - 5.0 ** 3)
    allow = lambda m: m + 6 * math.sqrt(m) + 16
    assert c[0].value == 4 * math.ceil(math.ceil(allow(mc) + min(10, allow(ms))) / 4) and c[1].value == 512
    assert lib.rbl_plan_workspace_bytes(h) >= 1000 * c[0].value * 4
    assert lib.rbl_plan_capacity(None, *[ctypes.byref(a) for a in c]) == _lib.RBE_EINVAL
    assert lib.rbl_plan_set_timing_events(h, None, None, None, None) == 0      # clears, records nothing
    assert lib.rbl_plan_set_timing_events(None, None, None, None, None) == _lib.RBE_EINVAL
    lib.rbl_plan_destroy(h)
    st, h = _rbl(L=21.0, rc=5.0, rs=10.0)                # 4 cells per axis: the stencil wraps
    assert st == 0
    assert lib.rbl_plan_grid(h, *[ctypes.byref(a) for a in v]) == 0
    assert (v[0].value, v[2].value) == (4, 4)
    lib.rbl_plan_destroy(h)
    for bad in (dict(rs=20.0), dict(rc=0.0), dict(rc=11.0), dict(p=0), dict(N=-1), dict(alpha=-1.0),
                dict(L=float("nan"))):
        st, h = _rbl(**bad)
        assert st == _lib.RBE_EINVAL and not h.value, bad
    st, h = _rbl()
    assert lib.rbl_short_force(h, *([None] * 6), 1, 0, None, None, None, None) == _lib.RBE_EWORKSPACE
    if not torch.cuda.is_available():
        assert lib.rbl_short_force(h, *([ctypes.c_void_p(256)] * 6), 1, 0, ctypes.c_void_p(256), None,
                                   ctypes.c_void_p(256), None) == _lib.RBE_ENODEV
    lib.rbl_plan_destroy(h)
