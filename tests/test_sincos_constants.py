"""The FP64 sin/cos constants of the kernels, checked on the CPU.

The FP64 passes evaluate sin and cos of 2 pi t from polynomial coefficients and a table
size kept in paper_2407_09315_amd/csrc/sincos_coeffs.h.  These tests parse that header,
replay its two forms in float64 (the same operation order as the kernels, with separate
multiply and add where the kernels fuse them) and compare with mpmath at 40 digits:
  - the wide-range form (quarter-turn reduction, |f| <= 1/8) that builds the table rows;
  - the table form: a phase in units of 1/N turn (N = kTurnSteps), q = rint(t),
    g = t - q, short polynomials in g, and a rotation of table row q mod N.
A wrong coefficient, a dropped term or a table size the polynomials were not fitted for
moves the error far above the bounds used here.
"""
import os
import re

import mpmath
import numpy as np
import pytest

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_2407_09315_amd", "csrc", "sincos_coeffs.h")


def _parse():
    text = open(HEADER).read()
    ints = {k: int(v) for k, v in re.findall(r"constexpr int (\w+) = (\d+);", text)}
    arrays = {}
    for name, body in re.findall(r"constexpr double (\w+)\[\w+\] = \{([^}]*)\};", text):
        arrays[name] = [float.fromhex(v.strip()) for v in body.split(",")]
    return ints, arrays


INTS, ARR = _parse()
mpmath.mp.dps = 40


def _horner(cs, u):
    p = cs[-1]
    for c in reversed(cs[:-1]):
        p = p * u + c
    return p


def sincos_wide(r):
    """sin and cos of 2 pi r for |r| <= 1/2 from the wide-range coefficients."""
    q = np.rint(4.0 * r)
    f = r - q * 0.25                      # exact: q/4 is exact and |r - q/4| <= 1/8
    f2 = f * f
    sn = _horner(ARR["kSin"], f2) * f
    pc = _horner(ARR["kCos"], f2)
    aq = np.abs(q)
    cq = 1.0 - aq                         # cos(pi q / 2) for q in {-2..2}
    sq = q * (2.0 - aq)                   # sin(pi q / 2)
    return sn * cq + pc * sq, pc * cq - sn * sq


def sincos_table(t, tab_c, tab_s):
    """sin and cos of 2 pi t / N for a phase t in units of 1/N turn, from the table."""
    n = INTS["kTurnSteps"]
    q = np.rint(t)
    g = t - q
    u = g * g
    sf = g * _horner(ARR["kSinShort"], u)
    cm1 = u * _horner(ARR["kCosm1Short"], u)
    row = q.astype(np.int64) & (n - 1)
    c, s = tab_c[row], tab_s[row]
    return s * cm1 + (c * sf + s), c * cm1 + (-s * sf + c)


def _exact(turns):
    """sin and cos of 2 pi x for each float x, exactly rounded (mpmath)."""
    sn = np.array([float(mpmath.sin(2 * mpmath.pi * mpmath.mpf(float(x)))) for x in turns])
    cs = np.array([float(mpmath.cos(2 * mpmath.pi * mpmath.mpf(float(x)))) for x in turns])
    return sn, cs


def test_header_shape():
    n = INTS["kTurnSteps"]
    assert n > 0 and n & (n - 1) == 0, "the kernels index the table with q & (N - 1)"
    assert len(ARR["kSin"]) == INTS["kSinTerms"] and len(ARR["kCos"]) == INTS["kCosTerms"]
    assert len(ARR["kSinShort"]) == INTS["kSinShortTerms"] == 3
    assert len(ARR["kCosm1Short"]) == INTS["kCosm1ShortTerms"] == 2
    # leading terms: sin(2 pi g / N) ~ (2 pi / N) g and cos(2 pi g / N) - 1 ~ -(2 pi / N)^2 g^2 / 2
    assert ARR["kSinShort"][0] == pytest.approx(2 * np.pi / n, rel=1e-15)
    assert ARR["kCosm1Short"][0] == pytest.approx(-0.5 * (2 * np.pi / n) ** 2, rel=1e-12)
    assert ARR["kSin"][0] == pytest.approx(2 * np.pi, rel=1e-15) and ARR["kCos"][0] == 1.0


def test_wide_range_form():
    rng = np.random.default_rng(11)
    r = np.concatenate([rng.uniform(-0.5, 0.5, 1500), np.linspace(-0.5, 0.5, 257),
                        [0.0, 0.125, -0.125, 0.25, -0.25, 0.375, 0.5, -0.5, 1e-9]])
    s, c = sincos_wide(r)
    es, ec = _exact(r)
    assert np.max(np.abs(s - es)) < 5e-16
    assert np.max(np.abs(c - ec)) < 5e-16


def test_table_form():
    n = INTS["kTurnSteps"]
    qi = np.arange(n)
    qs = np.where(qi <= n // 2, qi, qi - n) / n          # table rows as the kernels build them
    tab_s, tab_c = sincos_wide(qs)
    rng = np.random.default_rng(12)
    # phases m.s' in units of 1/N turn, up to |m| ~ 100 per component of a unit cell
    t = np.concatenate([rng.uniform(-3e2 * n, 3e2 * n, 2000), rng.uniform(-2.0, 2.0, 200),
                        np.arange(-n, n + 1, 37) + 0.5, [0.0, 0.5, -0.5, n / 2.0, n / 4.0]])
    s, c = sincos_table(t, tab_c, tab_s)
    es, ec = _exact(t / n)                                # t / n is exact (power of two)
    assert np.max(np.abs(s - es)) < 8e-16
    assert np.max(np.abs(c - ec)) < 8e-16

