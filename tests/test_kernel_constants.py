"""Constants written into the HIP kernels, checked against the mathematics
they stand for (no GPU needed).

The ocean current is a sum of Fourier modes evaluated in FP32 by angle
addition around the cell centre; the phase offset d stays within |d| <= 1.6
when the host selects the direct path, where sin d and cos d come from two
fixed polynomials.  Their coefficients are read from the kernel source and
the polynomials evaluated like the kernel does (FP32 fused multiply-adds),
then compared with numpy's sin and cos in FP64.

The closure MLP's GELU takes the normal tail erfc(|z| / sqrt 2) as a base-2
exponential of a fitted polynomial; its constants are read the same way and
the GELU evaluated like the kernel, against scipy's erf.
"""
import os
import re

import numpy as np
import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2303_07819_amd", "csrc", "dem_kernels.h")


def _coefficients():
    text = open(SRC).read()
    body = text[text.index("void sincos_direct("):]
    body = body[:body.index("\n}\n")]
    lits = [float(x) for x in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    # sin: c9, c7 | c5 | c3 ; cos: c10, c8 | c6 | c4 | c2 (-0.5) | 1.0
    sin_c = [lits[0], lits[1], lits[2], lits[3]]
    cos_c = [lits[4], lits[5], lits[6], lits[7], lits[8]]
    assert lits[9] == 1.0
    return np.float32(sin_c), np.float32(cos_c)


def _fma32(a, b, c):
    return np.float32(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def _eval32(x):
    s_c, c_c = _coefficients()
    x2 = np.float32(x * x)
    sp = _fma32(x2, np.full_like(x2, s_c[0]), np.full_like(x2, s_c[1]))
    sp = _fma32(x2, sp, np.full_like(x2, s_c[2]))
    sp = _fma32(x2, sp, np.full_like(x2, s_c[3]))
    s = _fma32(np.float32(x * x2), sp, x)
    cp = _fma32(x2, np.full_like(x2, c_c[0]), np.full_like(x2, c_c[1]))
    for k in (2, 3, 4):
        cp = _fma32(x2, cp, np.full_like(x2, c_c[k]))
    c = _fma32(x2, cp, np.ones_like(x2))
    return s, c


def test_direct_sincos_polynomials_are_accurate():
    x = np.linspace(-1.62, 1.62, 400001).astype(np.float32)
    s, c = _eval32(x)
    xd = x.astype(np.float64)
    es = np.max(np.abs(s.astype(np.float64) - np.sin(xd)))
    ec = np.max(np.abs(c.astype(np.float64) - np.cos(xd)))
    # FP32 evaluation: about one FP32 ulp of values near 1
    assert es < 1.3e-7, es
    assert ec < 1.7e-7, ec


def test_direct_sincos_approximation_error_in_fp64():
    """The polynomials themselves (FP32 coefficients, FP64 evaluation): the
    minimax errors stated in the kernel source.  A wrong or transposed
    coefficient moves them by orders of magnitude."""
    s_c, c_c = _coefficients()
    x = np.linspace(-1.62, 1.62, 400001)
    x2 = x * x
    sp = ((s_c[0] * x2 + s_c[1]) * x2 + s_c[2]) * x2 + s_c[3]
    s = x + x * x2 * sp
    cp = (((c_c[0] * x2 + c_c[1]) * x2 + c_c[2]) * x2 + c_c[3]) * x2 + c_c[4]
    c = 1.0 + x2 * cp
    assert np.max(np.abs(s - np.sin(x))) < 4.5e-8
    assert np.max(np.abs(c - np.cos(x))) < 1.5e-8
    # the sin error equioscillates (a minimax polynomial): extrema of both signs
    e = s - np.sin(x)
    assert e.max() > 3e-8 and e.min() < -3e-8


# ------------------------------------------------------------ GELU of the MLP
MLP_SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2303_07819_amd", "csrc", "mlp_kernels.h")


def _erfc_tail_constants():
    """(scale, coefficients of R from the highest degree down to degree 1)."""
    text = open(MLP_SRC).read()
    body = text[text.index("float erfc_tail("):]
    body = body[:body.index("\n}\n")]
    lits = [float(x) for x in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    return np.float32(lits[0]), np.float32(lits[1:])


def _twice_gelu32(z):
    """twice_gelu evaluated like the kernel: FP32 multiplies and fused
    multiply-adds, the base-2 exponential correctly rounded."""
    a, c = _erfc_tail_constants()
    z = z.astype(np.float32)
    az = np.abs(z)
    s = np.float32(az * a)
    q = np.full_like(s, c[0])
    for cc in c[1:]:
        q = _fma32(q, s, np.full_like(s, cc))
    e = np.float32(s * np.float32(q - s))
    E = np.float32(np.exp2(e.astype(np.float64)))
    return _fma32(-az, E, np.float32(z + az)), E


def test_erfc_tail_scale_and_degree():
    from scipy.special import erfc
    a, c = _erfc_tail_constants()
    assert a == np.float32(np.sqrt(0.5 / np.log(2.0)))
    assert len(c) == 7 and c[0] < 0.0                   # degree 7, falling past the fit range
    # R'(0) = log2(e) P'(0) / sqrt(log2 e), P'(0) = d/dx log erfc(x) at 0 = -2 / sqrt(pi)
    assert c[-1] == pytest.approx(-2.0 / np.sqrt(np.pi) * np.sqrt(1.0 / np.log(2.0)), rel=2e-3)
    # the polynomial in FP64: erfc(x) = exp(-x^2 + P(x)) within 4e-6 relative on [0, 4]
    x = np.linspace(0.0, 4.0, 200001)
    s = x * np.sqrt(1.0 / np.log(2.0))
    q = np.zeros_like(s)
    for cc in c:
        q = q * s + float(cc)
    E = np.exp2(s * (q - s))
    assert np.max(np.abs(E / erfc(x) - 1.0)) < 4e-6


def test_gelu_in_fp32_is_within_7e_7_for_every_z():
    from scipy.special import erf
    z = np.concatenate([np.linspace(-12.0, 12.0, 800001), -np.geomspace(12.0, 1e30, 2001),
                        np.geomspace(12.0, 1e30, 2001)]).astype(np.float32)
    with np.errstate(over="ignore"):                  # s^7 overflows to -inf far out, as on the GPU
        g2, E = _twice_gelu32(z)
    zz = z.astype(np.float64)
    exact = 0.5 * zz * (1.0 + erf(zz / np.sqrt(2.0)))
    g = 0.5 * g2.astype(np.float64)
    assert not np.isnan(g).any()
    inner = np.abs(zz) <= 12.0
    assert np.max(np.abs(g - exact)[inner]) < 7e-7
    # relative on the positive side, and the tail vanishes (not NaN or growing) far out
    pos = zz > 0.05
    m = pos & inner
    assert np.max(np.abs(g[m] - exact[m]) / exact[m]) < 4e-6
    assert np.all(E[np.abs(zz) > 6.0] < 1e-8)
    assert g2[zz == 0.0].max() == 0.0
