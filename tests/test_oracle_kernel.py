"""Pins of the oracle's kernel (Wendland C2, 3D) against what the paper and the
mathematics fix: the printed polynomial, normalisation, the second moment that
defines gamma_k, derivatives by finite differences, and support/continuity."""
import json
import math
import os

import numpy as np
import pytest

import oracle

P = oracle.Params()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _gl(f, a, b, n=24):
    x, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (b - a) * x + 0.5 * (b + a)
    return 0.5 * (b - a) * np.sum(w * f(t))


def test_kernel_matches_printed_polynomial():
    g = json.load(open(GOLDEN))["wendland_c2_3d"]
    for h in (0.05, 0.7, 3.0):
        H = P.gamma_k * h
        u = np.linspace(0.0, 0.999, 257)
        w, _, _ = oracle.wc2(u * H, h)
        ref = (g["prefactor_numerator"] / (g["prefactor_denominator_over_pi"] * math.pi * H ** 3)
               * np.polyval(g["poly_coeffs_high_to_low"], u))
        # the polynomial cancels towards u = 1: compare on the scale of W(0)
        np.testing.assert_allclose(w, ref, rtol=0, atol=1e-13 * ref[0])


def test_kernel_zero_outside_support():
    h = 0.4
    H = P.gamma_k * h
    w, d1, d2 = oracle.wc2(np.array([H, H * (1 + 1e-12), 2 * H, 10.0]), h)
    assert np.all(w == 0) and np.all(d1 == 0) and np.all(d2 == 0)


@pytest.mark.parametrize("h", [0.01, 0.3, 1.0, 4.0])
def test_kernel_normalised(h):
    # int W d^3r = 1 (the kernel must be normalised, Section 3.1). The
    # integrand is a polynomial of degree 7 in r: Gauss-Legendre is exact.
    H = P.gamma_k * h
    val = _gl(lambda r: 4 * math.pi * r * r * oracle.wc2(r, h)[0], 0.0, H)
    assert abs(val - 1.0) < 1e-13


def test_second_moment_fixes_gamma_k():
    # <r^2> = int r^2 W d^3r = H^2/5 for this kernel, i.e. per-axis variance
    # sigma^2 = H^2/15. The Dehnen & Aly convention h = 2 sigma then gives
    # H/h = sqrt(15)/2: the oracle's gamma_k must reproduce 3 (h/2)^2.
    h = 0.9
    H = P.gamma_k * h
    m2 = _gl(lambda r: 4 * math.pi * r ** 4 * oracle.wc2(r, h)[0], 0.0, H)
    assert abs(m2 - H * H / 5.0) < 1e-13 * H * H
    assert abs(m2 / 3.0 - (h / 2.0) ** 2) < 1e-13


def test_kernel_derivatives_by_finite_differences():
    h = 0.8
    H = P.gamma_k * h
    r = np.linspace(0.01, 0.99, 61) * H
    _, d1, d2 = oracle.wc2(r, h)
    e = 1e-6 * H
    fd_r = (oracle.wc2(r + e, h)[0] - oracle.wc2(r - e, h)[0]) / (2 * e)
    scale = np.abs(d1).max()
    np.testing.assert_allclose(d1, fd_r, rtol=0, atol=1e-8 * scale)
    eh = 1e-6 * h
    fd_h = (oracle.wc2(r, h + eh)[0] - oracle.wc2(r, h - eh)[0]) / (2 * eh)
    np.testing.assert_allclose(d2, fd_h, rtol=0, atol=1e-8 * np.abs(d2).max())


def test_kernel_central_gradient_zero_and_c2_edge():
    # Section 3.1: zero central gradient; Wendland C2 is twice continuously
    # differentiable, so W and W' vanish at the support edge.
    h = 1.3
    H = P.gamma_k * h
    _, d1, _ = oracle.wc2(np.array([0.0]), h)
    assert d1[0] == 0.0
    w, d1, _ = oracle.wc2(np.array([H * (1 - 1e-5)]), h)
    w0, _, _ = oracle.wc2(np.array([0.0]), h)
    # (the expanded polynomial carries ~1e-16 rounding noise near u = 1)
    assert abs(w[0]) < 1e-14 * w0[0] and abs(d1[0]) < 1e-12 * w0[0] / H


def test_kernel_scale_free():
    # W(r, h) = h^-3 w(r/h): rescaling r and h by s rescales W by s^-3.
    r = np.linspace(0, 1.9, 40)
    w1, d1, _ = oracle.wc2(r, 1.0)
    for s in (0.01, 7.0):
        w2, d2, _ = oracle.wc2(r * s, s)
        np.testing.assert_allclose(w2, w1 / s ** 3, rtol=0, atol=1e-13 * w1[0] / s ** 3)
        np.testing.assert_allclose(d2, d1 / s ** 4, rtol=0, atol=1e-13 * np.abs(d1).max() / s ** 4)
