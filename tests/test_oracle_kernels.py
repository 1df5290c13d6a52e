"""Pins of the oracle's kernel family (Section 3.1 lists Wendland C2, C4, C6
and the cubic, quartic and quintic B-splines, all normalised, with a central
gradient of zero, and one smoothing length h for every kernel, H = gamma_k h).

Fixed by what the mathematics says of each kernel, not by retyping it: unit
integral over space; the second moment, which must give h = twice the
standard deviation for the exact gamma_k^2 of the table; W' and dW/dh
against finite differences; the smoothness every member of the family has
(C2 at least: a wrong coefficient or knot of a spline breaks it); W'(0) = 0,
compact support, positivity and monotonicity; and, end to end, the number
density of a lattice and exact momentum conservation of the force pass.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

NAMES = sorted(oracle.KERNELS)
# u = r/H of the knots of each kernel: polynomial between consecutive knots
KNOTS = {"wendland_c2": [0, 1], "wendland_c4": [0, 1], "wendland_c6": [0, 1],
         "cubic_spline": [0, 0.5, 1], "quartic_spline": [0, 0.2, 0.6, 1],
         "quintic_spline": [0, 1 / 3, 2 / 3, 1]}


def _gl(f, knots, H, n=32):
    """Integral over [0, H) by Gauss-Legendre on each polynomial piece
    (exact for these piecewise polynomials of degree <= 15 times r^4)."""
    x, w = np.polynomial.legendre.leggauss(n)
    tot = 0.0
    for a, b in zip(knots[:-1], knots[1:]):
        a, b = a * H, b * H
        t = 0.5 * (b - a) * x + 0.5 * (b + a)
        tot += 0.5 * (b - a) * np.sum(w * f(t))
    return tot


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("h", [0.02, 1.0, 3.5])
def test_normalised(name, h):
    H = oracle.kernel_gamma(name) * h
    val = _gl(lambda r: 4 * math.pi * r * r * oracle.kernel(name, r, h)[0], KNOTS[name], H)
    assert abs(val - 1.0) < 1e-13


@pytest.mark.parametrize("name", NAMES)
def test_second_moment_gives_h_twice_sigma(name):
    # per-axis variance sigma^2 = (1/3) int r^2 W d^3r must be (h/2)^2 at the
    # table's gamma_k: the exact fractions are the kernels' own moments
    h = 0.7
    H = oracle.kernel_gamma(name) * h
    m2 = _gl(lambda r: 4 * math.pi * r ** 4 * oracle.kernel(name, r, h)[0], KNOTS[name], H)
    assert abs(m2 / 3.0 - (h / 2.0) ** 2) < 1e-13


def test_wendland_c2_is_the_default_and_matches_its_factored_form():
    assert oracle.Params().kernel == "wendland_c2"
    assert oracle.Params().gamma_k == oracle.kernel_gamma("wendland_c2")
    h = 0.6
    H = oracle.kernel_gamma("wendland_c2") * h
    u = np.linspace(0, 0.999, 301)
    w, _, _ = oracle.kernel("wendland_c2", u * H, h)
    ref = 21 / (2 * math.pi * H ** 3) * (1 - u) ** 4 * (1 + 4 * u)
    np.testing.assert_allclose(w, ref, rtol=0, atol=1e-13 * ref[0])
    np.testing.assert_array_equal(w, oracle.wc2(u * H, h)[0])


@pytest.mark.parametrize("name", NAMES)
def test_derivatives_by_finite_differences(name):
    h = 0.8
    H = oracle.kernel_gamma(name) * h
    r = np.linspace(0.003, 0.997, 331) * H
    _, d1, d2 = oracle.kernel(name, r, h)
    e = 1e-6 * H
    fd = (oracle.kernel(name, r + e, h)[0] - oracle.kernel(name, r - e, h)[0]) / (2 * e)
    np.testing.assert_allclose(d1, fd, rtol=0, atol=1e-8 * np.abs(d1).max())
    eh = 1e-6 * h
    fdh = (oracle.kernel(name, r, h + eh)[0] - oracle.kernel(name, r, h - eh)[0]) / (2 * eh)
    np.testing.assert_allclose(d2, fdh, rtol=0, atol=1e-8 * np.abs(d2).max())


@pytest.mark.parametrize("name", NAMES)
def test_twice_continuously_differentiable(name):
    # Every kernel of the family is at least C2 on [0, H]: the second
    # derivative (finite differences of the analytic W') changes by O(step)
    # between neighbouring points everywhere, knots included. A wrong
    # coefficient or knot of a spline leaves a jump of O(1) in W''.
    h = 1.0
    H = oracle.kernel_gamma(name) * h
    r = np.linspace(0.0, H * 1.02, 20001)
    _, d1, _ = oracle.kernel(name, r, h)
    d2 = np.diff(d1) / np.diff(r)
    jump = np.abs(np.diff(d2)).max()
    scale = np.abs(d2).max()
    assert jump < 2e-3 * scale, "W'' jumps by %.3g of its scale" % (jump / scale)


@pytest.mark.parametrize("name", NAMES)
def test_support_centre_and_shape(name):
    h = 1.3
    H = oracle.kernel_gamma(name) * h
    w, d1, d2 = oracle.kernel(name, np.array([H, H * (1 + 1e-12), 2 * H]), h)
    assert np.all(w == 0) and np.all(d1 == 0) and np.all(d2 == 0)
    _, g0, _ = oracle.kernel(name, np.array([0.0]), h)
    assert abs(g0[0]) < 1e-13 / H ** 4  # central gradient zero
    r = np.linspace(0, H * 0.9999, 5001)
    w, d1, _ = oracle.kernel(name, r, h)
    # (the expanded Wendland C2 polynomial rounds to ~0 right at the edge)
    assert np.all(w[r < 0.99 * H] > 0) and np.all(w >= -1e-14 * w[0])
    assert np.all(d1 <= 1e-12 * np.abs(d1).max())


@pytest.mark.parametrize("name", NAMES)
def test_scale_free(name):
    r = np.linspace(0, 2.5, 60)
    w1, g1, _ = oracle.kernel(name, r, 1.0)
    for s in (0.01, 7.0):
        w2, g2, _ = oracle.kernel(name, r * s, s)
        np.testing.assert_allclose(w2, w1 / s ** 3, rtol=0, atol=1e-13 * w1[0] / s ** 3)
        np.testing.assert_allclose(g2, g1 / s ** 4, rtol=0,
                                   atol=1e-13 * np.abs(g1).max() / s ** 4)


@pytest.mark.parametrize("name", NAMES)
def test_lattice_number_density(name):
    # On a cubic lattice of spacing D at h = eta D the kernel sum approximates
    # its unit integral: n D^3 = 1 to within the discretisation error (under
    # 2 % for every kernel at eta = 1.2348), identical for every particle.
    ps = inputs.lattice_box(10, 0, jitter=0.0, sigma_v=0.0)
    P = oracle.Params.with_kernel(name)
    d = oracle.density(ps, ps.h, P, recv=np.arange(0, ps.n, 97), mode="brute")
    nD3 = d["n"] * 0.1 ** 3
    assert np.all(np.abs(nD3 - 1.0) < 0.02)
    assert np.ptp(nD3) < 1e-12


@pytest.mark.parametrize("name", NAMES)
def test_force_conserves_momentum_and_energy(name):
    P = oracle.Params.with_kernel(name)
    ps = inputs.lognormal_box(14, 1500, 2.0, 3, sigma_v=0.2)
    h, _, conv, _, _ = oracle.solve_h(ps, P, mode="brute")
    assert conv.all()
    r = oracle.fixed_h_step(ps, P, mode="brute", h=h)
    m = ps.m.astype(np.float64)
    v = np.stack([ps.vx, ps.vy, ps.vz], 1).astype(np.float64)
    a = np.stack([r["ax"], r["ay"], r["az"]], 1)
    assert np.abs((m[:, None] * a).sum(0)).max() < 1e-13 * (m * np.linalg.norm(a, axis=1)).sum()
    e = (m * ((v * a).sum(1) + r["du"])).sum()
    assert abs(e) < 1e-13 * (m * (np.abs(v * a).sum(1) + np.abs(r["du"]))).sum()
    # the converged h solves n (h/eta)^3 = 1 whatever the kernel: the last
    # Newton step |ln G| / G' is below h_tol, except where h stopped at h_max
    # (voids of this small box, for the wider kernels)
    d = oracle.density(ps, h, P, mode="brute")
    G = d["n"] * (h / P.eta) ** 3
    Gp = 3.0 + h * d["n_dh"] / d["n"]
    free = h < P.hmax()
    assert free.mean() > 0.95
    assert np.all(np.abs(np.log(G[free])) / Gp[free] < 1.001 * P.h_tol)
    assert np.all(G[~free] < 1.0)
