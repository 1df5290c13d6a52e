"""Pins of the oracle's ghost: the f-factor and the sound speed.

Neither is checked by conservation (the pairwise exchange conserves momentum
and energy for any f and any c), so each is pinned here by what mathematics
fixes independently of the oracle's own formula:

* f (Section 3.2, with the inverse as the comoving section prints it): with
  h tied to the density by the constraint n h^3 = eta^3 (Section 3.1), the
  rate of change of the smoothed density along the particle motion is
  d rho_i / dt = f_i sum_j m_j v_ij . grad_i W_ij = -f_i rho_i (div v)_i.
  The test moves the particles to x +/- eps v, re-solves every h tightly and
  takes the central difference of rho_i.
* c (Section 3.1 equation of state; the sound speed of the Balsara switch in
  Section 3.2): c^2 is the derivative of P with respect to rho along an
  adiabat. The adiabat is integrated from the first law of thermodynamics,
  du = (P / rho^2) d rho, with the oracle's own pressure, and the derivative
  is taken by finite differences."""
import numpy as np

import oracle
from paper_2305_13380_amd import inputs

# A tight solve: the central difference below divides by 2 eps.
PT = oracle.Params(h_tol=1e-13, max_iter=80)


def _moved(ps, t):
    q = ps.copy()
    for a, v in (("x", "vx"), ("y", "vy"), ("z", "vz")):
        pos = getattr(ps, a) + t * getattr(ps, v).astype(np.float64)
        setattr(q, a, np.ascontiguousarray(np.mod(pos, 1.0)))
    return q


def _rho_at(ps, recv, h0):
    h, dens, conv, _, _ = oracle.solve_h(ps, PT, recv=recv, mode="brute", h0=h0)
    assert conv.all()
    return h, dens


def test_f_factor_is_the_constrained_continuity_equation():
    # Lognormal clustering (sigma 2) gives a spread of X = h rho'/(3 rho), so
    # that f = 1/(1 + X) and the tempting 1 + X (the form printed without
    # the inverse) differ clearly; O(1) random velocities make div v large.
    ps = inputs.lognormal_box(10, 900, 2.0, 11, sigma_v=1.0)
    recv = np.arange(0, ps.n, 3)
    h0, d0 = _rho_at(ps, recv, None)
    hfull = ps.h.astype(np.float64).copy()
    hfull[recv] = h0
    g = oracle.ghost(d0, ps.u.astype(np.float64)[recv], h0, PT)
    eps = 2e-6
    _, dp = _rho_at(_moved(ps, eps), recv, hfull)
    _, dm = _rho_at(_moved(ps, -eps), recv, hfull)
    fd = (dp["rho"] - dm["rho"]) / (2 * eps)
    # d rho/dt = -f rho div v = -f div_sum  (div_sum = sum m (v_j - v_i).grad_i W)
    pred = -g["f"] * d0["div_sum"]
    scale = np.abs(d0["div_sum"]) + 1e-3 * np.abs(d0["rho"])
    # particles held at h_max (voids of this small box) do not satisfy the
    # constraint, so the identity does not apply to them
    free = h0 < PT.hmax() * (1 - 1e-9)
    assert np.count_nonzero(free) > 0.8 * recv.size
    err = np.abs(fd - pred)[free] / scale[free]
    assert err.max() < 2e-5, err.max()
    # the test discriminates: the form without the inverse misses by far
    X = h0 * d0["rho_dh"] / (3 * d0["rho"])
    assert np.abs(X).max() > 0.1
    wrong = -(1.0 + X) * d0["div_sum"]
    bad = np.abs(fd - wrong)[free] / scale[free]
    assert np.count_nonzero(bad > 1e-2) > recv.size // 4


def test_f_factor_uniform_lattice_is_one():
    # A perfect lattice at rest: rho does not change, and both sides of the
    # identity are zero (div_sum exactly), with f finite and positive.
    ps = inputs.lattice_box(8, 0, jitter=0.0, sigma_v=0.0)
    h, dens, conv, _, _ = oracle.solve_h(ps, PT, mode="brute")
    g = oracle.ghost(dens, ps.u.astype(np.float64), h, PT)
    assert conv.all()
    assert np.all(np.isfinite(g["f"])) and np.all(g["f"] > 0)
    assert np.all(dens["div_sum"] == 0.0)


def _adiabat(rho0, u0, rho1, steps=400):
    """Integrate du/drho = P(rho, u)/rho^2 from (rho0, u0) to rho1 by RK4,
    with P from the oracle's ghost (its own equation of state)."""
    def Pof(rho, u):
        n = rho.shape[0]
        d = {"rho": rho, "rho_dh": np.zeros(n), "div_sum": np.zeros(n),
             "curl_x": np.zeros(n), "curl_y": np.zeros(n), "curl_z": np.zeros(n)}
        return oracle.ghost(d, u, np.ones(n), PT)["P"]

    def du(rho, u):
        return Pof(rho, u) / rho ** 2

    u = u0.copy()
    rho = rho0.copy()
    dr = (rho1 - rho0) / steps
    for _ in range(steps):
        k1 = du(rho, u)
        k2 = du(rho + dr / 2, u + dr / 2 * k1)
        k3 = du(rho + dr / 2, u + dr / 2 * k2)
        k4 = du(rho + dr, u + dr * k3)
        u = u + dr / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        rho = rho + dr
    return u, Pof(rho1, u)


def test_sound_speed_is_the_adiabatic_pressure_derivative():
    rng = np.random.default_rng(5)
    n = 64
    rho = 10.0 ** rng.uniform(-3, 3, n)
    u = 10.0 ** rng.uniform(-2, 2, n)
    d = {"rho": rho, "rho_dh": np.zeros(n), "div_sum": np.zeros(n),
         "curl_x": np.zeros(n), "curl_y": np.zeros(n), "curl_z": np.zeros(n)}
    g = oracle.ghost(d, u, np.ones(n), PT)
    delta = 1e-3
    _, Pp = _adiabat(rho, u, rho * (1 + delta))
    _, Pm = _adiabat(rho, u, rho * (1 - delta))
    c2_fd = (Pp - Pm) / (2 * delta * rho)
    np.testing.assert_allclose(g["c"] ** 2, c2_fd, rtol=1e-6)
    # the test discriminates: an isothermal c^2 = P/rho misses by gamma
    assert np.all(np.abs(g["P"] / rho / c2_fd - 1) > 0.3)


def test_adiabat_keeps_the_printed_entropy_function():
    # The equation of state is printed in two forms, (gamma - 1) u rho and
    # A rho^gamma: along an adiabat of the first law, A = P / rho^gamma must
    # stay constant for the oracle's pressure and gamma = 5/3.
    rng = np.random.default_rng(6)
    n = 16
    rho = 10.0 ** rng.uniform(-2, 2, n)
    u = 10.0 ** rng.uniform(-1, 1, n)
    d = {"rho": rho, "rho_dh": np.zeros(n), "div_sum": np.zeros(n),
         "curl_x": np.zeros(n), "curl_y": np.zeros(n), "curl_z": np.zeros(n)}
    P0 = oracle.ghost(d, u, np.ones(n), PT)["P"]
    _, P1 = _adiabat(rho, u, 3.0 * rho, steps=2000)
    g = PT.gamma_gas
    np.testing.assert_allclose(P1 / (3.0 * rho) ** g, P0 / rho ** g, rtol=1e-9)
