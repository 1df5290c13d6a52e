"""Pins of the oracle's density-entropy flavour (the Gadget2 solver of
Section 3.2): the adiabat A is the thermodynamic variable, P = A rho^gamma
(the second printed form of the equation of state), dA/dt = 0 but for the
viscous heating, no conduction.

Fixed by: equivalence with the density-energy passes when A is set from u
(same pressure, hence the same accelerations and the same internal-energy
rate), dA/dt = 0 exactly without viscosity, dA/dt >= 0 with it (viscosity
only heats), exact energy conservation of the implied internal-energy rate,
and the sound speed as the adiabatic derivative of P = A rho^gamma."""
import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

PE = oracle.Params()
PS = oracle.Params(flavour="entropy")


def state(ps, params):
    h, _, conv, _, _ = oracle.solve_h(ps, params, mode="brute")
    assert conv.all()
    return h, oracle.fixed_h_step(ps, params, mode="brute", h=h)


def as_entropy(ps, h):
    """The same particles with u replaced by A = (gamma - 1) u / rho^(gamma - 1)."""
    d = oracle.density(ps, h, PE, mode="brute")
    g = PE.gamma_gas
    q = ps.copy()
    q.u = (g - 1.0) * ps.u.astype(np.float64) / d["rho"] ** (g - 1.0)
    q.alpha_c = np.zeros_like(ps.alpha_c)
    return q


@pytest.mark.parametrize("kind", ["lattice", "lognormal"])
def test_entropy_flavour_equals_energy_flavour_for_the_same_pressure(kind):
    if kind == "lattice":
        ps = inputs.lattice_box(10, 8, u="logu", sigma_v=0.3)
    else:
        ps = inputs.lognormal_box(12, 2000, 2.0, 9, sigma_v=0.3)
    ps.alpha_c[:] = 0.0  # density-entropy has no conduction
    h, re = state(ps, PE)
    q = as_entropy(ps, h)
    rs = oracle.fixed_h_step(q, PS, mode="brute", h=h)
    np.testing.assert_allclose(rs["P"], re["P"], rtol=1e-12)
    np.testing.assert_allclose(rs["c"], re["c"], rtol=1e-12)
    a_e = np.stack([re[k] for k in ("ax", "ay", "az")], 1)
    a_s = np.stack([rs[k] for k in ("ax", "ay", "az")], 1)
    scale = np.linalg.norm(a_e, axis=1).max()
    assert np.abs(a_s - a_e).max() < 1e-11 * scale
    np.testing.assert_allclose(rs["du_energy"], re["du"], rtol=1e-10,
                               atol=1e-12 * np.abs(re["du"]).max())


def test_entropy_changes_only_by_viscous_heating():
    ps = inputs.lognormal_box(12, 2000, 2.0, 10, sigma_v=0.3)
    h, _ = state(ps, PE)
    q = as_entropy(ps, h)
    r = oracle.fixed_h_step(q, PS, mode="brute", h=h)
    # viscosity only heats: every pair term is >= 0
    assert np.all(r["du"] >= 0.0) and np.any(r["du"] > 0.0)
    # the implied internal-energy rate: the adiabatic part plus the heating
    q0 = q.copy()
    q0.alpha_v = np.zeros_like(q.alpha_v)
    r0 = oracle.fixed_h_step(q0, PS, mode="brute", h=h)
    assert np.all(r0["du"] == 0.0)  # no viscosity: A is constant
    g = PS.gamma_gas
    heat = r["rho"] ** (g - 1.0) / (g - 1.0) * r["du"]
    np.testing.assert_allclose(r["du_energy"] - r0["du_energy"], heat, rtol=1e-9,
                               atol=1e-12 * np.abs(heat).max())


def test_entropy_flavour_conserves_momentum_and_energy():
    ps = inputs.lognormal_box(12, 2000, 2.0, 12, sigma_v=0.3)
    h, _ = state(ps, PE)
    q = as_entropy(ps, h)
    r = oracle.fixed_h_step(q, PS, mode="brute", h=h)
    s = oracle.sums(q.m, q.vx, q.vy, q.vz, r["ax"], r["ay"], r["az"], r["du_energy"])
    assert np.abs(s[:3]).max() < 1e-13 * s[4]
    assert abs(s[3]) < 1e-13 * (s[4] * 0.3 * 3 + s[5])


def test_entropy_sound_speed_is_the_adiabatic_derivative():
    rng = np.random.default_rng(4)
    n = 32
    rho = 10.0 ** rng.uniform(-2, 2, n)
    A = 10.0 ** rng.uniform(-1, 1, n)

    def ghost(rr):
        d = {"rho": rr, "rho_dh": np.zeros(n), "div_sum": np.zeros(n), "curl_x": np.zeros(n),
             "curl_y": np.zeros(n), "curl_z": np.zeros(n)}
        return oracle.ghost(d, A, np.ones(n), PS)

    g = ghost(rho)
    e = 1e-5
    c2 = (ghost(rho * (1 + e))["P"] - ghost(rho * (1 - e))["P"]) / (2 * e * rho)
    np.testing.assert_allclose(g["c"] ** 2, c2, rtol=1e-8)
    np.testing.assert_allclose(g["P"] / rho ** PS.gamma_gas, A, rtol=1e-13)
