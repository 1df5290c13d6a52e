"""Pins of the oracle's Phantom-like flavour (Appendix A): density-energy
with the SPHENIX viscosity switch at decay length 0.25, and conduction with
alpha_c = 1 for every particle and the conduction speed
sqrt(2 |P_i - P_j| / (rho_i + rho_j)).

Fixed by: the printed constant; equality with the density-energy passes when
every alpha_c is 1 and the particles are at rest (then both conduction
speeds are the pressure term alone); independence from the per-particle
alpha_c inputs; exact energy conservation; heat flowing from hot to cold
across a temperature step."""
import json
import os

import numpy as np

import oracle
from paper_2305_13380_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
PE = oracle.Params()
PP = oracle.Params(flavour="phantom")


def step(ps, params):
    h, _, conv, _, _ = oracle.solve_h(ps, PE, mode="brute")
    assert conv.all()
    return h, oracle.fixed_h_step(ps, params, mode="brute", h=h)


def test_constant_is_the_printed_one():
    assert oracle.PHANTOM_ELL == GOLD["phantom_viscosity_decay_length"]["value"]


def test_phantom_equals_energy_flavour_at_rest_with_unit_alpha_c():
    ps = inputs.lattice_box(10, 8, u="logu", sigma_v=0.0)
    ps.alpha_c[:] = 1.0
    h, re = step(ps, PE)
    rp = oracle.fixed_h_step(ps, PP, mode="brute", h=h)
    for k in ("ax", "ay", "az", "du", "vsig"):
        np.testing.assert_allclose(rp[k], re[k], rtol=1e-13, atol=1e-13 * np.abs(re[k]).max())
    assert np.abs(re["du"]).max() > 0  # conduction is at work (u varies)


def test_phantom_ignores_the_particles_alpha_c():
    ps = inputs.lognormal_box(12, 2000, 2.0, 13, sigma_v=0.3)
    h, a = step(ps, PP)
    q = ps.copy()
    q.alpha_c = np.zeros_like(ps.alpha_c)
    b = oracle.fixed_h_step(q, PP, mode="brute", h=h)
    for k in ("ax", "ay", "az", "du", "vsig"):
        assert np.array_equal(a[k], b[k]), k
    # while the density-energy flavour depends on them
    c = oracle.fixed_h_step(ps, PE, mode="brute", h=h)
    d = oracle.fixed_h_step(q, PE, mode="brute", h=h)
    assert not np.array_equal(c["du"], d["du"])


def test_phantom_conserves_energy_and_conducts_from_hot_to_cold():
    ps = inputs.lattice_box(12, 9, jitter=0.0, sigma_v=0.0)
    hot = ps.x < 0.5
    ps.u = np.where(hot, 4.0, 1.0).astype(np.float32)
    ps.alpha_v[:] = 0.0  # no viscosity: the particles are at rest anyway
    h, r = step(ps, PP)
    s = oracle.sums(ps.m, ps.vx, ps.vy, ps.vz, r["ax"], r["ay"], r["az"], r["du"])
    assert abs(s[3]) < 1e-13 * s[5]
    # the particles within a kernel support of the two interfaces (x = 0 and
    # x = 1/2, periodic); the others see one temperature only
    d = np.minimum(np.abs(ps.x - 0.5), np.minimum(ps.x, 1.0 - ps.x))
    near = d < PE.gamma_k * h.max()
    # conduction moves heat down the temperature step; the pressure term
    # (the particles are at rest) adds nothing to du
    assert np.all(r["du"][near & hot] < 0) and np.all(r["du"][near & ~hot] > 0)
    assert np.all(r["du"][~near] == 0.0)
