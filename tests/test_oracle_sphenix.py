"""Pins of the oracle's SPHENIX viscosity switch (Section 3.3): the shock
indicator S = H^2 max(0, -d(div v)/dt), the target alpha_loc = alpha_max S /
(v_sig^2 + S), the immediate rise to it, and the decay towards it on the time
scale H / (ell c) (reading of the printed update).

Fixed by: the printed constants (golden file), the closed form of a pure
decay, the semigroup property of the decay (two half steps are one step; a
linear or otherwise wrong decay breaks it), the jump to alpha_loc at a
compression, alpha_loc = alpha_max / 2 at S = v_sig^2 and its bounds, and
no change without time or without compression towards the target."""
import json
import math
import os

import numpy as np

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
P = oracle.Params()


def run(alpha, dold, dnew, c, h, vs, dt):
    alpha = np.atleast_1d(np.asarray(alpha, np.float64))
    n = len(alpha)
    f = lambda v: np.full(n, v, np.float64) if np.isscalar(v) else np.asarray(v, np.float64)
    return oracle.alpha_v_update(f(alpha), f(dold), f(dnew), f(c), f(h), f(vs), dt, P)


def test_constants_are_the_printed_ones():
    assert oracle.SPHENIX_ALPHA_V_MAX == GOLD["alpha_v_max"]["value"]
    assert oracle.SPHENIX_ELL == GOLD["viscosity_decay_length"]["value"]


def test_pure_decay_closed_form_and_semigroup():
    # expanding flow (div grows): no shock, alpha decays towards 0
    a0 = np.array([0.1, 1.0, 2.0])
    c, h, dt = 3.0, 0.02, 1e-3
    H = P.gamma_k * h
    a1 = run(a0, -1.0, 0.5, c, h, 1.0, dt)
    np.testing.assert_allclose(a1, a0 * math.exp(-0.05 * c * dt / H), rtol=1e-15)
    a_half = run(run(a0, 0.0, 0.0, c, h, 1.0, dt / 2), 0.0, 0.0, c, h, 1.0, dt / 2)
    a_full = run(a0, 0.0, 0.0, c, h, 1.0, dt)
    np.testing.assert_allclose(a_half, a_full, rtol=1e-14)


def test_jump_at_compression_and_target_bounds():
    c, h, dt, vs = 1.0, 0.05, 1e-2, 2.0
    H = P.gamma_k * h
    # S = v_sig^2 exactly: alpha_loc = alpha_max / 2, above alpha = 0.1
    ddiv = -(vs * vs) / (H * H)
    a = run(0.1, 0.0, ddiv * dt, c, h, vs, dt)
    np.testing.assert_allclose(a, 0.5 * GOLD["alpha_v_max"]["value"], rtol=1e-14)
    # very strong compression: alpha_loc tends to alpha_max from below
    a = run(0.0, 0.0, -1e12, c, h, vs, dt)
    assert np.all(a < 2.0) and np.all(a > 2.0 * (1 - 1e-9))
    # alpha above its target decays towards the target, never below it
    loc = 0.5 * GOLD["alpha_v_max"]["value"]
    a = run(1.9, 0.0, ddiv * dt, c, h, vs, dt)
    assert np.all(a > loc) and np.all(a < 1.9)
    np.testing.assert_allclose(a, loc + (1.9 - loc) * math.exp(-0.05 * c * dt / H), rtol=1e-14)


def test_degenerate_cases():
    # no signal velocity and no compression: alpha_loc = 0, plain decay
    a = run(0.5, 1.0, 1.0, 1.0, 0.1, 0.0, 1e-3)
    np.testing.assert_allclose(a, 0.5 * math.exp(-0.05 * 1e-3 / (P.gamma_k * 0.1)), rtol=1e-15)
    # compression with v_sig = 0: alpha_loc = alpha_max
    a = run(0.5, 0.0, -1.0, 1.0, 0.1, 0.0, 1e-3)
    assert np.all(a == GOLD["alpha_v_max"]["value"])
    # no sound speed: nothing decays
    a = run(0.7, 0.0, 0.0, 0.0, 0.1, 1.0, 1e-3)
    assert np.all(a == 0.7)
