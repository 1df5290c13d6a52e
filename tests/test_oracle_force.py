"""Pins of the oracle's ghost and force passes.

Fixed by: exact momentum and energy conservation of the pairwise exchange,
lattice symmetry, continuum limits (pressure gradient -grad P / rho and the
PdV work -P/rho div v for smooth periodic fields), the Balsara switch's
shear/compression limits, special cases that switch terms off, Galilean and
rotation invariance, angular momentum, and brute force vs tree."""
import math

import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

P = oracle.Params()


def run(ps, recv=None, mode="brute", params=P):
    return oracle.fixed_h_step(ps, params, recv=recv, mode=mode)


def mom_energy(ps, r):
    m = ps.m.astype(np.float64)
    v = np.stack([ps.vx, ps.vy, ps.vz], 1).astype(np.float64)
    a = np.stack([r["ax"], r["ay"], r["az"]], 1)
    p = (m[:, None] * a).sum(0)
    scale_p = (m * np.linalg.norm(a, axis=1)).sum()
    e = (m * ((v * a).sum(1) + r["du"])).sum()
    scale_e = (m * (np.abs(v * a).sum(1) + np.abs(r["du"]))).sum()
    return p, scale_p, e, scale_e


@pytest.mark.parametrize("kind", ["lattice", "lognormal", "sedov"])
def test_momentum_and_energy_conserved(kind):
    if kind == "lattice":
        ps = inputs.lattice_box(12, 7, u="logu", sigma_v=0.3)
    elif kind == "lognormal":
        ps = inputs.lognormal_box(14, 2500, 2.0, 3, sigma_v=0.2)
    else:
        ps = inputs.sedov_box(12, 2, n_hot=8)
        ps.vx[:] = np.random.default_rng(0).normal(0, 0.5, ps.n)
    h, _, conv, _, _ = oracle.solve_h(ps, P, mode="brute")
    r = oracle.fixed_h_step(ps, P, mode="brute", h=h)
    p, sp, e, se = mom_energy(ps, r)
    assert np.abs(p).max() < 1e-13 * sp
    assert abs(e) < 1e-13 * se
    assert r["n_force_total"] >= r["n_dens_total"]


def test_perfect_lattice_at_rest_has_no_forces():
    ps = inputs.lattice_box(12, 0, jitter=0.0, sigma_v=0.0)
    r = run(ps)
    a = np.stack([r["ax"], r["ay"], r["az"]], 1)
    # compare with the size of a single pair term
    single = ps.m[0] * r["A"][0] * 40.0 / P.gamma_k ** 4 / float(ps.h[0]) ** 4
    assert np.abs(a).max() < 1e-12 * single
    assert np.all(r["du"] == 0.0)
    np.testing.assert_allclose(r["vsig"], 2 * r["c"], rtol=1e-15)


def test_uniform_u_switches_conduction_off_and_v0_switches_viscosity_off():
    ps = inputs.lattice_box(10, 4, sigma_v=0.05)  # u = 1 everywhere
    r1 = run(ps)
    q = ps.copy()
    q.alpha_c[:] = 0.0
    r2 = run(q)
    assert np.array_equal(r1["du"], r2["du"])
    ps = inputs.lattice_box(10, 5, u="logu", sigma_v=0.0)
    r1 = run(ps)
    q = ps.copy()
    q.alpha_v[:] = 0.0
    r2 = run(q)
    for k in ("ax", "ay", "az"):
        assert np.array_equal(r1[k], r2[k])
    # no relative motion: v_sig,ij = c_i + c_j, so v_sig,i = max(2 c_i, c_i + max_j c_j)
    assert np.all(r1["vsig"] >= 2 * r1["c"] * (1 - 1e-15))
    assert np.all(r1["vsig"] <= r1["c"] + r1["c"].max() + 1e-12)


def _sine_lattice(n_side, field, eps):
    ps = inputs.lattice_box(n_side, 0, jitter=0.0, sigma_v=0.0, alpha=False)
    ps.alpha_v[:] = 0.0
    ps.alpha_c[:] = 0.0
    x = ps.x.astype(np.float64)
    if field == "u":
        ps.u[:] = 1.0 + eps * np.sin(2 * math.pi * x)
    elif field == "vx":
        ps.vx[:] = eps * np.sin(2 * math.pi * x)
    elif field == "vx_shear":
        ps.vx[:] = eps * np.sin(2 * math.pi * ps.y.astype(np.float64))
    return ps, x


def test_pressure_gradient_continuum_limit():
    # u = 1 + eps sin(2 pi x) on a uniform lattice at rest: P = (gamma-1) u rho
    # so a_x -> -grad P / rho = -(gamma-1) 2 pi eps cos(2 pi x).
    eps = 0.05
    ps, x = _sine_lattice(24, "u", eps)
    r = run(ps, mode="tree")
    expect = -(P.gamma_gas - 1) * 2 * math.pi * eps * np.cos(2 * math.pi * x)
    amp = (P.gamma_gas - 1) * 2 * math.pi * eps
    assert np.abs(r["ax"] - expect).max() < 0.03 * amp
    assert np.abs(r["ay"]).max() < 1e-10 * amp and np.abs(r["az"]).max() < 1e-10 * amp


def test_compression_work_and_divergence_continuum_limit():
    # v_x = eps sin(2 pi x), uniform u, no dissipation: div v -> 2 pi eps
    # cos(2 pi x) and du/dt -> -(P/rho) div v = -(gamma-1) u div v. The lattice
    # estimate of a gradient at eta = 1.2348 is a few per cent low (the
    # lattice constant K of the linear-field test times the kernel smoothing
    # of the sine), hence 6 per cent.
    eps = 0.01
    ps, x = _sine_lattice(24, "vx", eps)
    r = run(ps, mode="tree")
    div = 2 * math.pi * eps * np.cos(2 * math.pi * x)
    amp = 2 * math.pi * eps
    assert np.abs(r["div_v"] - div).max() < 0.06 * amp
    du = -(P.gamma_gas - 1) * 1.0 * div
    assert np.abs(r["du"] - du).max() < 0.06 * (P.gamma_gas - 1) * amp
    # Exact identity between the two loops without dissipation:
    # du_i = sum_j m_j A_i g_i (v_ij . e) = -f_i (P_i / rho_i) (div v)_i.
    np.testing.assert_allclose(r["du"], -r["f"] * r["P"] / r["rho"] * r["div_v"],
                               rtol=1e-10, atol=1e-13 * amp)
    # compression without shear: Balsara switch near 1 where |div v| is large
    big = np.abs(np.cos(2 * math.pi * x)) > 0.7
    assert r["balsara"][big].min() > 0.9
    # pure shear: no divergence, the switch turns viscosity off
    ps, _ = _sine_lattice(24, "vx_shear", eps)
    r = run(ps, mode="tree")
    assert np.abs(r["div_v"]).max() < 1e-9 * amp
    assert r["balsara"].max() < 1e-6


def test_galilean_boost_and_rotation():
    ps = inputs.lattice_box(10, 9, u="logu", sigma_v=0.2)
    r1 = run(ps)
    q = ps.copy()
    q.vx += np.float32(0.5)
    q.vy -= np.float32(0.25)
    # v + V in float32 is exact only up to rounding: compare with the boosted
    # velocities' own differences by running both with the same float32 values
    r2 = run(q)
    q2 = q.copy()
    q2.vx -= np.float32(0.5)
    q2.vy += np.float32(0.25)
    r3 = run(q2)
    scale = np.abs(np.stack([r1["ax"], r1["ay"], r1["az"]])).max()
    for k in ("ax", "ay", "az"):
        np.testing.assert_allclose(r2[k], r3[k], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(r2["du"], r3["du"], rtol=0, atol=1e-12 * np.abs(r3["du"]).max())
    # rotation by 90 degrees about z: (x, y) -> (1 - y, x), (vx, vy) -> (-vy, vx)
    q = ps.copy()
    q.x = np.mod(1.0 - ps.y, 1.0)
    q.y = ps.x.copy()
    q.vx = -ps.vy
    q.vy = ps.vx.copy()
    r4 = run(q)
    np.testing.assert_allclose(r4["ax"], -r1["ay"], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(r4["ay"], r1["ax"], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(r4["az"], r1["az"], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(r4["du"], r1["du"], rtol=0, atol=1e-11 * np.abs(r1["du"]).max())


def test_angular_momentum_of_isolated_cluster():
    rng = np.random.default_rng(12)
    n = 1200
    pos = 0.5 + 0.08 * rng.standard_normal((n, 3))
    ps = inputs.uniform_random_box(n, 1, sigma_v=0.3)
    ps.x, ps.y, ps.z = (np.ascontiguousarray(pos[:, k]) for k in range(3))
    q = oracle.Params(periodic=False)
    h, _, _, _, _ = oracle.solve_h(ps, q, mode="brute")
    r = oracle.fixed_h_step(ps, q, mode="brute", h=h)
    a = np.stack([r["ax"], r["ay"], r["az"]], 1)
    m = ps.m.astype(np.float64)
    L = (m[:, None] * np.cross(pos, a)).sum(0)
    scale = (m * np.linalg.norm(pos, axis=1) * np.linalg.norm(a, axis=1)).sum()
    assert np.abs(L).max() < 1e-13 * scale


@pytest.mark.parametrize("kind", ["lattice", "lognormal"])
def test_force_tree_mode_is_bit_identical_to_brute_force(kind):
    if kind == "lattice":
        ps = inputs.lattice_box(10, 2, u="logu", sigma_v=0.1)
    else:
        ps = inputs.lognormal_box(14, 2500, 2.0, 5)
    h = np.minimum(ps.h.astype(np.float64), P.hmax())
    a = oracle.fixed_h_step(ps, P, mode="brute", h=h)
    b = oracle.fixed_h_step(ps, P, mode="tree", h=h)
    for k in ("ax", "ay", "az", "du", "vsig", "nforce", "rho", "nngb", "f", "balsara"):
        assert np.array_equal(a[k], b[k]), k


def test_sampled_receivers_match_full_evaluation():
    ps = inputs.lognormal_box(14, 2500, 2.0, 5)
    h = np.minimum(ps.h.astype(np.float64), P.hmax())
    full = oracle.fixed_h_step(ps, P, mode="brute", h=h)
    sub = np.array([0, 17, 999, 2000, ps.n - 1])
    s = oracle.fixed_h_step(ps, P, recv=sub, mode="tree", h=h)
    for k in ("ax", "ay", "az", "du", "vsig", "nforce", "rho", "nngb"):
        assert np.array_equal(s[k], full[k][sub]), k


def test_global_sums_of_a_lattice_step():
    ps = inputs.lattice_box(10, 3, u="logu", sigma_v=0.1)
    res = oracle.nr_step(ps, P, mode="brute")
    s = res["sums"]
    assert np.abs(s[:3]).max() < 1e-13 * s[4]
    assert abs(s[3]) < 1e-12 * (s[4] * 0.1 * 3 + s[5])
    assert res["converged"].all()
