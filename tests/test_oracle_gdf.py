"""Oracle pins of the Gasoline-2-like (GDF) flavour (Appendix A): the
geometric density average correction f, the conduction parameter from the
trace-free shear tensor, and the GDF equations of motion, against what the
paper and the mathematics fix:

* the printed conduction constant C = 0.03;
* f = 1 where every neighbour has the receiver's density, and f = lambda
  where every neighbour's density is lambda times the receiver's (the ratio's
  orientation);
* for v = A x on a cubic lattice the velocity-gradient tensor is A exactly
  (cubic symmetry), so alpha_c = C |S(A)| h^2 in closed form, and 0 for a pure
  rotation and for an isotropic compression (the symmetrisation and the trace
  removal);
* on a uniform lattice with one h the GDF forces equal the density-energy
  ones with f = 1 (the two equations of motion coincide there);
* momentum and total energy are conserved by the pair exchange, conduction
  included, and conduction carries heat from hot to cold.
"""
import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

P = oracle.Params()


def gdf_state(ps, params, alpha_c=None):
    """Density at the set's h, ghost, the GDF correction and conduction
    parameter: the force pass's inputs (the GDF f replaces the grad-h f)."""
    d = oracle.density(ps, ps.h, params)
    g = oracle.ghost(d, ps.u, ps.h, params)
    f, ac = oracle.gdf(ps, ps.h, d["rho"], params)
    g = dict(g)
    g["f"] = f
    return d, g, f, ac if alpha_c is None else np.full(ps.n, alpha_c)


def test_constant_is_the_printed_one():
    assert oracle.GDF_C == 0.03


def test_uniform_lattice_correction_is_one():
    ps = inputs.lattice_box(10, 1, jitter=0.0)
    d = oracle.density(ps, ps.h, P)
    f, _ = oracle.gdf(ps, ps.h, d["rho"], P)
    assert np.allclose(f, 1.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("lam", [0.5, 3.0])
def test_correction_is_the_density_ratio(lam):
    """Every neighbour's density lambda times the receiver's: f = lambda (the
    inverse orientation of the ratio would give 1/lambda)."""
    ps = inputs.lognormal_box(8, 600, 2.0, 3)
    rho = np.full(ps.n, lam)
    recv = np.array([5, 77, 301])
    rho[recv] = 1.0
    for i in recv:
        f, _ = oracle.gdf(ps, ps.h, np.where(np.arange(ps.n) == i, 1.0, lam), P, recv=[i])
        assert f[0] == pytest.approx(lam, rel=1e-12)


def linear_flow(A):
    """A cubic lattice (no jitter) in an open unit box with v = A x; the
    receivers whose support lies inside the box."""
    ps = inputs.lattice_box(16, 2, jitter=0.0, sigma_v=0.0)
    x = np.stack([ps.x, ps.y, ps.z], 1)
    v = x @ np.asarray(A, np.float64).T
    ps.vx, ps.vy, ps.vz = v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()
    p = oracle.Params(periodic=False)
    H = p.gamma_k * float(ps.h[0])
    inner = np.nonzero(np.all((x > H + 1e-9) & (x < 1.0 - H - 1e-9), axis=1))[0]
    assert inner.size > 100
    d = oracle.density(ps, ps.h, p)
    return ps, p, d, inner


def shear_norm(A):
    A = np.asarray(A, np.float64)
    S = 0.5 * (A + A.T) - np.eye(3) * np.trace(A) / 3.0
    return np.sqrt((S * S).sum())


@pytest.mark.parametrize("A", [
    [[0.3, 1.0, 0.0], [0.2, -0.1, 0.5], [0.0, 0.4, 0.7]],
    [[0.0, 2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]],
])
def test_conduction_parameter_of_a_linear_flow(A):
    ps, p, d, inner = linear_flow(A)
    _, ac = oracle.gdf(ps, ps.h, d["rho"], p, recv=inner)
    want = oracle.GDF_C * shear_norm(A) * float(ps.h[0]) ** 2
    assert np.allclose(ac, want, rtol=1e-10, atol=0)


@pytest.mark.parametrize("A", [
    [[0.0, 1.0, -0.5], [-1.0, 0.0, 2.0], [0.5, -2.0, 0.0]],   # a rotation
    [[-0.7, 0.0, 0.0], [0.0, -0.7, 0.0], [0.0, 0.0, -0.7]],   # isotropic compression
])
def test_rotation_and_isotropic_compression_have_no_shear(A):
    ps, p, d, inner = linear_flow(A)
    _, ac = oracle.gdf(ps, ps.h, d["rho"], p, recv=inner)
    scale = oracle.GDF_C * np.abs(np.asarray(A)).max() * float(ps.h[0]) ** 2
    assert np.all(np.abs(ac) < 1e-10 * scale)


def test_uniform_lattice_forces_equal_density_energy():
    """One h, one u, one density: (P_i + P_j) G / (2 rho_i rho_j) is the
    density-energy P_i g_i / rho_i^2 + P_j g_j / rho_j^2 with f = 1."""
    ps = inputs.lattice_box(10, 4, jitter=0.0, sigma_v=0.05)
    ps.alpha_c[:] = 0.0
    pg = oracle.Params(flavour="gdf")
    d, g, f, ac = gdf_state(ps, pg, alpha_c=0.0)
    ps.alpha_c[:] = ac
    gg = oracle.force(ps, ps.h, g, d["rho"], pg)
    g0 = dict(g)
    g0["f"] = np.ones(ps.n)
    ge = oracle.force(ps, ps.h, g0, d["rho"], P)
    scale = max(np.abs(ge["ax"]).max(), 1e-30)
    for k in ("ax", "ay", "az"):
        assert np.allclose(gg[k], ge[k], rtol=0, atol=1e-10 * scale)
    dscale = max(np.abs(ge["du"]).max(), 1e-30)
    assert np.allclose(gg["du"], ge["du"], rtol=0, atol=1e-10 * dscale)


def test_conservation_with_conduction():
    ps = inputs.lognormal_box(8, 1500, 2.0, 11)
    pg = oracle.Params(flavour="gdf")
    h, _, conv, _, _ = oracle.solve_h(ps, pg)
    ps.h = h.astype(np.float32)
    d, g, f, ac = gdf_state(ps, pg)
    ps.alpha_c = ac.astype(np.float32)
    assert np.all(ac > 0) and np.any(np.abs(f - 1.0) > 0.05)
    o = oracle.force(ps, ps.h, g, d["rho"], pg)
    s = oracle.sums(ps.m, ps.vx, ps.vy, ps.vz, o["ax"], o["ay"], o["az"], o["du"])
    assert np.abs(s[:3]).max() < 1e-12 * s[4]
    assert abs(s[3]) < 1e-12 * (s[4] + s[5])


def test_conduction_carries_heat_from_hot_to_cold():
    ps = inputs.lattice_box(10, 5, jitter=0.0, sigma_v=0.0)
    hot = ps.x < 0.5
    ps.u = np.where(hot, 2.0, 1.0).astype(np.float32)
    pg = oracle.Params(flavour="gdf")
    d, g, f, _ = gdf_state(ps, pg, alpha_c=0.0)
    ps.alpha_c[:] = 0.01
    o = oracle.force(ps, ps.h, g, d["rho"], pg)
    # at rest the pressure terms leave u alone (v_ij = 0): du is conduction only
    edge = np.abs(o["du"]) > 1e-9 * np.abs(o["du"]).max()
    assert np.all(o["du"][hot & edge] < 0) and np.all(o["du"][~hot & edge] > 0)
    assert abs((ps.m * o["du"]).sum()) < 1e-12 * (ps.m * np.abs(o["du"])).sum()


def linear_flow_with_gradient(A, g):
    """linear_flow with u = 1 + g . x: the pressure gradient points along g
    on the lattice (the kernel sum of a linear field is isotropic)."""
    ps, p, d, inner = linear_flow(A)
    x = np.stack([ps.x, ps.y, ps.z], 1)
    ps.u = (1.0 + x @ np.asarray(g, np.float64)).astype(np.float32)
    return ps, p, inner


@pytest.mark.parametrize("A,g", [
    ([[0.3, 1.0, 0.0], [0.2, -0.1, 0.5], [0.0, 0.4, 0.7]], [0.2, -0.1, 0.3]),
    ([[-0.9, 0.1, 0.0], [0.3, -0.4, 0.2], [0.0, 0.1, -0.5]], [0.0, 0.0, 0.4]),
])
def test_shock_detector_of_a_linear_flow(A, g):
    """D = 3/2 [n.A.n + max(-tr A / 3, 0)] with n along g: the detector's
    projection on the pressure gradient and its compression term (a wrong
    sign of the gradient or a dropped max fails one of the two flows)."""
    ps, p, inner = linear_flow_with_gradient(A, g)
    D = oracle.gdf_detector(ps, ps.h, p, recv=inner)
    A = np.asarray(A, np.float64)
    n = np.asarray(g, np.float64) / np.linalg.norm(g)
    want = 1.5 * (n @ A @ n + max(-np.trace(A) / 3.0, 0.0))
    # (u is stored in FP32: the gradient's direction carries its rounding)
    assert np.allclose(D, want, rtol=2e-5, atol=1e-12)


def test_switch_closed_form_and_limits():
    """The viscosity parameter: an immediate rise to alpha_loc, else the
    linear relaxation integrated exactly (closed form); no source where D
    grows; alpha_loc -> alpha_max for a collapse much faster than
    v_sig^2 / h^2."""
    rng = np.random.default_rng(7)
    n = 500
    a0 = rng.uniform(0, 2, n)
    Dold = rng.normal(0, 5, n)
    Dnew = rng.normal(0, 5, n)
    c = rng.uniform(0.5, 2, n)
    h = rng.uniform(0.01, 0.05, n)
    vs = rng.uniform(1, 3, n)
    B = rng.uniform(0, 1, n)
    dt = 1e-3
    a = oracle.gdf_alpha_v_update(a0, Dold, Dnew, c, h, vs, B, dt)
    A = 2 * h * h * B * np.maximum(-(Dnew - Dold) / dt, 0)
    loc = 2.0 * A / (A + vs * vs)
    want = np.where(loc > a0, loc, loc + (a0 - loc) * np.exp(-0.2 * c * dt / h))
    assert np.allclose(a, want, rtol=1e-13, atol=0)
    assert (loc > a0).sum() > 50 and (loc < a0).sum() > 50  # both branches
    # D growing: pure decay
    a = oracle.gdf_alpha_v_update(a0, Dold, Dold + 1.0, c, h, vs, B, dt)
    assert np.allclose(a, a0 * np.exp(-0.2 * c * dt / h), rtol=1e-13)
    # a collapse: alpha_loc close to alpha_max, reached after many decay times
    a = oracle.gdf_alpha_v_update(np.zeros(n), Dold, Dold - 1e15, c, h, vs, np.ones(n), dt)
    assert np.allclose(a, 2.0, rtol=1e-6)
