"""GPU pressure-energy flavour (pressure-smoothed SPH of Appendix A) against
the oracle, output by output at the step's own h:

* the density loop's smoothed pressure P_hat and its h-derivative,
* the ghost's P = P_hat, c = sqrt(gamma P_hat / rho), its grad-h term F
  (sphx_ghost_out.A) and the rest of the ghost state,
* the force pass's pressure-energy accelerations and du/dt, and the FP64
  conservation sums,

for whole steps (h iteration), the fixed-h passes, other kernels and loop
shapes, the captured-step path (bit-identical to the pass-by-pass step) and
an active subset whose inactive sources keep an earlier step's state.

Tolerances: P_hat is a sum of positive terms (the rho tolerance); its
h-derivative is a difference of such sums, compared on the scale 3 P_hat / h
of its terms; F = h P_hat' / ((gamma - 1) n G') with G' = 3 + h n'/n takes
the P_hat' tolerance through that formula. On top of these, each sum carries
the FP32 rounding of u = r / H (below 1e-6 relative: a few ulp from the
cell-relative coordinates, the reciprocal square root and 1/H) times the
sensitivity of its terms to u, sum_j m_j u_j |u dT/du| with T the term's
kernel factor: negligible in a smooth medium, dominant where a source
thousands of times hotter than the receiver's other neighbours sits near the
edge of its support (the Sedov case), since the kernel's relative slope
grows without bound there. The rest as the density-energy flavour.
"""
import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

from helpers import RHO_TOL, check_density, check_force, check_ghost, gpu_fixed_h, gpu_step

pytestmark = pytest.mark.gpu
PPE = oracle.Params(flavour="pressure_energy")
FL = {"flavour": "pressure_energy"}


def unequal(ps, seed):
    """Unequal masses (the generated boxes have equal ones)."""
    rng = np.random.default_rng(seed)
    q = ps.copy()
    q.m = np.ascontiguousarray((rng.uniform(0.5, 1.5, ps.n) / ps.n).astype(np.float32))
    return q


CASES = {
    "lattice16_logu": lambda: inputs.config_small(1, u="logu"),
    "lognormal_6000_unequal_m": lambda: unequal(
        inputs.lognormal_box(16, 6000, 2.0, 61, sigma_v=0.3), 3),
    "sedov16": lambda: inputs.sedov_box(16, 2, n_hot=8),
}


U_ROUND = 1e-6  # bound on the FP32 relative rounding of u = r / H


def sensitivity(ps, h, params, recv):
    """Per receiver, (gamma - 1) sum_j m_j u_j |u dT/du| over its density
    neighbours for T = W and T = dW/dh (at the receiver's h), by central
    differences of the oracle's kernel in r."""
    h = np.asarray(h, np.float64)
    off, idx = oracle.density_candidates(ps, h, params, recv)
    k = np.repeat(np.arange(len(recv)), np.diff(off))
    i = np.asarray(recv)[k]
    pos = np.stack([ps.x, ps.y, ps.z], 1)
    d = pos[i] - pos[idx]
    b = np.asarray(ps.box)
    d -= b * np.round(d / b)
    r = np.sqrt((d * d).sum(1))
    keep = r < params.gamma_k * h[i]
    k, i, idx, r = k[keep], i[keep], idx[keep], r[keep]
    e = 1e-6
    wp, _, dp = oracle.kernel(params.kernel, r * (1 + e), h[i], params.gamma_k)
    wm, _, dm = oracle.kernel(params.kernel, r * (1 - e), h[i], params.gamma_k)
    mu = ps.m[idx].astype(np.float64) * ps.u[idx].astype(np.float64)
    gm1 = params.gamma_gas - 1.0
    sw = np.bincount(k, gm1 * mu * np.abs(wp - wm) / (2 * e), minlength=len(recv))
    sd = np.bincount(k, gm1 * mu * np.abs(dp - dm) / (2 * e), minlength=len(recv))
    return sw, sd


def check_pressure(g, ref, recv, h, where, ps, params=PPE):
    recv = np.asarray(recv)
    gm1 = params.gamma_gas - 1.0
    hh = np.asarray(h, np.float64)[recv]
    sw, sd = sensitivity(ps, h, params, recv)
    tol_dh = 2 * RHO_TOL * 3.0 * ref["P_hat"] / hh + U_ROUND * sd
    tol_P = 2 * RHO_TOL * ref["P_hat"] + U_ROUND * sw
    if "P_hat" in g:
        a = g["P_hat"][recv].astype(np.float64)
        tol = tol_P
        err = np.abs(a - ref["P_hat"])
        assert np.all(err <= tol), "%s P_hat: %d mismatches, worst %.3g of tolerance" % (
            where, int((err > tol).sum()), (err / tol).max())
        err = np.abs(g["P_hat_dh"][recv] - ref["P_hat_dh"])
        assert np.all(err <= tol_dh), "%s P_hat_dh: %d mismatches, worst %.3g of tolerance" % (
            where, int((err > tol_dh).sum()), (err / tol_dh).max())
    # F = h P_hat' / ((gamma - 1) n G'): the P_hat' tolerance through it
    gp = 3.0 + hh * ref["n_dh"] / ref["n"]
    F, Fr = g["A"][recv].astype(np.float64), ref["A"]
    # (a particle alone in its support at a fixed h has G' = 0: F is a pole)
    ok = np.isfinite(Fr) & (gp > 1e-3)
    tol = (2 * RHO_TOL * np.abs(Fr) + hh * tol_dh / (gm1 * ref["n"] * np.abs(gp)))[ok]
    err = np.abs(F - Fr)[ok]
    assert np.all(err <= tol), "%s F: %d mismatches, worst %.3g of tolerance" % (
        where, int((err > tol).sum()), (err / tol).max())
    return tol_P


def run_and_check(ps, params, where, fixed=False):
    """One step (or the fixed-h passes) of a smoothed-pressure flavour
    (params["flavour"]) against the oracle at the step's own h."""
    if fixed:
        g = gpu_fixed_h(ps, params=params)
        h = ps.h.astype(np.float64)
    else:
        g = gpu_step(ps, params=params)
        assert g["status"] >= 0 and g["info"].unconverged == 0
        h = g["h"].astype(np.float64)
    pk = oracle.Params.with_kernel(params.get("kernel", PPE.kernel), flavour=params["flavour"])
    ref = oracle.fixed_h_step(ps, pk, h=h)
    recv = np.arange(ps.n)
    check_density(g, ref, ps, h, recv, pk, where)
    tol_P = check_pressure(g, ref, recv, h, where, ps, pk)
    check_ghost(g, ref, recv, where, A=False, P_tol=tol_P)
    check_force(g, ref, ps, h, recv, pk, where)
    return g, ref


@pytest.mark.parametrize("case", sorted(CASES))
def test_pressure_energy_step_matches_oracle(case):
    ps = CASES[case]()
    if case == "sedov16":
        ps.vx[:] = np.random.default_rng(5).normal(0, 0.5, ps.n).astype(np.float32)
    print("pressure-energy step:", case, "N=%d" % ps.n, flush=True)
    g, ref = run_and_check(ps, FL, "pressure-energy %s at its h" % case)
    s_ref = oracle.sums(ps.m, ps.vx, ps.vy, ps.vz, ref["ax"], ref["ay"], ref["az"], ref["du"])
    s = g["sums"]
    assert np.abs(s[:3]).max() < 2e-5 * s[4]
    np.testing.assert_allclose(s[4:], s_ref[4:], rtol=1e-4)
    assert abs(s[3] - s_ref[3]) <= 1e-4 * (s_ref[4] * 1.0 + s_ref[5])


def test_pressure_energy_fixed_h_passes_match_oracle():
    ps = unequal(inputs.lognormal_box(16, 6000, 2.0, 62, sigma_v=0.3), 4)
    print("pressure-energy fixed-h passes N=%d" % ps.n, flush=True)
    run_and_check(ps, FL, "pressure-energy fixed h", fixed=True)


@pytest.mark.parametrize("kernel,shape", [
    ("cubic_spline", {"density_tile": 64, "density_waves": 2, "force_tile": 128}),
    ("quintic_spline", {"density_tile": 256, "density_waves": 1, "force_waves": 2}),
    ("wendland_c4", {"density_tile": 128, "density_waves": 2}),
])
def test_pressure_energy_other_kernels_and_shapes(kernel, shape):
    ps = unequal(inputs.lognormal_box(12, 3000, 2.0, 63, sigma_v=0.3), 5)
    params = dict(FL, kernel=kernel, **shape)
    print("pressure-energy", kernel, shape, "N=%d" % ps.n, flush=True)
    run_and_check(ps, params, "pressure-energy %s %s" % (kernel, shape))


def test_pressure_energy_captured_step_is_bit_identical():
    ps = unequal(inputs.lognormal_box(16, 6000, 2.0, 64, sigma_v=0.3), 6)
    print("pressure-energy captured step N=%d" % ps.n, flush=True)
    a = gpu_step(ps, params=FL)
    b = gpu_step(ps, params=dict(FL, graph_passes=4))
    assert a["status"] >= 0 and b["status"] >= 0
    for k in ("h", "rho", "P_hat", "P", "c", "A", "f", "ax", "ay", "az", "du_dt", "v_sig"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    np.testing.assert_array_equal(a["sums"], b["sums"])


def test_pressure_energy_active_subset_step():
    """Inactive sources keep an earlier all-active step's P_hat and F; their
    (gamma - 1)^2 u / P_hat is formed from the caller's current u."""
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lognormal_box(16, 5000, 2.0, 22, time_bins=(0.1, 0.2, 0.3, 0.4))
    act = ps.active.astype(bool)
    all_on = ps.copy()
    all_on.active = None
    print("pressure-energy active subset N=%d active=%d" % (ps.n, act.sum()), flush=True)
    ctx = sphx.Context(sphx.default_params(**FL), 0)
    dp = sphx.DeviceParticles.from_set(all_on)
    out = sphx.Outputs(ps.n, pressure=True)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    st1, _ = sphx.step(ctx, grid, tasks, dp, out)
    assert st1 >= 0
    h1 = dp.t["h"].cpu().numpy()
    dp.t["active"] = torch.from_numpy(ps.active).cuda()
    q = ps.copy()
    q.h = h1.copy()
    q.u = q.u * np.float32(1.5)
    dp.t["u"] = torch.from_numpy(q.u).cuda()
    grid2 = sphx.Grid(ctx, dp)
    tasks2 = sphx.Tasks(ctx, grid2, dp)
    st, info = sphx.step(ctx, grid2, tasks2, dp, out)
    torch.cuda.synchronize()
    assert st >= 0 and info.unconverged == 0
    g = {k: v.cpu().numpy() for k, v in {**out.d, **out.g, **out.f}.items()}
    hg = dp.t["h"].cpu().numpy().astype(np.float64)
    ridx = np.nonzero(act)[0]
    assert np.array_equal(hg[~act], h1[~act])
    # the oracle at the step's own h: inactive sources at h1 with the step-1
    # u, receivers at their final h with the new u
    s1 = oracle.fixed_h_step(ps, PPE, h=h1.astype(np.float64), mode="tree")
    d2 = oracle.density(q, hg, PPE, recv=ridx, mode="tree")
    g2 = oracle.ghost(d2, q.u[ridx], hg[ridx], PPE)
    state = {k: s1[k].copy() for k in ("P", "c", "f", "balsara", "A")}
    rho = s1["rho"].copy()
    rho[ridx] = d2["rho"]
    for k in state:
        state[k][ridx] = g2[k]
    fo = oracle.force(q, hg, state, rho, PPE, recv=ridx, mode="tree")
    ref = {**{k: v for k, v in d2.items() if k != "total"}, **g2,
           **{k: v for k, v in fo.items() if k != "total"}}
    g["du"], g["vsig"] = g["du_dt"], g["v_sig"]
    where = "pressure-energy active step at its h"
    check_density(g, ref, q, hg, ridx, PPE, where)
    tol_P = check_pressure(g, ref, ridx, hg, where, q)
    check_ghost(g, ref, ridx, where, A=False, P_tol=tol_P)
    check_force(g, ref, q, hg, ridx, PPE, where)
