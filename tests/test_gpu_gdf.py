"""GPU GDF flavour (the Gasoline-2-like flavour of Appendix A) against the
oracle:

* the GDF loop alone (sphx_gdf): the geometric-density correction f and
  the conduction parameter alpha_c = C |S| h^2, given the GPU's own h and rho
  (their parity is checked by the step tests);
* whole steps: the h iteration, then f and alpha_c formed inside the step,
  and the GDF forces with the conduction term, against the oracle's chain
  (density, ghost, GDF quantities, force) at the step's own h;
* the standalone force pass fed with the step's f and alpha_c repeats the
  step's forces bitwise, and a captured step repeats the pass-by-pass one;
* an active subset, whose inactive sources keep their previous f and
  alpha_c, against the oracle at the step's own h;
* the loop with other kernels of the family.
"""
import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

from helpers import check_density, check_force, gpu_step, rms

pytestmark = pytest.mark.gpu
PG = oracle.Params(flavour="gdf")
FL = {"flavour": "gdf"}
GDF_TOL = 1e-4

CASES = {
    "lattice16_shear": lambda: inputs.lattice_box(16, 52, u="logu", sigma_v=0.2),
    "lognormal_6000": lambda: inputs.lognormal_box(16, 6000, 2.0, 61, sigma_v=0.3),
    "sedov16": lambda: inputs.sedov_box(16, 2, n_hot=8),
}


def check_gdf(f, ac, f_ref, ac_ref, where):
    """f: a ratio of sums of positive terms, relative error. alpha_c: the
    norm of a sum with cancellation, on the scale max(|ref|, rms(ref))."""
    e = np.abs(f.astype(np.float64) - f_ref)
    assert np.all(e <= GDF_TOL * np.abs(f_ref)), "%s f: %d mismatches, worst %.3g" % (
        where, int((e > GDF_TOL * np.abs(f_ref)).sum()), (e / np.abs(f_ref)).max())
    s = np.maximum(np.abs(ac_ref), rms(ac_ref)) + 1e-30
    e = np.abs(ac.astype(np.float64) - ac_ref)
    assert np.all(e <= GDF_TOL * s), "%s alpha_c: %d mismatches, worst %.3g" % (
        where, int((e > GDF_TOL * s).sum()), (e / s).max())


def oracle_chain(ps, h):
    """Density, ghost, GDF f and alpha_c and the GDF force at the given h."""
    d = oracle.density(ps, h, PG)
    g = dict(oracle.ghost(d, ps.u, h, PG))
    f, ac = oracle.gdf(ps, h, d["rho"], PG)
    g["f"] = f
    q = ps.copy()
    q.alpha_c = ac.astype(np.float32)
    fo = oracle.force(q, h, g, d["rho"], PG)
    ref = {k: v for k, v in d.items() if k != "total"}
    ref.update({k: v for k, v in fo.items() if k != "total"})
    return ref, f, ac


@pytest.mark.parametrize("case", ["lognormal", "lattice_shear"])
def test_gdf_loop_matches_oracle(case):
    import torch
    from paper_2305_13380_amd import sphx
    if case == "lognormal":
        ps = inputs.lognormal_box(16, 6000, 2.0, 71, sigma_v=0.3)
    else:
        ps = inputs.lattice_box(16, 72, u="logu", sigma_v=0.2)
    print("gdf loop: %s N=%d" % (case, ps.n), flush=True)
    ctx = sphx.Context(sphx.default_params(), 0)
    dp = sphx.DeviceParticles.from_set(ps)
    out = sphx.Outputs(ps.n)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    st, _ = sphx.step(ctx, grid, tasks, dp, out)
    assert st >= 0
    f, ac = sphx.gdf(ctx, grid, tasks, dp, out.d["rho"])
    torch.cuda.synchronize()
    h = dp.t["h"].cpu().numpy().astype(np.float64)
    rho = out.d["rho"].cpu().numpy().astype(np.float64)
    f_ref, ac_ref = oracle.gdf(ps, h, rho, PG)
    if case == "lognormal":
        assert np.abs(f_ref - 1.0).max() > 1e-2  # a correction that is not trivial
    assert ac_ref.min() > 0.0
    check_gdf(f.cpu().numpy(), ac.cpu().numpy(), f_ref, ac_ref, "gdf loop %s" % case)


@pytest.mark.parametrize("case", sorted(CASES))
def test_gdf_step_matches_oracle(case):
    ps = CASES[case]()
    if case == "sedov16":
        ps.vx[:] = np.random.default_rng(5).normal(0, 0.5, ps.n).astype(np.float32)
    print("gdf flavour step:", case, "N=%d" % ps.n, flush=True)
    g = gpu_step(ps, params=FL)
    assert g["status"] >= 0 and g["info"].unconverged == 0
    h = g["h"].astype(np.float64)
    ref, f_ref, ac_ref = oracle_chain(ps, h)
    recv = np.arange(ps.n)
    where = "gdf %s at its h" % case
    check_density(g, ref, ps, h, recv, PG, where)
    # the step returns the GDF f in f and alpha_c in A
    check_gdf(g["f"], g["A"], f_ref, ac_ref, where)
    check_force(g, ref, ps, h, recv, PG, where)
    s_ref = oracle.sums(ps.m, ps.vx, ps.vy, ps.vz, ref["ax"], ref["ay"], ref["az"], ref["du"])
    s = g["sums"]
    assert np.abs(s[:3]).max() < 2e-5 * s[4]
    np.testing.assert_allclose(s[4:], s_ref[4:], rtol=1e-4)
    assert abs(s[3] - s_ref[3]) <= 1e-4 * (s_ref[4] * 1.0 + s_ref[5])


def test_gdf_conduction_is_on():
    """The conduction term changes du/dt where u varies (the step's du/dt
    differs from the oracle's with alpha_c = 0 by far more than the
    tolerance), so the step's alpha_c reaches the force pass."""
    ps = CASES["lattice16_shear"]()
    g = gpu_step(ps, params=FL)
    h = g["h"].astype(np.float64)
    ref, f_ref, _ = oracle_chain(ps, h)
    d = oracle.density(ps, h, PG)
    gs = dict(oracle.ghost(d, ps.u, h, PG))
    gs["f"] = f_ref
    q = ps.copy()
    q.alpha_c = np.zeros(ps.n, np.float32)
    fo0 = oracle.force(q, h, gs, d["rho"], PG)
    gap = np.abs(ref["du"] - fo0["du"])
    assert gap.max() > 100 * GDF_TOL * rms(ref["du"])
    e = np.abs(g["du_dt"] - ref["du"])
    assert e.max() < 0.01 * gap.max()


def test_gdf_force_alone_and_captured_step_repeat_the_step():
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lognormal_box(16, 6000, 2.0, 73, sigma_v=0.3)
    print("gdf standalone force and captured step N=%d" % ps.n, flush=True)
    ctx = sphx.Context(sphx.default_params(**FL), 0)
    dp = sphx.DeviceParticles.from_set(ps)
    out = sphx.Outputs(ps.n)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    st, _ = sphx.step(ctx, grid, tasks, dp, out)
    assert st >= 0
    torch.cuda.synchronize()
    a = {k: v.cpu().numpy().copy() for k, v in {**out.g, **out.f}.items()}
    # the force pass alone, from the step's f and alpha_c (in f and A)
    sphx.force(ctx, grid, tasks, dp, out)
    torch.cuda.synchronize()
    for k in ("ax", "ay", "az", "du_dt", "v_sig"):
        np.testing.assert_array_equal(out.f[k].cpu().numpy(), a[k], err_msg=k)
    b = gpu_step(ps, params=FL)
    c = gpu_step(ps, params=dict(FL, graph_passes=4))
    for k in ("h", "f", "A", "ax", "ay", "az", "du_dt", "v_sig"):
        np.testing.assert_array_equal(b[k], c[k], err_msg=k)


def test_gdf_active_subset_step():
    """Only active particles receive. Inactive ones are sources that keep the
    state of a previous all-active step, including their GDF f and alpha_c
    (read back from sphx_ghost_out.f and .A). Every output of the active
    step is checked against the oracle at the step's own h: the receivers at
    their final h with the new u, the inactive sources at their step-1 h."""
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lognormal_box(16, 5000, 2.0, 23, sigma_v=0.3,
                              time_bins=(0.1, 0.2, 0.3, 0.4))
    print("gdf active subset N=%d" % ps.n, flush=True)
    act = ps.active.astype(bool)
    all_on = ps.copy()
    all_on.active = None
    ctx = sphx.Context(sphx.default_params(**FL), 0)
    dp = sphx.DeviceParticles.from_set(all_on)
    out = sphx.Outputs(ps.n)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    st1, _ = sphx.step(ctx, grid, tasks, dp, out)
    assert st1 >= 0
    h1 = dp.t["h"].cpu().numpy()
    step1 = {k: v.cpu().numpy() for k, v in {**out.d, **out.g, **out.f}.items()}
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
    g["du"], g["vsig"] = g["du_dt"], g["v_sig"]
    hg = dp.t["h"].cpu().numpy().astype(np.float64)
    ridx = np.nonzero(act)[0]
    for k in g:  # the inactive particles' outputs are untouched
        if k in step1:
            assert np.array_equal(g[k][~act], step1[k][~act]), k
    # the oracle: step-1 state of everything at h1 with the step-1 u
    h1d = h1.astype(np.float64)
    d1 = oracle.density(ps, h1d, PG)
    s1 = dict(oracle.ghost(d1, ps.u, h1d, PG))
    f1, ac1 = oracle.gdf(ps, h1d, d1["rho"], PG)
    # the receivers at their final h with the new u
    d2 = oracle.density(q, hg, PG, recv=ridx)
    g2 = oracle.ghost(d2, q.u[ridx], hg[ridx], PG)
    rho = d1["rho"].copy()
    rho[ridx] = d2["rho"]
    f2, ac2 = oracle.gdf(q, hg, rho, PG, recv=ridx)
    state = {k: s1[k].copy() for k in ("P", "c", "balsara")}
    for k in state:
        state[k][ridx] = g2[k]
    state["f"] = f1.copy()
    state["f"][ridx] = f2
    qa = q.copy()
    ac = ac1.copy()
    ac[ridx] = ac2
    qa.alpha_c = ac.astype(np.float32)
    fo = oracle.force(qa, hg, state, rho, PG, recv=ridx)
    ref = {**{k: v for k, v in d2.items() if k != "total"}, **g2,
           **{k: v for k, v in fo.items() if k != "total"}}
    where = "gdf active step at its h"
    check_density(g, ref, q, hg, ridx, PG, where)
    check_gdf(g["f"][ridx], g["A"][ridx], f2, ac2, where)
    check_force(g, ref, q, hg, ridx, PG, where)


@pytest.mark.parametrize("name", ["wendland_c6", "cubic_spline", "quintic_spline"])
def test_gdf_loop_other_kernels(name):
    """The GDF loop with the other kernels of the family (the bare w(u) of
    each, its normalisation cancelling), at the step's own h and rho."""
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lognormal_box(16, 6000, 2.0, 75, sigma_v=0.3)
    print("gdf loop, kernel %s N=%d" % (name, ps.n), flush=True)
    P = oracle.Params.with_kernel(name, flavour="gdf")
    ctx = sphx.Context(sphx.default_params(kernel=name, **FL), 0)
    dp = sphx.DeviceParticles.from_set(ps)
    out = sphx.Outputs(ps.n)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    st, _ = sphx.step(ctx, grid, tasks, dp, out)
    assert st >= 0
    f, ac = sphx.gdf(ctx, grid, tasks, dp, out.d["rho"])
    torch.cuda.synchronize()
    h = dp.t["h"].cpu().numpy().astype(np.float64)
    rho = out.d["rho"].cpu().numpy().astype(np.float64)
    f_ref, ac_ref = oracle.gdf(ps, h, rho, P)
    check_gdf(f.cpu().numpy(), ac.cpu().numpy(), f_ref, ac_ref, "gdf loop %s" % name)
    # the step's own f and alpha_c are the loop's (the same inputs)
    np.testing.assert_array_equal(out.g["f"].cpu().numpy(), f.cpu().numpy())
    np.testing.assert_array_equal(out.g["A"].cpu().numpy(), ac.cpu().numpy())


@pytest.mark.parametrize("frac", [0.03, 0.4])
def test_gdf_loop_sparse_active(frac):
    """The GDF loop for a sparse set of active receivers (cells with few of
    them give each several lanes, whose sums meet in a butterfly)."""
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lognormal_box(16, 6000, 2.0, 77, sigma_v=0.3)
    print("gdf loop, active fraction %g N=%d" % (frac, ps.n), flush=True)
    ctx = sphx.Context(sphx.default_params(), 0)
    dp = sphx.DeviceParticles.from_set(ps)
    out = sphx.Outputs(ps.n)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    st, _ = sphx.step(ctx, grid, tasks, dp, out)
    assert st >= 0
    act = (np.random.default_rng(78).uniform(size=ps.n) < frac).astype(np.uint8)
    dp.t["active"] = torch.from_numpy(act).cuda()
    f, ac = sphx.gdf(ctx, grid, tasks, dp, out.d["rho"])
    torch.cuda.synchronize()
    h = dp.t["h"].cpu().numpy().astype(np.float64)
    rho = out.d["rho"].cpu().numpy().astype(np.float64)
    recv = np.nonzero(act)[0]
    f_ref, ac_ref = oracle.gdf(ps, h, rho, PG, recv=recv)
    fg, acg = f.cpu().numpy(), ac.cpu().numpy()
    check_gdf(fg[recv], acg[recv], f_ref, ac_ref, "gdf loop, active %g" % frac)
    assert np.all(np.isnan(fg[act == 0])) and np.all(np.isnan(acg[act == 0]))


def test_gdf_detector_matches_oracle():
    """The shock detector D of sphx_gdf against the oracle at the GPU's h, on
    a jittered lattice in an open box with u = 1 + g . x (a pressure gradient
    whose direction the sums fix well) and random velocities; receivers whose
    support lies inside the box."""
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lattice_box(16, 79, jitter=0.1, sigma_v=0.3)
    x = np.stack([ps.x, ps.y, ps.z], 1)
    ps.u = (1.0 + x @ np.array([0.3, -0.2, 0.4])).astype(np.float32)
    print("gdf detector N=%d" % ps.n, flush=True)
    ctx = sphx.Context(sphx.default_params(periodic=0), 0)
    dp = sphx.DeviceParticles.from_set(ps)
    out = sphx.Outputs(ps.n)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    st, _ = sphx.step(ctx, grid, tasks, dp, out)
    assert st >= 0
    _, _, D = sphx.gdf(ctx, grid, tasks, dp, out.d["rho"], detector=True)
    torch.cuda.synchronize()
    h = dp.t["h"].cpu().numpy().astype(np.float64)
    p = oracle.Params(periodic=False)
    H = p.gamma_k * h
    inner = np.nonzero(np.all((x > H[:, None]) & (x < 1.0 - H[:, None]), axis=1))[0]
    assert inner.size > 100
    ref = oracle.gdf_detector(ps, h, p, recv=inner)
    s = np.maximum(np.abs(ref), rms(ref))
    e = np.abs(D.cpu().numpy()[inner].astype(np.float64) - ref)
    assert np.all(e <= 1e-3 * s), "D: worst %.3g of its scale" % (e / s).max()
    assert (ref > 0).sum() > 10 and (ref < 0).sum() > 10  # both signs exercised


def test_gdf_switch_matches_oracle():
    import torch
    from paper_2305_13380_amd import sphx
    rng = np.random.default_rng(80)
    n = 30011
    a0 = rng.uniform(0, 2, n).astype(np.float32)
    Dold = rng.normal(0, 5, n).astype(np.float32)
    Dnew = (Dold + rng.normal(0, 5, n)).astype(np.float32)
    c = rng.uniform(0.5, 2, n).astype(np.float32)
    h = rng.uniform(0.01, 0.05, n).astype(np.float32)
    vs = rng.uniform(1, 3, n).astype(np.float32)
    B = rng.uniform(0, 1, n).astype(np.float32)
    act = (rng.uniform(size=n) < 0.7).astype(np.uint8)
    ctx = sphx.Context(sphx.default_params(**FL), 0)
    t = [torch.from_numpy(v).cuda() for v in (a0, Dold, Dnew, c, h, vs, B, act)]
    sphx.gdf_alpha_v_update(ctx, t[0], t[1], t[2], t[3], t[4], t[5], t[6], 1e-3, active=t[7])
    torch.cuda.synchronize()
    got = t[0].cpu().numpy().astype(np.float64)
    ref = oracle.gdf_alpha_v_update(a0, Dold, Dnew, c, h, vs, B, 1e-3)
    on = act == 1
    assert np.all(np.abs(got[on] - ref[on]) <= 2e-5 * np.abs(ref[on]) + 1e-7)
    assert np.array_equal(got[~on], a0[~on].astype(np.float64))


def test_gdf_sedov_run_conserves_energy():
    """A 24^3 blast over 40 leapfrog steps with the GDF flavour and its
    viscosity switch: the total energy is conserved, the switch stays within
    [0, 2] and rises at the shock, and the blast expands."""
    import torch
    from paper_2305_13380_amd import sphx
    from paper_2305_13380_amd.sphenix import SphenixRun
    ps = inputs.sedov_box(24, 2, n_hot=16)
    ps.alpha_v[:] = 0.1
    ps.alpha_c[:] = 0.0
    print("gdf sedov run N=%d" % ps.n, flush=True)
    run = SphenixRun(ps, params=sphx.default_params(**FL), c_cfl=0.1)
    m = ps.m.astype(np.float64)
    E0 = float((m * ps.u.astype(np.float64)).sum())
    run.run(40)
    t = run.dp.t
    v = torch.stack([t["vx"], t["vy"], t["vz"]]).cpu().numpy().astype(np.float64)
    u = t["u"].cpu().numpy().astype(np.float64)
    E = 0.5 * (m * (v * v).sum(0)).sum() + (m * u).sum()
    av = t["alpha_v"].cpu().numpy()
    print("gdf sedov: t=%.4g dE/E=%.2e alpha_v in [%.3f, %.3f]" % (
        run.state.t, E / E0 - 1, av.min(), av.max()), flush=True)
    assert abs(E / E0 - 1) < 5e-3
    assert av.min() >= 0.0 and av.max() <= 2.0 and av.max() > 0.5
    assert np.sqrt((v * v).sum(0)).max() > 0.0
    run.close()
