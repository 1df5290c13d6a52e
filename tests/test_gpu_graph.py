"""Captured steps (graph_passes > 0): the h iteration's passes and the force
pass recorded as one HIP graph and replayed.

The captured step launches the same kernels in the same order as the
pass-by-pass step (passes after convergence find no receiver), so every
output must be bitwise the same, also when the iteration outlives the graph
(it continues pass by pass), when a pass meets a stale task list (rebuild and
continue), at the iteration cap, and on every replay with eager work and
synchronisation in between.
"""
import numpy as np
import pytest

from paper_2305_13380_amd import inputs

from helpers import gpu_step

pytestmark = pytest.mark.gpu

KEYS = ("h", "rho", "rho_dh", "n", "nngb", "f", "P", "A", "balsara", "converged", "ax", "ay",
        "az", "du_dt", "v_sig", "nforce", "sums")

CASES = {
    "lattice16_logu": lambda: inputs.config_small(1, u="logu"),
    "poisson_3001": lambda: inputs.uniform_random_box(3001, 5),
    "lognormal_6000": lambda: inputs.lognormal_box(16, 6000, 2.0, 11),
    "sedov16": lambda: inputs.sedov_box(16, 2, n_hot=8),
}


def same(a, b, where):
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8)), \
            "%s: %s differs" % (where, k)
    for f in ("passes", "unconverged", "clamped", "pairs_cellpair"):
        assert getattr(a["info"], f) == getattr(b["info"], f), "%s: info.%s" % (where, f)


@pytest.mark.parametrize("graph_passes", [8, 2])
@pytest.mark.parametrize("case", sorted(CASES))
def test_graph_step_equals_pass_by_pass(case, graph_passes):
    ps = CASES[case]()
    host = gpu_step(ps)
    reps = gpu_step(ps, params={"graph_passes": graph_passes}, repeat=3)
    for r, g in enumerate(reps):
        same(host, g, "%s graph_passes=%d replay %d" % (case, graph_passes, r))


def test_graph_replays_with_eager_work_between():
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lognormal_box(16, 6000, 2.0, 12)
    host = gpu_step(ps)
    ctx = sphx.Context(sphx.default_params(graph_passes=8))
    dp = sphx.DeviceParticles.from_set(ps)
    out = sphx.Outputs(ps.n)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    h0 = dp.t["h"].clone()
    scratch = torch.zeros(1 << 20, device="cuda")
    for r in range(4):
        dp.t["h"].copy_(h0)
        for k in out.f:
            out.f[k].zero_()  # eager work on the same arrays between replays
        scratch.add_(1.0)
        torch.cuda.synchronize()
        st, info = sphx.step(ctx, grid, tasks, dp, out)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for grp in (out.d, out.g, out.f) for k, v in grp.items()}
        g["h"] = dp.t["h"].cpu().numpy()
        g["sums"] = out.sums.cpu().numpy()
        g["info"] = info
        same(host, g, "replay %d" % r)


def test_graph_step_with_task_rebuild():
    ps = inputs.lattice_box(14, 3, u="logu")
    ps.h *= np.float32(0.45)  # h must more than double: the tasks go stale
    host = gpu_step(ps)
    g = gpu_step(ps, params={"graph_passes": 8})
    assert host["info"].task_rebuilds >= 1 and g["info"].task_rebuilds >= 1
    same(host, g, "rebuild")


def test_graph_step_at_the_iteration_cap():
    ps = inputs.lattice_box(12, 5)
    ps.h *= np.float32(1.3)
    host = gpu_step(ps, params={"max_iter": 2})
    g = gpu_step(ps, params={"max_iter": 2, "graph_passes": 8})
    assert host["info"].unconverged > 0
    same(host, g, "cap")


def test_graph_step_active_subset():
    ps = inputs.lognormal_box(16, 5000, 2.0, 21, time_bins=(0.1, 0.2, 0.3, 0.4))
    host = gpu_step(ps)
    g = gpu_step(ps, params={"graph_passes": 8})
    same(host, g, "active")


def test_graph_rebuilds_inside():
    """A clustered set iterated from its generator's h rebuilds its task list
    during the step. With enough slots every pass runs inside the graph (the
    rebuilds are walked in place, decided on the device), on every replay,
    bitwise as pass by pass."""
    ps = inputs.lognormal_box(16, 6000, 2.0, 11)
    host = gpu_step(ps)
    assert host["info"].task_rebuilds >= 1
    reps = gpu_step(ps, params={"graph_passes": host["info"].passes + 1}, repeat=3)
    for r, g in enumerate(reps):
        same(host, g, "replay %d" % r)
        assert g["info"].captured_passes == g["info"].passes, "replay %d" % r
        assert g["info"].task_rebuilds >= 1


def test_graph_step_outgrowing_the_layout():
    """h five times too small with leaves of 8: the first rebuild inside the
    graph outgrows the slots sized at the first build; the graph stops there,
    the list is laid out anew and the step goes on pass by pass, bitwise as
    without a graph."""
    ps = inputs.lattice_box(14, 3, u="logu")
    ps.h *= np.float32(0.2)
    kw = {"leaf_max": 8}
    host = gpu_step(ps, params=kw)
    g = gpu_step(ps, params=dict(kw, graph_passes=12))
    same(host, g, "outgrown")
    assert 0 < g["info"].passes and g["info"].captured_passes < g["info"].passes
