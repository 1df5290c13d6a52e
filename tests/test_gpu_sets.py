"""Several independent particle sets in one grid (sphx_grid_build_sets, the
serving loop's batches): every set's outputs and conservation sums must be
bitwise those of the set alone, since no leaf or task joins two sets and
each set's sums are reduced on their own."""
import numpy as np
import pytest

from paper_2305_13380_amd import inputs

from helpers import gpu_step

pytestmark = pytest.mark.gpu

KEYS = ("rho", "rho_dh", "n", "n_dh", "nngb", "f", "P", "c", "balsara", "A", "div_v", "curl_v",
        "converged", "ax", "ay", "az", "du_dt", "v_sig", "nforce")


def sets_step(sets, params=None, repeat=1):
    """One step of the sets concatenated in one grid; results per set."""
    import torch
    from paper_2305_13380_amd import sphx
    kw = {} if params is None else dict(params)
    ctx = sphx.Context(sphx.default_params(**kw), 0)
    dps = [sphx.DeviceParticles.from_set(ps, "cuda:0") for ps in sets]
    dp, off = sphx.DeviceParticles.concat(dps)
    out = sphx.Outputs(dp.n, "cuda:0", n_sets=len(sets))
    grid = sphx.Grid(ctx, dp, sets=off)
    tasks = sphx.Tasks(ctx, grid, dp)
    h0 = dp.t["h"].clone()
    runs = []
    for _ in range(repeat):
        dp.t["h"].copy_(h0)
        st, info = sphx.step(ctx, grid, tasks, dp, out)
        torch.cuda.synchronize()
        res = []
        for b in range(len(sets)):
            a, e = off[b], off[b + 1]
            r = {k: v[a:e].cpu().numpy() for grp in (out.d, out.g, out.f) for k, v in grp.items()}
            r["h"] = dp.t["h"][a:e].cpu().numpy()
            r["sums"] = out.sums[6 * b:6 * b + 6].cpu().numpy()
            res.append(r)
        runs.append((res, info))
    tasks.close()
    grid.close()
    ctx.close()
    return runs if repeat > 1 else runs[0]


def same_as_alone(batch, sets, params=None, where=""):
    for b, ps in enumerate(sets):
        alone = gpu_step(ps, params=params)
        got = batch[b]
        for k in KEYS + ("h", "sums"):
            assert np.array_equal(np.asarray(alone[k]).view(np.uint8),
                                  np.asarray(got[k]).view(np.uint8)), \
                "%s set %d: %s differs" % (where, b, k)


def mixed_sets():
    return [inputs.lattice_box(8, 3, u="logu"),
            inputs.lognormal_box(16, 3000, 2.0, 7),
            inputs.sedov_box(12, 2, n_hot=8),
            inputs.uniform_random_box(700, 9),
            inputs.lognormal_box(8, 300, 2.5, 4)]


def test_sets_step_equals_each_set_alone():
    sets = mixed_sets()
    res, info = sets_step(sets)
    assert info.passes >= 2 and info.n_leaves > len(sets)
    same_as_alone(res, sets)


def test_sets_with_empty_and_single_particle_sets():
    """Empty sets and a set of one particle among the others; an empty set's
    sums are zero."""
    one = inputs.uniform_random_box(1, 3)
    one.h[:] = np.float32(0.1)  # (the generator's h for one particle is beyond h_max)
    empty = one.subset(np.zeros(0, np.int64))
    sets = [inputs.lattice_box(8, 2), empty, one, inputs.lognormal_box(8, 400, 2.0, 5), empty]
    res, _ = sets_step(sets)
    for b in (1, 4):
        assert res[b]["n"].size == 0 and np.all(res[b]["sums"] == 0.0)
    for b in (0, 2, 3):
        same_as_alone([res[b]], [sets[b]], where="set %d" % b)


def test_sets_captured_step_replays():
    """The captured step (task rebuilds inside the graph) over a grid of sets,
    replayed: bitwise the sets alone on every replay."""
    sets = mixed_sets()[:3]
    runs = sets_step(sets, params={"graph_passes": 10}, repeat=3)
    for r, (res, info) in enumerate(runs):
        assert info.captured_passes > 0
        same_as_alone(res, sets, where="replay %d" % r)


def test_sets_active_subsets():
    """Sets with active subsets (time bins) next to fully active ones."""
    sets = [inputs.lognormal_box(16, 4000, 2.0, 21, time_bins=(0.3, 0.7)),
            inputs.lattice_box(9, 4)]
    res, _ = sets_step(sets)
    same_as_alone(res, sets)


def test_noalloc_force_refuses_a_grid_of_sets():
    """The no-allocation force pass holds the sums' reduction of one set only:
    a grid of several sets is refused before anything is enqueued."""
    import ctypes as C
    from paper_2305_13380_amd import sphx
    sets = [inputs.lattice_box(8, 1), inputs.lattice_box(8, 2)]
    ctx = sphx.Context()
    dps = [sphx.DeviceParticles.from_set(ps, "cuda:0") for ps in sets]
    dp, off = sphx.DeviceParticles.concat(dps)
    out = sphx.Outputs(dp.n, "cuda:0", n_sets=2)
    grid = sphx.Grid(ctx, dp, sets=off)
    tasks = sphx.Tasks(ctx, grid, dp)
    pv, dv, gv, fv = dp.view(), out.dens_view(), out.ghost_view(), out.force_view()
    st = sphx.lib.sphx_force_noalloc(ctx.handle, grid.handle, tasks.handle, C.byref(pv),
                                     C.byref(dv), C.byref(gv), C.byref(fv),
                                     C.c_void_p(out.sums.data_ptr()), None)
    assert st == sphx.E_INVALID and "several particle sets" in sphx.last_error()
    tasks.close()
    grid.close()
    ctx.close()


def test_sets_gdf_step_equals_each_set_alone():
    """The GDF flavour on a grid of sets: its loop and force law per set are
    bitwise the ones each set gets alone (f and alpha_c included)."""
    sets = mixed_sets()
    for ps in sets:
        ps.vx[:] = np.random.default_rng(ps.n).normal(0, 0.3, ps.n).astype(np.float32)
    res, info = sets_step(sets, params={"flavour": "gdf"})
    assert info.passes >= 2
    same_as_alone(res, sets, params={"flavour": "gdf"}, where="gdf")
