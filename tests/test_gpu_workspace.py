"""The device memory a grid, its task lists and a step take, against
sphx_workspace_bytes (the figure the serving admission reserves per
request). The library allocates its workspace from the device's default
stream-ordered memory pool, whose used-bytes counter is read through the
HIP runtime the library is bound to (the one torch loaded)."""
import ctypes as C

import numpy as np
import pytest

from paper_2305_13380_amd import inputs

pytestmark = pytest.mark.gpu


def _runtime():
    """The HIP runtime mapped in the process (one: the library binds to the
    runtime torch loaded)."""
    from paper_2305_13380_amd import sphx  # noqa: F401
    maps = open("/proc/self/maps").read().splitlines()
    paths = sorted(set(l.split()[-1] for l in maps if "libamdhip64" in l))
    assert len(paths) == 1, paths
    return C.CDLL(paths[0])  # already mapped: the same handle


def _pool_used():
    hip = _runtime()
    pool = C.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(C.byref(pool), 0) == 0
    used = C.c_uint64()
    attr_used_current = 7  # hipMemPoolAttrUsedMemCurrent
    assert hip.hipMemPoolGetAttribute(pool, attr_used_current, C.byref(used)) == 0
    return int(used.value)


@pytest.mark.parametrize("case", ["lognormal_s2", "lognormal_s3", "lognormal_s3_small_leaves",
                                  "sedov"])
def test_step_workspace_within_the_estimate(case):
    import torch
    from paper_2305_13380_amd import sphx
    kw = {}
    if case == "lognormal_s2":
        ps = inputs.lognormal_box(32, 60000, 2.0, 41)
    elif case == "lognormal_s3":
        ps = inputs.lognormal_box(32, 60000, 3.0, 43)
    elif case == "lognormal_s3_small_leaves":
        ps = inputs.lognormal_box(32, 60000, 3.0, 42)
        kw["leaf_max"] = 16
    else:
        ps = inputs.sedov_box(24, 2, n_hot=16)
    params = sphx.default_params(**kw)
    torch.cuda.synchronize()
    before = _pool_used()
    ctx = sphx.Context(params, 0)
    dp = sphx.DeviceParticles.from_set(ps)
    out = sphx.Outputs(ps.n)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    st, info = sphx.step(ctx, grid, tasks, dp, out)
    torch.cuda.synchronize()
    used = _pool_used() - before
    est = ctx.workspace_bytes(ps.n)
    print("%s: N=%d leaves=%d tasks=%d rebuilds=%d pool %.1f MB, estimate %.1f MB" % (
        case, ps.n, grid.n_leaves, tasks.count, info.task_rebuilds, used / 2**20, est / 2**20),
          flush=True)
    assert st >= 0
    assert used <= est, "the workspace took %d bytes, the estimate is %d" % (used, est)
    tasks.close()
    grid.close()
    ctx.close()
