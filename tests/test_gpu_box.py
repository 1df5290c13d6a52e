"""A periodic box of unequal sides (1.0 x 0.6 x 0.8): the grid keys, the cell
offsets and the minimum image take each axis's own length. Density, ghost
and force at a fixed h and over a whole step, friends-of-friends groups and
short-range gravity, each against the oracle with the same box."""
import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

from helpers import check_density, check_force, check_ghost, gpu_fixed_h, gpu_step

pytestmark = pytest.mark.gpu
BOX = (1.0, 0.6, 0.8)


def box_set(n, seed):
    ps = inputs.uniform_random_box(n, seed, sigma_v=0.1)
    ps.x = np.ascontiguousarray(ps.x * BOX[0])
    ps.y = np.ascontiguousarray(ps.y * BOX[1])
    ps.z = np.ascontiguousarray(ps.z * BOX[2])
    ps.box = BOX
    ps.h = (ps.h * np.float32(np.prod(BOX) ** (1.0 / 3.0))).astype(np.float32)
    return ps


def test_box_fixed_h_and_step():
    ps = box_set(5000, 21)
    P = oracle.Params(box=BOX)
    g = gpu_fixed_h(ps, params={"box": BOX})
    ref = oracle.fixed_h_step(ps, P, mode="auto")
    recv = np.arange(ps.n)
    h = ps.h.astype(np.float64)
    check_density(g, ref, ps, h, recv, P, "box fixed h")
    check_ghost(g, ref, recv, "box fixed h")
    check_force(g, ref, ps, h, recv, P, "box fixed h")
    s = gpu_step(ps, params={"box": BOX})
    assert s["status"] >= 0 and s["info"].unconverged == 0
    hs = s["h"].astype(np.float64)
    hr = oracle.nr_step(ps, P, mode="auto")["h"]
    assert np.all(np.abs(hs - hr) <= 2 * P.h_tol * hr)
    at = oracle.fixed_h_step(ps, P, mode="auto", h=hs)
    check_density(s, at, ps, hs, recv, P, "box step at its h")
    check_force(s, at, ps, hs, recv, P, "box step at its h")


def test_box_fof_and_gravity():
    import torch
    from paper_2305_13380_amd import sphx
    from test_gpu_gravity import check
    ps = box_set(6000, 22)
    sep = (np.prod(BOX) / ps.n) ** (1.0 / 3.0)
    ctx = sphx.Context(sphx.default_params(box=BOX), 0)
    dp = sphx.DeviceParticles.from_set(ps, "cuda:0")
    b = 0.6 * sep
    group, gsize, counts = sphx.fof(ctx, dp, b)
    torch.cuda.synchronize()
    ref, links = oracle.fof(ps, b, mode="auto")
    assert np.array_equal(group.cpu().numpy(), ref)
    assert int(counts[1].item()) == links and links > 0
    ax, ay, az, pot = sphx.gravity(ctx, dp, 1.0, 0.5 * sep, 1.25 * sep, 1.5 * sep)
    torch.cuda.synchronize()
    a = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], 1)
    check(ps, a, pot.cpu().numpy(), 1.0, 0.5 * sep, 1.25 * sep, 1.5 * sep, "box gravity")


def test_fof_and_gravity_ignore_h_and_active():
    # h may be NULL and the active mask does not matter: every particle links
    # and receives
    import ctypes as C
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lognormal_box(16, 5000, 2.0, 8)
    sep = (1.0 / ps.n) ** (1.0 / 3.0)
    ctx = sphx.Context(sphx.default_params(), 0)
    dp = sphx.DeviceParticles.from_set(ps, "cuda:0")
    g0, _, c0 = sphx.fof(ctx, dp, 0.5 * sep)
    a0 = sphx.gravity(ctx, dp, 1.0, 0.5 * sep, 1.25 * sep, 1.5 * sep)
    dp.t["active"] = torch.from_numpy((np.arange(ps.n) % 7 == 0).astype(np.uint8)).cuda()
    pv = dp.view()
    pv.h = None
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    g1 = torch.empty(ps.n, dtype=torch.int32, device="cuda:0")
    c1 = torch.empty(2, dtype=torch.int64, device="cuda:0")
    assert sphx.lib.sphx_fof(ctx.handle, C.byref(pv), 0.5 * sep, C.c_void_p(g1.data_ptr()), None,
                             C.c_void_p(c1.data_ptr()), stream) == 0
    a1 = [torch.empty(ps.n, dtype=torch.float32, device="cuda:0") for _ in range(4)]
    assert sphx.lib.sphx_gravity(ctx.handle, C.byref(pv), 1.0, 0.5 * sep, 1.25 * sep, 1.5 * sep,
                                 *[C.c_void_p(t.data_ptr()) for t in a1], None, stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(g0, g1) and torch.equal(c0, c1)
    for x, y in zip(a0, a1):
        assert torch.equal(x, y)
