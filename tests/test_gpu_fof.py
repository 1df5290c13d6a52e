"""GPU friends-of-friends groups (sphx_fof) against the oracle, bit for bit:
the group of every particle (its smallest member index), the group sizes, the
number of groups and the number of linked pairs. Both sides decide every link
in FP64 with the same operations, so the partition is unique and identical."""
import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

pytestmark = pytest.mark.gpu


def gpu_fof(ps, b, params=None, device="cuda:0"):
    import torch
    from paper_2305_13380_amd import sphx
    kw = {} if params is None else dict(params)
    ctx = sphx.Context(sphx.default_params(**kw), 0)
    dp = sphx.DeviceParticles.from_set(ps, device)
    group, gsize, counts = sphx.fof(ctx, dp, b)
    torch.cuda.synchronize()
    return group.cpu().numpy(), gsize.cpu().numpy(), counts.cpu().numpy()


def compare(ps, b, where, params=None, periodic=True):
    print("fof case:", where, "N=%d b=%.6g" % (ps.n, b), flush=True)
    g, gs, cnt = gpu_fof(ps, b, params)
    ref, links = oracle.fof(ps, b, periodic=periodic, mode="auto")
    bad = np.nonzero(g != ref)[0]
    assert bad.size == 0, "%s: %d particles in another group (first %s)" % (
        where, bad.size, bad[:5])
    sizes = np.bincount(ref, minlength=ps.n)[ref]
    np.testing.assert_array_equal(gs, sizes)
    assert cnt[0] == len(np.unique(ref)), where + " group count"
    assert cnt[1] == links, "%s links %d, oracle %d" % (where, cnt[1], links)
    return ref, links


def sep(ps):
    return (float(np.prod(ps.box)) / ps.n) ** (1.0 / 3.0)


CASES = {
    "lognormal_6000": lambda: inputs.lognormal_box(16, 6000, 2.0, 11),
    "poisson_3001": lambda: inputs.uniform_random_box(3001, 5),
    "sedov16": lambda: inputs.sedov_box(16, 2, n_hot=8),
    "lognormal_20000": lambda: inputs.lognormal_box(24, 20000, 2.0, 4),
}


@pytest.mark.parametrize("frac", [0.2, 0.5, 0.9])
@pytest.mark.parametrize("case", sorted(CASES))
def test_fof_matches_oracle(case, frac):
    ps = CASES[case]()
    ref, links = compare(ps, frac * sep(ps), "%s b=%.1f sep" % (case, frac))
    if frac == 0.9 and case.startswith("lognormal"):
        # past percolation: one group holds much of the box
        assert np.bincount(ref).max() > ps.n // 4


def test_fof_lattice_is_strict_at_the_spacing():
    ps = inputs.lattice_box(8, 0, jitter=0.0, sigma_v=0.0)  # spacing 1/8, exact
    ref, links = compare(ps, 0.125, "lattice b = spacing")
    assert links == 0
    ref, links = compare(ps, 0.125 * (1 + 1e-9), "lattice b > spacing")
    assert links == 3 * ps.n and np.all(ref == 0)


def test_fof_chain_across_the_boundary_and_open_box():
    ps = inputs.uniform_random_box(10, 1)
    b = 0.05
    ps.x[:] = (0.97 + 0.9 * b * np.arange(10)) % 1.0
    ps.y[:] = 0.5
    ps.z[:] = 0.5
    ref, links = compare(ps, b, "periodic chain")
    assert links == 9 and np.all(ref == ref[0])
    ref, links = compare(ps, b, "open chain", params={"periodic": 0}, periodic=False)
    assert len(np.unique(ref)) == 2


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 200])
def test_fof_tiny_inputs(n):
    ps = inputs.uniform_random_box(n, 9)
    compare(ps, 0.3, "tiny n=%d" % n)


def test_fof_empty_and_invalid():
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.uniform_random_box(1, 1).subset(np.zeros(0, np.int64))
    g, gs, cnt = gpu_fof(ps, 0.1)
    assert g.size == 0 and list(cnt) == [0, 0]
    ps = inputs.uniform_random_box(100, 1)
    ctx = sphx.Context(sphx.default_params(), 0)
    dp = sphx.DeviceParticles.from_set(ps, "cuda:0")
    for b in (0.0, -1.0, 0.34, float("nan")):
        with pytest.raises(sphx.SphxError):
            sphx.fof(ctx, dp, b)
    torch.cuda.synchronize()


def test_fof_small_leaves_and_repeat():
    ps = inputs.lognormal_box(16, 8000, 2.0, 12)
    b = 0.5 * sep(ps)
    ref, _ = compare(ps, b, "leaf_max=8", params={"leaf_max": 8})
    g1 = gpu_fof(ps, b)
    g2 = gpu_fof(ps, b)
    for a, c in zip(g1, g2):
        np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(g1[0], ref)


def test_fof_without_sizes_or_counts():
    # group_size and d_counts may be NULL: the library counts into its own
    # workspace and writes the groups alone
    import ctypes as C
    import torch
    from paper_2305_13380_amd import sphx
    ps = inputs.lognormal_box(16, 6000, 2.0, 11)
    b = 0.5 * sep(ps)
    ctx = sphx.Context(sphx.default_params(), 0)
    dp = sphx.DeviceParticles.from_set(ps, "cuda:0")
    group = torch.full((ps.n,), -1, dtype=torch.int32, device="cuda:0")
    pv = dp.view()
    st = sphx.lib.sphx_fof(ctx.handle, C.byref(pv), b, C.c_void_p(group.data_ptr()), None, None,
                           C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == 0
    ref, _ = oracle.fof(ps, b, mode="auto")
    np.testing.assert_array_equal(group.cpu().numpy(), ref)
