"""The seeded generators: reproducible, the right layout, and the structure
each workload is meant to have."""
import numpy as np

from paper_2305_13380_amd import inputs


def test_generators_are_seeded_and_laid_out():
    a = inputs.lattice_box(8, 3)
    b = inputs.lattice_box(8, 3)
    for k in ("x", "y", "z", "vx", "h", "alpha_v"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert a.x.dtype == np.float64 and a.vx.dtype == np.float32 and a.h.dtype == np.float32
    assert a.x.flags["C_CONTIGUOUS"]
    for k in ("x", "y", "z"):
        v = getattr(a, k)
        assert v.min() >= 0.0 and v.max() < 1.0
    c = inputs.lattice_box(8, 4)
    assert not np.array_equal(a.x, c.x)


def test_sedov_energy_and_hot_spot():
    s = inputs.sedov_box(16, 2, n_hot=32)
    e = (s.m.astype(np.float64) * s.u).sum()
    assert abs(e - 1.0 - (s.n - 32) * 1e-6 / s.n) < 1e-6
    assert np.count_nonzero(s.u > 1.0) == 32
    assert np.all(s.vx == 0)


def test_lognormal_is_clustered_and_active_fraction():
    p = inputs.lognormal_box(32, 32 ** 3, 2.0, 3)
    assert p.n == 32 ** 3
    # density contrast of the mesh-cell counts (mean 1 per cell)
    ijk = np.floor(np.stack([p.x, p.y, p.z], 1) * 32).astype(np.int64)
    counts = np.bincount((ijk[:, 0] * 32 + ijk[:, 1]) * 32 + ijk[:, 2], minlength=32 ** 3)
    assert counts.max() > 100 and np.mean(counts == 0) > 0.3
    assert p.h.max() / p.h.min() > 4.0
    q = inputs.lognormal_box(16, 4096, 2.5, 5, time_bins=(0.1, 0.2, 0.3, 0.4))
    frac = q.active.mean()
    assert 0.07 < frac < 0.13


def test_serving_stream_sizes_and_order():
    sizes, lat = inputs.serving_sizes(512, 4)
    assert sizes.min() >= 1000 and sizes.max() <= 1_000_000
    assert 0.4 < lat.mean() < 0.6
    reqs = list(inputs.serving_stream(100.0, n_req=3))
    assert [r.rid for r in reqs] == [0, 1, 2]
    assert reqs[0].arrival < reqs[1].arrival < reqs[2].arrival
