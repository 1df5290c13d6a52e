"""Pins of the oracle's friends-of-friends groups (Section 9.1: particles
closer than the linking length are linked, chains of links form groups).

Fixed by: connected components from an independent routine (scipy's graph
components over a brute-force distance matrix), exact lattice geometry
(six links per particle just above the spacing, none just below, none at
exactly the spacing: the link test is strict), transitivity along a chain,
the periodic wrap, permutation invariance, and tree candidates = brute force.
"""
import types

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from paper_2305_13380_amd import inputs


def pset(pos, box=1.0):
    pos = np.asarray(pos, np.float64)
    n = len(pos)
    return types.SimpleNamespace(n=n, x=np.ascontiguousarray(pos[:, 0]),
                                 y=np.ascontiguousarray(pos[:, 1]),
                                 z=np.ascontiguousarray(pos[:, 2]), box=(box, box, box))


def canonical(labels):
    """Relabel a partition by the smallest index of each part."""
    labels = np.asarray(labels)
    first = {}
    for i, l in enumerate(labels):
        first.setdefault(l, i)
    return np.array([first[l] for l in labels])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_groups_are_the_connected_components(seed):
    rng = np.random.default_rng(seed)
    n = 400
    # clumps of points, so that groups of many sizes appear
    centres = rng.random((12, 3))
    pos = (centres[rng.integers(0, 12, n)] + 0.03 * rng.standard_normal((n, 3))) % 1.0
    ps = pset(pos)
    b = 0.02
    group, links = oracle.fof(ps, b, mode="brute")
    d = pos[:, None, :] - pos[None, :, :]
    d -= np.round(d)
    r2 = (d * d).sum(2)
    i, j = np.nonzero(np.triu(r2 < b * b, 1))
    assert links == len(i)
    A = coo_matrix((np.ones(len(i)), (i, j)), shape=(n, n))
    ncomp, lab = connected_components(A, directed=False)
    np.testing.assert_array_equal(group, canonical(lab))
    assert len(np.unique(group)) == ncomp and 1 < ncomp < n
    # the group id is the smallest member's index
    for g in np.unique(group):
        assert np.nonzero(group == g)[0].min() == g


def test_lattice_links_strict_at_the_spacing():
    # spacing 1/8 is exact in binary, so pairs sit at exactly b = 1/8
    k = 8
    g = (np.arange(k) + 0.5) / k
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    ps = pset(pos)
    group, links = oracle.fof(ps, 1.0 / k * (1 + 1e-9), mode="brute")
    assert links == 3 * ps.n and np.all(group == 0)
    group, links = oracle.fof(ps, 1.0 / k, mode="brute")  # r = b exactly: no link
    assert links == 0 and np.array_equal(group, np.arange(ps.n))
    group, links = oracle.fof(ps, 1.0 / k * (1 - 1e-9), mode="brute")
    assert links == 0
    # just above sqrt(2) spacing: 6 + 12 neighbours each
    group, links = oracle.fof(ps, np.sqrt(2.0) / k * (1 + 1e-9), mode="brute")
    assert links == 9 * ps.n


def test_chain_is_transitive_and_wraps_periodically():
    b = 0.05
    xs = (0.97 + 0.9 * b * np.arange(10)) % 1.0  # crosses x = 1 -> 0
    pos = np.stack([xs, np.full(10, 0.5), np.full(10, 0.5)], 1)
    group, links = oracle.fof(pset(pos), b, mode="brute")
    assert links == 9 and np.all(group == group[0])
    group, _ = oracle.fof(pset(pos), b, periodic=False, mode="brute")
    assert len(np.unique(group)) == 2  # the wrap link is gone
    # a gap of 1.1 b splits the chain
    xs2 = 0.1 + 0.9 * b * np.arange(10)
    xs2[5:] += 0.2 * b
    pos2 = np.stack([xs2, np.full(10, 0.5), np.full(10, 0.5)], 1)
    group, links = oracle.fof(pset(pos2), b, mode="brute")
    assert links == 8 and list(np.unique(group)) == [0, 5]


def test_permutation_and_tree_mode():
    ps = inputs.lognormal_box(16, 5000, 2.0, 7)
    b = oracle.fof_link_length(ps)
    assert abs(b - 0.2 * 5000 ** (-1.0 / 3.0)) < 1e-15
    g1, l1 = oracle.fof(ps, b, mode="brute")
    g2, l2 = oracle.fof(ps, b, mode="tree")
    assert l1 == l2 > 0 and np.array_equal(g1, g2)
    perm = np.random.default_rng(3).permutation(ps.n)
    q = pset(np.stack([ps.x, ps.y, ps.z], 1)[perm])
    g3, l3 = oracle.fof(q, b, mode="brute")
    assert l3 == l1
    np.testing.assert_array_equal(canonical(g3), canonical(g1[perm]))
