"""GPU parity for every smoothing kernel of Section 3.1 (Wendland C2, C4,
C6; cubic, quartic, quintic splines): density, ghost and force at a fixed h
element by element against the oracle, and a whole step (the h iteration
from the input h, then the force pass) at the step's own final h, at the
tolerances of the Wendland C2 cases."""
import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

from helpers import check_density, check_force, check_ghost, gpu_fixed_h, gpu_step

pytestmark = pytest.mark.gpu
NAMES = sorted(oracle.KERNELS)

CASES = {
    "lattice16_logu": lambda: inputs.config_small(1, u="logu"),
    "lognormal_6000": lambda: inputs.lognormal_box(16, 6000, 2.0, 11),
    "sedov16": lambda: inputs.sedov_box(16, 2, n_hot=8),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("name", NAMES)
def test_fixed_h_parity_every_kernel(name, case):
    ps = CASES[case]()
    P = oracle.Params.with_kernel(name)
    where = "%s/%s" % (name, case)
    print("kernel parity case:", where, "N=%d" % ps.n, flush=True)
    g = gpu_fixed_h(ps, params={"kernel": name})
    assert g["counters"][3] == 0, "density pass ran on a stale task list"
    ref = oracle.fixed_h_step(ps, P, mode="auto")
    recv = np.arange(ps.n)
    h = ps.h.astype(np.float64)
    check_density(g, ref, ps, h, recv, P, where)
    check_ghost(g, ref, recv, where)
    check_force(g, ref, ps, h, recv, P, where)


@pytest.mark.parametrize("name", NAMES)
def test_step_parity_every_kernel(name):
    ps = inputs.lognormal_box(16, 6000, 2.0, 11)
    P = oracle.Params.with_kernel(name)
    print("kernel step case:", name, "N=%d" % ps.n, flush=True)
    g = gpu_step(ps, params={"kernel": name})
    info = g["info"]
    assert g["status"] >= 0 and info.unconverged == 0
    # the h iteration against the oracle's own solve
    ref = oracle.nr_step(ps, P, mode="auto")
    h, hr = g["h"].astype(np.float64), ref["h"]
    dh = np.abs(h - hr) / hr
    assert np.all(dh <= 2 * P.h_tol), "%s h: worst %.3g" % (name, dh.max())
    assert np.all(g["converged"] == 1)
    # every output at the step's own h, at the fixed-h tolerances
    at = oracle.fixed_h_step(ps, P, mode="auto", h=h)
    recv = np.arange(ps.n)
    where = name + " step at its h"
    check_density(g, at, ps, h, recv, P, where)
    check_ghost(g, at, recv, where)
    check_force(g, at, ps, h, recv, P, where)
    s = g["sums"]
    assert np.abs(s[:3]).max() < 2e-5 * s[4]


def test_kernels_give_different_densities():
    # the kernel choice reaches the loops: same particles and h, six kernels,
    # six different densities (each matching its own oracle above)
    ps = inputs.lognormal_box(16, 3000, 2.0, 5)
    rho = [gpu_fixed_h(ps, params={"kernel": k})["rho"] for k in NAMES]
    for a in range(len(NAMES)):
        for b in range(a):
            assert np.abs(rho[a] - rho[b]).max() > 1e-3 * np.abs(rho[b]).max()


@pytest.mark.parametrize("variant", ["lists", "graph"])
@pytest.mark.parametrize("name", ["quartic_spline", "wendland_c6"])
def test_step_paths_with_other_kernels(name, variant):
    # the neighbour-list density loop and the captured step run the same
    # kernel templates: a whole step through each, at the step's own h
    ps = inputs.lognormal_box(16, 6000, 2.0, 11)
    P = oracle.Params.with_kernel(name)
    kw = {"kernel": name}
    kw.update({"neighbour_lists": 1} if variant == "lists" else {"graph_passes": 4})
    print("kernel step path:", name, variant, flush=True)
    g = gpu_step(ps, params=kw)
    assert g["status"] >= 0 and g["info"].unconverged == 0
    h = g["h"].astype(np.float64)
    ref = oracle.nr_step(ps, P, mode="auto")
    assert np.all(np.abs(h - ref["h"]) <= 2 * P.h_tol * ref["h"])
    at = oracle.fixed_h_step(ps, P, mode="auto", h=h)
    recv = np.arange(ps.n)
    where = "%s %s step at its h" % (name, variant)
    check_density(g, at, ps, h, recv, P, where)
    check_ghost(g, at, recv, where)
    check_force(g, at, ps, h, recv, P, where)
