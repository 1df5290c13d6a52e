"""Continuous-batching serving: requests of different sizes and geometries
overlap on the device, each on its own stream and grid.

* every result of a request is bitwise the same alone, in the mix, and in a
  batch of requests run as one step over a grid of independent sets;
* a tiny HBM budget makes requests wait (never an out-of-memory failure), and
  a request larger than the budget is rejected with a message;
* latencies are completion minus arrival, and the percentiles are ordered;
* the two smallest lattice and lognormal requests agree with the oracle's
  own smoothing-length solve, and every output and the FP64 sums with the
  oracle at the request's own final h.
"""
import numpy as np
import pytest

import oracle
from paper_2305_13380_amd import inputs

pytestmark = pytest.mark.gpu
P = oracle.Params()


def log(*a):
    print(*a, flush=True)


def mix_requests(n_req=14, seed=21):
    """A seeded mix with the serving stream's recipe, sizes 10^3 .. 10^5.3."""
    sizes, lattice = inputs.serving_sizes(n_req, seed, 3.0, 5.3)
    return [inputs.serving_request(k, int(sizes[k]), bool(lattice[k]), seed)
            for k in range(n_req)]


@pytest.fixture(scope="module")
def served():
    from paper_2305_13380_amd import serve, sphx
    reqs = mix_requests()
    log("serving: %d requests, sizes %s" % (len(reqs), [r.n for r in reqs]))
    dev = [sphx.DeviceParticles.from_set(r, "cuda:0") for r in reqs]
    spec = [(k, 0.0, r.n) for k, r in enumerate(reqs)]
    alone = serve.Server(n_slots=1, keep_outputs=True)
    res_alone = alone.run(spec, lambda k: dev[k])
    log("serving: alone run done, peak running %d" % alone.peak_running)
    mix = serve.Server(n_slots=6, keep_outputs=True)
    res_mix = mix.run(spec, lambda k: dev[k])
    log("serving: mix run done, peak running %d" % mix.peak_running)
    # batches of at most 150,000 particles on 2 slots: several batches, some
    # of several requests, overlapping
    batched = serve.Server(n_slots=2, keep_outputs=True, batch_particles=150000)
    res_batch = batched.run(spec, lambda k: dev[k])
    log("serving: batched run done, peak running %d" % batched.peak_running)
    out = dict(reqs=reqs, alone=res_alone, mix=res_mix, mix_server=mix, dev=dev,
               batch=res_batch, batch_server=batched)
    yield out
    alone.close()
    mix.close()
    batched.close()


def test_alone_equals_batch_bitwise(served):
    """Requests run as batches (one grid of independent sets per batch) give
    bitwise the results of each request alone, its FP64 sums included."""
    assert served["batch_server"].peak_running > 2  # batches of several requests
    starts = {}
    for a, b in zip(served["alone"], served["batch"]):
        assert a.error is None and b.error is None, (a.error, b.error)
        assert b.status >= 0 and a.interactions == b.interactions
        starts.setdefault(b.start, []).append(b.rid)
        for key, va in a.outputs.items():
            vb = b.outputs[key]
            assert va.dtype == vb.dtype and va.shape == vb.shape
            assert np.array_equal(va.view(np.uint8), vb.view(np.uint8)), (a.rid, key)
    assert 1 < len(starts) < len(served["reqs"])  # several batches, not one per request


def test_alone_equals_mix_bitwise(served):
    assert served["mix_server"].peak_running > 1  # the requests really overlapped
    for a, b in zip(served["alone"], served["mix"]):
        assert a.error is None and b.error is None, (a.error, b.error)
        assert a.status >= 0 and a.passes == b.passes and a.interactions == b.interactions
        for key, va in a.outputs.items():
            vb = b.outputs[key]
            assert va.dtype == vb.dtype and va.shape == vb.shape
            assert np.array_equal(va.view(np.uint8), vb.view(np.uint8)), (a.rid, key)


def test_served_inputs_unchanged(served):
    """A request given as device arrays is not modified by serving it."""
    for r, d in zip(served["reqs"], served["dev"]):
        assert np.array_equal(d.t["h"].cpu().numpy(), r.h)


def test_results_finite_and_converged(served):
    for r in served["mix"]:
        o = r.outputs
        for key in ("rho", "ax", "ay", "az", "du_dt", "v_sig", "h"):
            assert np.all(np.isfinite(o[key])), (r.rid, key)
        assert np.all(o["converged"] == 1), r.rid
        s = o["sums"]
        assert np.abs(s[:3]).max() < 1e-5 * s[4]


def test_latency_accounting(served):
    from paper_2305_13380_amd import serve
    for r in served["mix"]:
        assert r.arrival <= r.start <= r.done
    q = serve.percentiles(served["mix"])
    assert 0 < q["p50_s"] <= q["p99_s"] <= q["max_s"]


@pytest.mark.parametrize("rank", [0, 1])
@pytest.mark.parametrize("geometry", ["lattice", "lognormal"])
def test_small_requests_match_oracle(served, geometry, rank):
    """The smallest and second-smallest request of each geometry: h against
    the oracle's own solve, then every density, ghost and force output of
    the served step against the oracle evaluated at the step's own h."""
    from helpers import RHO_TOL, check_density, check_force, check_ghost
    reqs = served["reqs"]
    ks = sorted((k for k, r in enumerate(reqs) if r.name.endswith(geometry)),
                key=lambda k: reqs[k].n)
    k = ks[rank]
    ps, g = reqs[k], served["mix"][k].outputs
    log("serving: oracle check of request %d (%s, N=%d)" % (k, geometry, ps.n))
    hr, dens, conv, _, _ = oracle.solve_h(ps, P)
    assert conv.all()
    hg = g["h"].astype(np.float64)
    dh = np.abs(hg - hr) / hr
    assert np.all(dh <= 2 * P.h_tol), dh.max()
    sens = np.abs(hr * dens["rho_dh"] / dens["rho"])
    rho = g["rho"].astype(np.float64)
    assert np.all(np.abs(rho - dens["rho"]) <= (RHO_TOL + 1.5 * sens * dh) * dens["rho"])
    ref = oracle.fixed_h_step(ps, P, h=hg)
    recv = np.arange(ps.n)
    where = "served request %d at its h" % k
    check_density(g, ref, ps, hg, recv, P, where)
    check_ghost(g, ref, recv, where)
    check_force(g, ref, ps, hg, recv, P, where)
    s_ref = oracle.sums(ps.m, ps.vx, ps.vy, ps.vz, g["ax"], g["ay"], g["az"], g["du_dt"])
    np.testing.assert_allclose(g["sums"], s_ref, rtol=1e-12, atol=1e-12 * (s_ref[4] + s_ref[5]))


def test_tiny_budget_queues_and_rejects():
    """With room for about one large request at a time, requests wait for
    memory instead of failing; one larger than the whole budget is refused."""
    from paper_2305_13380_amd import serve, sphx
    reqs = [inputs.serving_request(k, n, k % 2 == 0, 33)
            for k, n in enumerate([20000, 30000, 25000, 1000, 28000, 200000])]
    srv = serve.Server(n_slots=4, budget_bytes=1, keep_outputs=False)
    need = [serve.request_bytes(srv.ctxs[0], r.n) for r in reqs]
    srv.budget = int(1.2 * max(need[:5]))  # the 200k request does not fit
    spec = [(k, 0.0, r.n) for k, r in enumerate(reqs)]
    res = srv.run(spec, lambda k: reqs[k])  # host sets: each request uploads its own
    srv.close()
    for r in res[:5]:
        assert r.error is None and r.status >= 0 and r.interactions > 0, r.error
    assert res[5].error is not None and "budget" in res[5].error
    assert srv.peak_bytes <= srv.budget
    # only the 1000-particle request can share the budget with a large one
    assert srv.peak_running <= 2
