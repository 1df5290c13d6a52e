#!/usr/bin/env python3
"""Benchmark: SPH pair interactions per second (density + force) on one GPU.

One step = the whole hot path on device-resident inputs: every density pass of
the smoothing-length iteration (from the initial h), the ghost passes, the
force pass and the FP64 global sums (sphx_step through the C-ABI). Grid and
task builds are timed separately, outside the step.

value = (N_dens + N_force) / seconds per step, with
  N_dens  = sum_i #{j != i : r_ij < H_i}            at the final h,
  N_force = sum_i #{j != i : r_ij < max(H_i, H_j)}  (active receivers only).

Then (unless --no-serving) the serving stream of 512 independent boxes of
10^3..10^6 particles is run through the continuous-batching server (requests
overlapping in slots of one request each, and in batches, each batch one step
over a grid of independent sets) and through the plain per-call form:
saturated throughput, and p50/p99 latency under Poisson arrivals at 0.5 and
0.8 of the first form's saturated rate (top-level p50_ms/p99_ms are the
one-request-per-slot form at 0.8).

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 FLOPs per accepted directed interaction, counted from the formulas as
# the kernels evaluate them (FMA = 2, sqrt/rsqrt/rcp = 1; compares, min/max and
# selects not counted), with the Wendland C2 kernel.
FLOP_DENSITY = 51
FLOP_FORCE = 84
# The kernel's own share of those counts, for each kernel as written in the
# device code: w(u) and phi(u) in the density loop (both pieces of a spline
# are evaluated), -w'(u) at each end of a force pair.
KERNEL_FLOP_DENSITY = {"wendland_c2": 7, "wendland_c4": 13, "wendland_c6": 18,
                       "cubic_spline": 13, "quartic_spline": 23, "quintic_spline": 27}
KERNEL_FLOP_FORCE_END = {"wendland_c2": 4, "wendland_c4": 8, "wendland_c6": 11,
                         "cubic_spline": 6, "quartic_spline": 13, "quintic_spline": 16}
# FP32 FLOPs per summed pair of the truncated gravity loop, as evaluated:
# separation and r^2 8, rsqrt and r 2, u and u^2 2, f and g by Horner 18, the
# two branches 4, x, x^2 and exp 3, t = 1/(1 + p x) 3, the erfc polynomial 9,
# chi 1, chi'/r 2, the combination 3, the three accelerations 7, the
# potential 3.
FLOP_GRAVITY = 65
KERNEL_NAMES = {"wendland_c2": "Wendland C2", "wendland_c4": "Wendland C4",
                "wendland_c6": "Wendland C6", "cubic_spline": "cubic spline",
                "quartic_spline": "quartic spline", "quintic_spline": "quintic spline"}


def flops_per_interaction(kernel):
    """(density, force) FLOPs per interaction with the given kernel."""
    d = FLOP_DENSITY - KERNEL_FLOP_DENSITY["wendland_c2"] + KERNEL_FLOP_DENSITY[kernel]
    f = FLOP_FORCE + 2 * (KERNEL_FLOP_FORCE_END[kernel] - KERNEL_FLOP_FORCE_END["wendland_c2"])
    return d, f
PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0

CONFIGS = {
    "small": ("4,096-particle jittered lattice (16^3), u=1", lambda inp: inp.config_small(1)),
    "sedov": ("Sedov blast, 64^3 = 262,144 particles on a jittered lattice",
              lambda inp: inp.config_sedov(2)),
    "clustered": ("clustered box, 128^3 = 2,097,152 particles, lognormal sigma=2, P(k)~k^-2",
                  lambda inp: inp.config_clustered(3)),
    "large": ("large clustered box, 256^3 = 16,777,216 particles, lognormal sigma=2.5, "
              "~10% active", lambda inp: inp.config_large(5)),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(ps, make_params, n_recv, seed=0):
    """The oracle (FP64, C + OpenMP, k-d tree candidates) timed on the host
    over the work of a GPU step, for a bounded random sample of receivers: the
    h iteration from the initial h (every density pass, with the oracle's
    candidate search in each) for the receivers and every particle in their
    force neighbourhoods at the initial h, the ghost, and the force pass over
    the receivers. Interactions are counted as on the GPU: the density
    interactions at the final h once, plus the force interactions. Timed on
    all host threads, and on one thread for a sample 4 times smaller. The
    oracle's candidate search (scipy k-d tree queries, one thread) is part of
    every pass and takes most of the time.
    (Neighbours outside the sampled neighbourhoods carry no ghost state: their
    force terms are NaN, which costs the same time.)"""
    import ctypes

    import numpy as np
    import oracle
    P = make_params()
    u_all = np.asarray(ps.u, np.float64)
    h0 = np.asarray(ps.h, np.float64)

    def run(n):
        rng = np.random.default_rng(seed)
        recv = np.sort(rng.choice(ps.n, size=min(n, ps.n), replace=False))
        t0 = time.perf_counter()
        need = oracle.force_needed(ps, h0, P, recv, mode="tree")
        h, dens, conv, iters, passes = oracle.solve_h(ps, P, recv=need, mode="tree")
        g = oracle.ghost(dens, u_all[need], h, P)
        h_all = h0.copy()
        h_all[need] = h
        full = {k: np.full(ps.n, np.nan) for k in ("P", "c", "f", "balsara")}
        for k in full:
            full[k][need] = g[k]
        rho = np.full(ps.n, np.nan)
        rho[need] = dens["rho"]
        fo = oracle.force(ps, h_all, full, rho, P, recv=recv, mode="tree")
        dt = time.perf_counter() - t0
        n_int = int(dens["nngb"].sum()) + int(fo["total"])
        return n_int / dt, ("%d random receivers and their %d force neighbours: %d h-iteration "
                            "passes (candidate search included), ghost, force for the "
                            "receivers; %d interactions in %.1f s" % (
                                len(recv), len(need) - len(recv), passes, n_int, dt))

    gomp = ctypes.CDLL("libgomp.so.1")  # the OpenMP runtime the oracle runs on
    threads = int(gomp.omp_get_max_threads())
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                         "")
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    rate, sample = run(n_recv)
    gomp.omp_set_num_threads(1)
    try:
        rate1, sample1 = run(max(1, n_recv // 4))
    finally:
        gomp.omp_set_num_threads(threads)
    return {"value": rate, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": sample, "value_1core": rate1, "sample_1core": sample1,
            "cores_are": "OpenMP threads of the oracle's loops (its k-d tree candidate search "
                         "runs on one thread)",
            "host_cpu_model": model, "host_logical_cpus": os.cpu_count(),
            "host_cpus_usable": usable}


# The batched serving form: slots and the most particles of one batch.
BATCH_SLOTS = 6
BATCH_PARTICLES = 1 << 23


def serving_bench(slots, n_req, seed=4):
    """The serving stream: n_req independent periodic boxes (N log-uniform in
    [1e3, 1e6], lattice or lognormal by a seeded coin) with inputs resident in
    HBM. Runs it saturated (all requests queued at t=0) with `slots` slots of
    one request each, in batches (BATCH_SLOTS slots, each running the waiting
    requests as one step over a grid of independent sets), and with one slot
    (the plain per-call form), then with seeded Poisson arrivals at 0.5 and
    0.8 times the first form's saturated request rate, for all three forms.
    Latency = completion - arrival."""
    import numpy as np
    import torch
    from paper_2305_13380_amd import inputs, serve, sphx
    t0 = time.perf_counter()
    sizes, lattice = inputs.serving_sizes(n_req, seed)
    dev = []
    for k in range(n_req):
        dev.append(sphx.DeviceParticles.from_set(
            inputs.serving_request(k, int(sizes[k]), bool(lattice[k]), seed), "cuda:0"))
    torch.cuda.synchronize()
    n_tot = sum(d.n for d in dev)
    log("bench: serving: %d requests, %d particles generated and uploaded in %.1f s" % (
        n_req, n_tot, time.perf_counter() - t0))
    servers = {"served": serve.Server(n_slots=slots),
               "batched": serve.Server(n_slots=BATCH_SLOTS, batch_particles=BATCH_PARTICLES),
               "per_call": serve.Server(n_slots=1)}
    warm = [(k, 0.0, dev[k].n) for k in range(min(16, n_req))]
    for srv in servers.values():
        srv.run(warm, lambda k: dev[k])

    def run(form, rate):
        if rate is None:
            arr = np.zeros(n_req)
        else:
            rng = np.random.default_rng(seed + 7919)
            arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
        spec = [(k, float(arr[k]), dev[k].n) for k in range(n_req)]
        res = servers[form].run(spec, lambda k: dev[k])
        bad = [r for r in res if r.error is not None or r.status < 0]
        if bad:
            raise RuntimeError("serving: request %d failed: %s" % (bad[0].rid, bad[0].error))
        span = max(r.done for r in res) - (0.0 if rate is None else float(arr[0]))
        q = serve.percentiles(res)
        rec = {"requests_per_s": n_req / span, "interactions_per_s":
               sum(r.interactions for r in res) / span, "makespan_s": span,
               "p50_ms": q["p50_s"] * 1e3, "p99_ms": q["p99_s"] * 1e3,
               "peak_running": servers[form].peak_running}
        if rate is not None:
            rec["arrival_rate_per_s"] = rate
        log("bench: serving %s rate=%s: %s" % (form, rate, json.dumps(rec)))
        return rec, res

    out = {"requests": n_req, "particles": n_tot, "slots": slots, "seed": seed,
           "inputs": "resident in HBM; each request builds its grid and tasks, runs the "
                     "h iteration, ghost, force and FP64 sums, and copies back its "
                     "interaction counts"}
    sat, res_sat = run("served", None)
    satb, _ = run("batched", None)
    sat1, _ = run("per_call", None)
    out["saturated"] = {"served": sat, "batched": satb, "per_call": sat1,
                        "speedup": sat["requests_per_s"] / sat1["requests_per_s"],
                        "batched_speedup": satb["requests_per_s"] / sat1["requests_per_s"]}
    out["batched_form"] = {"slots": BATCH_SLOTS, "batch_particles": BATCH_PARTICLES,
                           "what": "a free slot runs the requests waiting for it, in arrival "
                                   "order up to batch_particles particles, as one step over "
                                   "a grid of independent sets (sphx_grid_build_sets)"}
    out["interactions"] = sum(r.interactions for r in res_sat)
    for frac in (0.5, 0.8):
        rate = frac * sat["requests_per_s"]
        out["poisson_%.1f" % frac] = {"served": run("served", rate)[0],
                                      "batched": run("batched", rate)[0],
                                      "per_call": run("per_call", rate)[0]}
    for srv in servers.values():
        srv.close()
    return out


def fof_bench(params, dp, reps):
    """Friends-of-friends groups of the workload at 0.2 of the mean particle
    separation (sphx_fof: cell and task build at that radius, the link loop,
    labels), inputs resident in HBM; one warm-up call, then the shortest of
    `reps` timed calls (host clock around a call and a device sync)."""
    import numpy as np
    import torch
    from paper_2305_13380_amd import sphx
    ctx = sphx.Context(params, 0)
    vol = float(np.prod(np.asarray(params.box)))
    b = 0.2 * (vol / dp.n) ** (1.0 / 3.0)
    group, gsize, counts = sphx.fof(ctx, dp, b)
    torch.cuda.synchronize()
    times = []
    for _ in range(max(1, reps)):
        t0 = time.perf_counter()
        group, gsize, counts = sphx.fof(ctx, dp, b)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    c = counts.cpu().numpy()
    biggest = int(torch.bincount(group.to(torch.int64)).max()) if dp.n else 0
    ctx.close()
    t = min(times)
    rec = {"link_length": b, "link_length_of_mean_separation": 0.2, "ms": t * 1e3,
           "particles_per_s": dp.n / t, "groups": int(c[0]), "links": int(c[1]),
           "largest_group": biggest, "reps": len(times),
           "timed": "whole sphx_fof call: cell and task build at radius b, link loop, labels"}
    log("bench: fof: %s" % json.dumps(rec))
    return rec


def gravity_bench(params, dp, reps):
    """Short-range softened gravity of the workload by direct summation
    (sphx_gravity) at G = 1, softening support H = 0.12, truncation scale
    r_s = 1.25 and summation radius r_p2p = 1.25 mean particle separations:
    one warm-up call, then the shortest of `reps` timed calls (host clock
    around a call and a device sync), and the gravity kernel's own time from
    the library's event profiler."""
    import numpy as np
    import torch
    from paper_2305_13380_amd import sphx
    ctx = sphx.Context(params, 0)
    d = (float(np.prod(np.asarray(params.box))) / dp.n) ** (1.0 / 3.0)
    H, rs, rp = 0.12 * d, 1.25 * d, 1.25 * d
    pairs = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    sphx.gravity(ctx, dp, 1.0, H, rs, rp, pairs=pairs)
    torch.cuda.synchronize()
    times = []
    ctx.profile(True)
    for _ in range(max(1, reps)):
        t0 = time.perf_counter()
        sphx.gravity(ctx, dp, 1.0, H, rs, rp, pairs=pairs)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    k_ms, k_n = ctx.profile_read(4)
    ctx.close()
    npairs = int(pairs.item())
    kern_s = k_ms / 1e3 / max(k_n, 1)
    rec = {"G": 1.0, "H": H, "r_s": rs, "r_p2p": rp, "of_mean_separation": [0.12, 1.25, 1.25],
           "pairs": npairs, "ms": min(times) * 1e3, "kernel_ms": kern_s * 1e3,
           "pairs_per_s": npairs / kern_s if kern_s > 0 else None,
           "kernel_tflops_algorithmic": npairs * FLOP_GRAVITY / kern_s / 1e12 if kern_s > 0 else None,
           "roofline": {"bound": "alu", "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                        "frac": (npairs * FLOP_GRAVITY / kern_s / 1e12 / PEAK_FP32_TFLOPS
                                 if kern_s > 0 else None)},
           "flop_per_pair": FLOP_GRAVITY, "reps": len(times),
           "timed": "ms: whole sphx_gravity call (cell and task build at r_p2p, the loop); "
                    "kernel_ms: the loop alone"}
    log("bench: gravity: %s" % json.dumps(rec))
    return rec


def graph_slots(info, params):
    """Captured pass slots for steps like the one `info` describes: its passes,
    one more when it rebuilt its task list (the first pass of a step can meet
    the previous step's list stale and is repeated), at most max_iter - 1."""
    k = info.passes + (1 if info.task_rebuilds > 0 else 0)
    return max(0, min(k, params.max_iter - 1, 64))


def time_steps(params, dp, out, h0, k, n=3):
    """Average HIP-event time of n whole steps with graph_passes = k (after one
    untimed step on fresh grid and tasks, which also captures the graph)."""
    import torch
    from paper_2305_13380_amd import sphx
    p = type(params).from_buffer_copy(params)
    p.graph_passes = k
    ctx = sphx.Context(p, 0)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    dp.t["h"].copy_(h0)
    sphx.step(ctx, grid, tasks, dp, out)
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(n):
        dp.t["h"].copy_(h0)
        sphx.step(ctx, grid, tasks, dp, out)
    b.record(stream)
    torch.cuda.synchronize()
    tasks.close()
    grid.close()
    ctx.close()
    return a.elapsed_time(b) / n


def choose_graph(params, dp, out, h0, info):
    """Captured pass slots for the timed steps (graph_slots of a warm-up
    step's info), kept only if the captured step is faster than pass by pass
    on a few steps (on a box whose step needs no rebuild the gated rebuild
    kernels of every slot can cost more than the per-pass readbacks they
    save). Returns (slots, {"captured_ms", "pass_by_pass_ms"})."""
    k = graph_slots(info, params)
    if k == 0:
        return 0, None
    t_g = time_steps(params, dp, out, h0, k)
    t_0 = time_steps(params, dp, out, h0, 0)
    return (k if t_g < t_0 else 0), {"slots": k, "captured_ms": t_g, "pass_by_pass_ms": t_0}


def step_leg(name, params, steps=5, warmup=1, flavour=None, graph=-1, tune=False):
    """One more workload of the step, timed like the headline one (HIP events
    on the stream around `steps` whole steps from the generator's h, inputs
    resident): the Sedov box and the large box with its active subset (after
    an untimed all-active step that gives the inactive particles their
    state), or the headline box with another SPH flavour (the density-entropy
    one with A set from u, the smoothed-pressure and GDF ones on the same
    u); tune: the leg's loop shapes by the autotuner on its own workload."""
    import numpy as np
    import torch
    from paper_2305_13380_amd import inputs, sphx
    desc, make = CONFIGS[name]
    t0 = time.perf_counter()
    ps = make(inputs)
    if flavour == "entropy":
        # the same particles carrying the adiabat A = (gamma - 1) u / rho^(gamma - 1),
        # rho from one density pass at the generator's h (on the GPU)
        c0 = sphx.Context(params, 0)
        d0 = sphx.DeviceParticles.from_set(ps, "cuda:0")
        o0 = sphx.Outputs(ps.n, "cuda:0")
        g0 = sphx.Grid(c0, d0)
        k0 = sphx.Tasks(c0, g0, d0)
        sphx.fixed_h_pass(c0, g0, k0, d0, o0)
        rho = o0.d["rho"].cpu().numpy().astype(np.float64)
        k0.close()
        g0.close()
        c0.close()
        gam = 5.0 / 3.0
        ps.u = np.ascontiguousarray(((gam - 1.0) * ps.u.astype(np.float64)
                                     / rho ** (gam - 1.0)).astype(np.float32))
        params = type(params).from_buffer_copy(params)
        params.flavour = sphx.FLAVOURS["entropy"]
    elif flavour in ("pressure_energy", "anarchy_pu"):
        # the smoothed-pressure flavours run the plain cell-pair density loop
        # (the tuned tile and wave count are kept)
        params = type(params).from_buffer_copy(params)
        params.flavour = sphx.FLAVOURS[flavour]
        params.density_balance = 0
        params.neighbour_lists = 0
    elif flavour == "gdf":
        # the density flavours' loops, then the GDF loop inside the step
        params = type(params).from_buffer_copy(params)
        params.flavour = sphx.FLAVOURS[flavour]
    dp = sphx.DeviceParticles.from_set(ps, "cuda:0")
    out = sphx.Outputs(ps.n, "cuda:0")
    if dp.t["active"] is not None:
        act = dp.t["active"]
        h_guess = dp.t["h"].clone()
        dp.t["active"] = None
        c1 = sphx.Context(params, 0)
        g1 = sphx.Grid(c1, dp)
        k1 = sphx.Tasks(c1, g1, dp)
        sphx.step(c1, g1, k1, dp, out)
        k1.close()
        g1.close()
        c1.close()
        dp.t["active"] = act
        dp.t["h"].copy_(torch.where(act.bool(), h_guess, dp.t["h"]))
    shapes = None
    if tune:
        # the flavour's own loop shapes (its loops differ from the headline
        # flavour's), by the autotuner on this workload at its initial h
        c0 = sphx.Context(params, 0)
        g0 = sphx.Grid(c0, dp)
        k0 = sphx.Tasks(c0, g0, dp)
        params = sphx.autotune(c0, g0, k0, dp, out, reps=3)
        torch.cuda.synchronize()
        k0.close()
        g0.close()
        c0.close()
        shapes = {k: getattr(params, k) for k in ("density_tile", "density_waves",
                                                  "density_balance", "force_tile", "force_waves")}
    h0 = dp.t["h"].clone()
    # the warm-up pass by pass, then the timed steps captured (graph_slots)
    p0 = type(params).from_buffer_copy(params)
    p0.graph_passes = 0
    ctx0 = sphx.Context(p0, 0)
    grid = sphx.Grid(ctx0, dp)
    tasks = sphx.Tasks(ctx0, grid, dp)
    for _ in range(max(warmup, 1)):
        dp.t["h"].copy_(h0)
        info = sphx.step(ctx0, grid, tasks, dp, out)[1]
    tasks.close()
    grid.close()
    ctx0.close()
    params = type(params).from_buffer_copy(params)
    choice = None
    if graph < 0:
        params.graph_passes, choice = choose_graph(params, dp, out, h0, info)
    else:
        params.graph_passes = graph
    ctx = sphx.Context(params, 0)
    grid = sphx.Grid(ctx, dp)
    tasks = sphx.Tasks(ctx, grid, dp)
    dp.t["h"].copy_(h0)
    sphx.step(ctx, grid, tasks, dp, out)  # (captures the graph)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    infos = []
    a.record(stream)
    for _ in range(steps):
        dp.t["h"].copy_(h0)
        infos.append(sphx.step(ctx, grid, tasks, dp, out)[1])
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    recv = dp.t["active"].bool() if dp.t["active"] is not None else slice(None)
    n_dens = int(out.d["nngb"].to(torch.int64)[recv].sum())
    n_force = int(out.f["nforce"].to(torch.int64)[recv].sum())
    sums = out.sums.cpu().numpy()
    rec = {"workload": desc, "n_particles": ps.n,
           "active": int(dp.t["active"].sum()) if dp.t["active"] is not None else ps.n,
           "flavour": flavour or "energy", "ms_per_step": ms,
           "interactions_per_s": (n_dens + n_force) / (ms / 1e3), "n_dens": n_dens,
           "n_force": n_force, "density_passes": infos[-1].passes,
           "task_rebuilds_per_step": infos[-1].task_rebuilds,
           "graph_passes": int(params.graph_passes), "graph_choice": choice, "steps": steps,
           "loop_shapes": shapes if shapes is not None else "the headline's",
           "momentum_err_rel": float(np.abs(sums[:3]).max() / max(sums[4], 1e-300)),
           "timed": "HIP events on the stream around whole steps from the generator's h "
                    "(h iteration with task rebuilds, ghost, force, FP64 sums); inputs "
                    "resident; %.1f s with the set-up" % (time.perf_counter() - t0)}
    tasks.close()
    grid.close()
    ctx.close()
    log("bench: step leg %s%s: %s" % (name, " " + flavour if flavour else "", json.dumps(rec)))
    return rec


def sphenix_leg(params, n_steps=20):
    """The SPHENIX row as a run: the Sedov box (64^3 jittered lattice, one unit
    of energy in the central 32 particles) integrated over n_steps leapfrog
    steps with one global step size (paper_2305_13380_amd.sphenix): each step
    drifts, builds a new grid and task list, iterates h, runs the ghost and
    force pass, the viscosity switch, the gradient loop, the conduction
    parameter and the step-size limiter. Timed on the host clock (the step
    size is read back every step), after three untimed steps."""
    import torch
    from paper_2305_13380_amd import inputs
    from paper_2305_13380_amd.sphenix import SphenixRun
    ps = inputs.config_sedov(2)
    ps.alpha_v[:] = 0.1
    ps.alpha_c[:] = 0.0
    run = SphenixRun(ps, params, c_cfl=0.1)
    # interactions summed on the device (no read-back inside the loop)
    n_dev = torch.zeros((), dtype=torch.int64, device=run.out.d["nngb"].device)
    for _ in range(3):  # warm-up, the counting included
        run.step()
        n_dev += run.out.d["nngb"].sum(dtype=torch.int64)
        n_dev += run.out.f["nforce"].sum(dtype=torch.int64)
    n_dev.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        run.step()
        n_dev += run.out.d["nngb"].sum(dtype=torch.int64)
        n_dev += run.out.f["nforce"].sum(dtype=torch.int64)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_int = int(n_dev.item())
    rec = {"workload": CONFIGS["sedov"][0] + ", multi-step SPHENIX", "steps": n_steps,
           "ms_per_step": wall / n_steps * 1e3, "interactions_per_s": n_int / wall,
           "t_end": run.state.t,
           "timed": "host clock over whole leapfrog steps (kick, drift, grid and task build, "
                    "h iteration, ghost, force, viscosity switch, gradient loop, conduction "
                    "parameter, step size with its read-back)"}
    run.close()
    log("bench: sphenix run: %s" % json.dumps(rec))
    return rec


def switch_bench(params, n, reps=200, sets=6):
    """The SPHENIX viscosity switch over n particles (sphx_alpha_v_update),
    inputs resident in HBM: reps launches timed with events on the stream they
    run on; 28 bytes per particle (six FP32 words read, one written). The
    launches rotate over `sets` independent input sets whose total exceeds
    the device's 256 MB last-level cache, so each launch streams from HBM."""
    import torch
    from paper_2305_13380_amd import sphx
    ctx = sphx.Context(params, 0)
    g = torch.Generator(device="cuda:0").manual_seed(7)
    t = [[torch.rand(n, device="cuda:0", generator=g) for _ in range(6)] for _ in range(sets)]
    for x in t:
        sphx.alpha_v_update(ctx, x[0], x[1], x[2], x[3], x[4], x[5], 1e-3)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for k in range(reps):
        x = t[k % sets]
        sphx.alpha_v_update(ctx, x[0], x[1], x[2], x[3], x[4], x[5], 1e-3)
    b.record(stream)
    torch.cuda.synchronize()
    per = a.elapsed_time(b) / reps / 1e3
    ctx.close()
    rec = {"particles": n, "us_per_launch": per * 1e6, "bytes_per_particle": 28,
           "GB_per_s": 28.0 * n / per / 1e9, "of_hbm_peak": 28.0 * n / per / 1e9 / PEAK_HBM_GBS,
           "reps": reps, "input_sets": sets,
           "working_set_MB": 28.0 * n * sets / 1e6,
           "timed": "back-to-back launches rotating over the input sets (more than the "
                    "256 MB last-level cache), events on the launch stream"}
    log("bench: viscosity switch: %s" % json.dumps(rec))
    return rec


def oracle_beside(ps, fof_rec, grav_rec, sw_rec, n_recv=2048, seed=0):
    """The oracle timed on the host for the rows beyond the step, on the same
    workload: friends-of-friends of the whole box (k-d tree candidates,
    sequential union-find), short-range gravity for a random sample of
    receivers (all their pairs, FP64), and the viscosity switch of every
    particle. Threads as the oracle uses them (OpenMP in the gravity sum)."""
    import numpy as np
    import oracle
    out = {}
    if fof_rec is not None:
        t0 = time.perf_counter()
        _, links = oracle.fof(ps, fof_rec["link_length"], mode="tree")
        t = time.perf_counter() - t0
        out["fof"] = {"particles_per_s": ps.n / t, "s": t, "links": links, "kind": "oracle",
                      "sample": "the whole box"}
    if grav_rec is not None:
        recv = np.sort(np.random.default_rng(seed).choice(ps.n, size=min(n_recv, ps.n),
                                                          replace=False))
        oracle.gravity(ps, 1.0, grav_rec["H"], grav_rec["r_s"], grav_rec["r_p2p"],
                       recv=recv[:16], mode="tree")  # the k-d tree, built once
        t0 = time.perf_counter()
        o = oracle.gravity(ps, 1.0, grav_rec["H"], grav_rec["r_s"], grav_rec["r_p2p"],
                           recv=recv, mode="tree")
        t = time.perf_counter() - t0
        out["gravity"] = {"pairs_per_s": o["pairs"] / t, "s": t, "pairs": o["pairs"],
                          "kind": "oracle", "sample": "%d random receivers" % len(recv)}
    if sw_rec is not None:
        rng = np.random.default_rng(seed)
        a = [rng.random(ps.n) for _ in range(6)]
        t0 = time.perf_counter()
        oracle.alpha_v_update(a[0], a[1], a[2], a[3], a[4], a[5], 1e-3, oracle.Params())
        t = time.perf_counter() - t0
        out["viscosity_switch"] = {"particles_per_s": ps.n / t, "s": t, "kind": "oracle",
                                   "sample": "every particle"}
    log("bench: oracle beside the other rows: %s" % json.dumps(out))
    return out


def measured_traffic(config, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<config>.json: FETCH_SIZE and WRITE_SIZE scaled by a
    plain copy of known size), or None when the summary is missing or the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % config)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    if kernel_source_hash(kernel) != rec["source_hash"]:
        return None
    return rec["mean_bytes_per_launch"]


def measured_counter_rate(config, kernel):
    """FP32 VALU rate of `kernel` counted by the hardware (issued ADD, MUL,
    2 x FMA and TRANS FP32 lane operations per second) from the committed
    counter summary (profiles/valu_<config>.json), or None when it is missing
    or the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "valu_%s.json" % config)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec or kernel_source_hash(kernel) != rec["source_hash"]:
        return None
    return rec["counter_tflops"]


def kernel_source_hash(kernel):
    """Hash of the sources a neighbour-loop kernel is compiled from, with
    comments and blank space removed (a comment cannot change the kernel)."""
    import hashlib
    import re
    base = os.path.join(ROOT, "paper_2305_13380_amd", "csrc")
    srcs = {"k_density": ["density.hip", "pairs.h", "kernel_shapes.h", "sphx_internal.h"],
            "k_force": ["force.hip", "pairs.h", "kernel_shapes.h", "sphx_internal.h"]}[kernel]
    hsh = hashlib.sha256()
    for f in srcs:
        text = open(os.path.join(base, f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        hsh.update(" ".join(text.split()).encode())
    return hsh.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="clustered", choices=sorted(CONFIGS))
    ap.add_argument("--cpu-receivers", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", type=int, default=-1, metavar="K",
                    help="captured pass slots per step (HIP graph, task rebuilds inside); "
                         "0: pass by pass; -1 (default): the passes of a warm-up step, one "
                         "more if it rebuilt its task list (also for the step legs)")
    ap.add_argument("--skin", type=float, default=0.1,
                    help="relative enlargement of the task search radii")
    ap.add_argument("--leaf-max", type=int, default=64,
                    help="particles per leaf cell (8..64)")
    ap.add_argument("--kernel", default="wendland_c2", choices=sorted(KERNEL_NAMES),
                    help="smoothing kernel (default Wendland C2)")
    ap.add_argument("--flavour", default="energy", choices=["energy", "gdf"],
                    help="SPH flavour of the timed step: density-energy (default) or GDF "
                         "(the same density loop, then the GDF loop and its force law)")
    ap.add_argument("--no-tune", action="store_true",
                    help="default loop shapes instead of the autotuner's")
    ap.add_argument("--shape", default="", metavar="DT,DW,FT,FW[,DB]",
                    help="fixed loop shapes (density tile, density waves, force tile, force "
                         "waves, density rounds: 0 per lane, 2 grouped) instead of the "
                         "autotuner's")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving-stream latency measurement")
    ap.add_argument("--no-fof", action="store_true",
                    help="skip the friends-of-friends timing on the workload")
    ap.add_argument("--fof-reps", type=int, default=5,
                    help="timed calls of the friends-of-friends and gravity legs")
    ap.add_argument("--no-gravity", action="store_true",
                    help="skip the direct-summation gravity timing on the workload")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the other workloads of the step (Sedov box, large box, "
                         "the density-entropy, pressure-energy, Anarchy-PU and GDF flavours) "
                         "and the multi-step SPHENIX run")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        nbytes = args.calibrate_copy << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2305_13380_amd import inputs, sphx

    desc, make = CONFIGS[args.config]
    t0 = time.perf_counter()
    ps = make(inputs)
    log("bench: %s: N=%d generated in %.1f s" % (args.config, ps.n, time.perf_counter() - t0))

    dev = "cuda:0"
    params = sphx.default_params(leaf_max=args.leaf_max, skin=args.skin, kernel=args.kernel,
                                 flavour=args.flavour)
    dp = sphx.DeviceParticles.from_set(ps, dev)
    out = sphx.Outputs(ps.n, dev)
    stream = torch.cuda.current_stream()
    if dp.t["active"] is not None:
        # Time-step bins: an untimed all-active step gives every particle the
        # state (h, rho, P, c, f, B, A) it carries as an inactive neighbour.
        t0 = time.perf_counter()
        act = dp.t["active"]
        h_guess = dp.t["h"].clone()
        dp.t["active"] = None
        c_all = sphx.Context(params, 0)
        g_all = sphx.Grid(c_all, dp)
        k_all = sphx.Tasks(c_all, g_all, dp)
        sphx.step(c_all, g_all, k_all, dp, out)
        torch.cuda.synchronize()
        k_all.close()
        g_all.close()
        c_all.close()
        dp.t["active"] = act
        # the active particles start from the generator's guess, as in the
        # other workloads; only the inactive ones keep the converged h
        dp.t["h"].copy_(torch.where(act.bool(), h_guess, dp.t["h"]))
        log("bench: all-active step for the inactive particles' state: %.2f s" % (
            time.perf_counter() - t0))
    h0 = dp.t["h"].clone()
    torch.cuda.synchronize()
    shapes = "default"
    if args.shape:
        sh = [int(x) for x in args.shape.split(",")]
        dt, dw, ft, fw = sh[:4]
        db = sh[4] if len(sh) > 4 else 0
        params.density_tile, params.density_waves, params.density_balance = dt, dw, db
        params.force_tile, params.force_waves = ft, fw
        shapes = {"density_tile": dt, "density_waves": dw, "density_balance": db,
                  "force_tile": ft, "force_waves": fw}
    elif not args.no_tune:
        # Loop shapes by the library's autotuner, on this workload at its
        # initial h (outside the timed region).
        t0 = time.perf_counter()
        c0 = sphx.Context(params, 0)
        g0 = sphx.Grid(c0, dp)
        k0 = sphx.Tasks(c0, g0, dp)
        params = sphx.autotune(c0, g0, k0, dp, out, reps=3)
        torch.cuda.synchronize()
        k0.close()
        g0.close()
        c0.close()
        shapes = {k: getattr(params, k) for k in ("density_tile", "density_waves",
                                                  "density_balance", "force_tile", "force_waves")}
        log("bench: autotune %.1f s -> %s" % (time.perf_counter() - t0, shapes))
    def run_steps(c, g, t, k):
        infos = []
        for _ in range(k):
            dp.t["h"].copy_(h0)
            st, info = sphx.step(c, g, t, dp, out)
            infos.append(info)
        return infos

    # Pass by pass: warm-up, and the kernel durations (HIP events around every
    # neighbour-loop launch on the stream it runs on).
    params.graph_passes = 0
    ctxp = sphx.Context(params, 0)
    gridp = sphx.Grid(ctxp, dp)
    tasksp = sphx.Tasks(ctxp, gridp, dp)
    for w, info in enumerate(run_steps(ctxp, gridp, tasksp, max(args.warmup, 1))):
        log("bench: warmup %d: passes=%d rebuilds=%d" % (w, info.passes, info.task_rebuilds))
    # Captured passes: as many slots as the warm-up step's passes, plus one for
    # a first pass that meets the previous step's task list stale (task
    # rebuilds run inside the graph; a step that needs more goes on pass by
    # pass), kept if a few captured steps beat a few pass-by-pass ones.
    graph_k = args.graph
    graph_choice = None
    if graph_k < 0:
        graph_k, graph_choice = choose_graph(params, dp, out, h0, info)
    torch.cuda.synchronize()
    sphx.probe_read(ctxp, clear=True)
    ctxp.profile(True)
    run_steps(ctxp, gridp, tasksp, args.steps)
    torch.cuda.synchronize()
    ctxp.profile(False)
    # neighbour-test counters of a measurement build (SPHX_PROBE=1)
    probe_on, probe = sphx.probe_read(ctxp, clear=True)
    dens_ms, dens_n = ctxp.profile_read(0)
    force_ms, force_n = ctxp.profile_read(1)
    dlist_ms, dlist_n = ctxp.profile_read(2)
    build_ms, build_n = ctxp.profile_read(3)
    tasksp.close()
    gridp.close()
    ctxp.close()

    # The timed steps.
    params.graph_passes = graph_k
    ctx = sphx.Context(params, 0)
    t0 = time.perf_counter()
    grid = sphx.Grid(ctx, dp)
    torch.cuda.synchronize()
    t_grid = time.perf_counter() - t0
    t0 = time.perf_counter()
    tasks = sphx.Tasks(ctx, grid, dp)
    torch.cuda.synchronize()
    t_tasks = time.perf_counter() - t0
    log("bench: grid %.1f ms (%d leaves), tasks %.1f ms (%d tasks), %d captured passes" % (
        t_grid * 1e3, grid.n_leaves, t_tasks * 1e3, tasks.count, graph_k))
    run_steps(ctx, grid, tasks, 1)  # (captures the graph)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    infos = run_steps(ctx, grid, tasks, args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_ev = start.elapsed_time(stop) / 1e3
    ms_step = t_ev / args.steps * 1e3
    info = infos[-1]
    infos = [(i.passes, i.task_rebuilds, i.unconverged) for i in infos]
    log("bench: %d steps in %.3f s (events) / %.3f s (wall); cell-pair density %.2f ms over %d "
        "launches, list density %.2f ms over %d, list build %.2f ms over %d, force %.2f ms "
        "over %d" % (args.steps, t_ev, wall, dens_ms, dens_n, dlist_ms, dlist_n, build_ms,
                     build_n, force_ms, force_n))

    nngb = out.d["nngb"].to(torch.int64)
    nf = out.f["nforce"].to(torch.int64)
    if dp.t["active"] is not None:
        act = dp.t["active"].bool()
        n_dens = int(nngb[act].sum())
        n_force = int(nf[act].sum())
    else:
        n_dens = int(nngb.sum())
        n_force = int(nf.sum())
    inter = n_dens + n_force
    value = inter / (t_ev / args.steps)
    sums = out.sums.cpu().numpy()
    mom = float(np.abs(sums[:3]).max() / max(sums[4], 1e-300))
    en = float(abs(sums[3]) / max(sums[4] + sums[5], 1e-300))

    # Algorithmic FLOP rates of the neighbour-loop kernels: the interactions
    # each computes per step (the step is deterministic, so every timed step
    # computes the same) times the FLOPs per interaction, over the kernel's own
    # event-timed duration per step.
    S = args.steps
    fl_d, fl_f = flops_per_interaction(args.kernel)
    kern_units = {"k_density": (info.pairs_cellpair * fl_d, dens_ms / S, dens_n / S),
                  "k_dens_list": (info.pairs_list * fl_d, dlist_ms / S, dlist_n / S),
                  "k_force": (n_force * fl_f, force_ms / S, force_n / S)}
    rates = {k: (f / (ms / 1e3) / 1e12 if ms > 0 else 0.0) for k, (f, ms, _) in kern_units.items()}
    kern = max(kern_units, key=lambda k: kern_units[k][1])
    flops_step, _, launches_step = kern_units[kern]
    achieved = rates[kern]
    per_launch = flops_step / max(launches_step, 1)
    passes = sorted(set(p for p, _, _ in infos))
    line = {
        "metric": "SPH pair interactions/s (density+force) at 1 GPU",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n_particles": ps.n, "seed": ps.meta.get("seed"),
                   "kernel": KERNEL_NAMES[args.kernel], "flavour": args.flavour,
                   "eta": ps.eta, "h_tol": 1e-4,
                   "positions": "f64 (cell offsets f64, pair arithmetic f32)",
                   "n_dens": n_dens, "n_force": n_force, "density_passes": passes,
                   "task_rebuilds_per_step": infos[-1][1], "unconverged": infos[-1][2],
                   "n_leaves": grid.n_leaves, "n_tasks": tasks.count,
                   "grid_build_ms": t_grid * 1e3, "tasks_build_ms": t_tasks * 1e3,
                   "kernel_ms_per_step": {"k_density": dens_ms / S, "k_dens_list": dlist_ms / S,
                                          "k_list_build": build_ms / S, "k_force": force_ms / S},
                   "kernel_tflops": rates,
                   "density_pairs_per_step": {"cell_pair": info.pairs_cellpair,
                                              "list": info.pairs_list},
                   "list_builds_per_step": info.list_builds,
                   "list_fallback_receiver_passes": info.list_fallback,
                   "list_entries": info.list_entries, "loop_shapes": shapes,
                   "graph_passes": graph_k, "graph_choice": graph_choice,
                   "leaf_max": args.leaf_max, "skin": args.skin,
                   "momentum_err_rel": mom, "energy_err_rel": en},
        "roofline": {"bound": "alu", "kernel": kern, "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     # (the committed counter records are of the default kernel)
                     "traffic": (measured_traffic(args.config, kern)
                                 if args.kernel == "wendland_c2" else None),
                     "counter_tflops": (measured_counter_rate(args.config, kern)
                                        if args.kernel == "wendland_c2" else None),
                     "flop_per_launch": per_launch},
    }
    if probe_on and probe[2] > 0:
        line["probe"] = {
            "lane_slots_per_accepted_pair": probe[0] / probe[2],
            "receiver_lane_tests_per_accepted_pair": probe[1] / probe[2],
            "compute_lane_slot_fill": probe[4] / max(probe[3], 1),
            "accepted_pairs": probe[2], "steps": args.steps,
            "what": "cell-pair density loop of a measurement build (SPHX_PROBE=1): lane slots "
                    "of its candidate tests, the tests of lanes holding a receiver, accepted "
                    "pairs (own particle included); the share of its per-lane compute "
                    "loops' lane slots that evaluate a list entry"}
    del grid, tasks, out
    if not args.no_legs and args.config == "clustered":
        # the flavour legs tune their own loop shapes unless the headline's
        # were fixed (--no-tune, --shape)
        tune_legs = not args.no_tune and not args.shape
        line["other_workloads"] = {
            "sedov": step_leg("sedov", params, steps=10, graph=args.graph),
            "large": step_leg("large", params, steps=3, graph=args.graph),
            "clustered_entropy": step_leg("clustered", params, steps=5, flavour="entropy",
                                          graph=args.graph, tune=tune_legs),
            "clustered_pressure_energy": step_leg("clustered", params, steps=5,
                                                  flavour="pressure_energy", graph=args.graph,
                                                  tune=tune_legs),
            "clustered_anarchy_pu": step_leg("clustered", params, steps=5, flavour="anarchy_pu",
                                             graph=args.graph, tune=tune_legs),
            "clustered_gdf": step_leg("clustered", params, steps=5, flavour="gdf",
                                      graph=args.graph, tune=tune_legs),
        }
        line["sphenix_run"] = sphenix_leg(params)
    if not args.no_fof:
        line["fof"] = fof_bench(params, dp, args.fof_reps)
    if not args.no_gravity:
        line["gravity"] = gravity_bench(params, dp, args.fof_reps)
        line["viscosity_switch"] = switch_bench(params, dp.n)
    if not args.no_serving:
        sv = serving_bench(args.serving_slots, args.serving_requests)
        line["serving"] = sv
        line["p50_ms"] = sv["poisson_0.8"]["served"]["p50_ms"]
        line["p99_ms"] = sv["poisson_0.8"]["served"]["p99_ms"]
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host ...")
        import oracle
        line["cpu_baseline"] = cpu_baseline(
            ps, lambda: oracle.Params.with_kernel(args.kernel), args.cpu_receivers)
        line["cpu_oracle_other_rows"] = oracle_beside(
            ps, line.get("fof"), line.get("gravity"), line.get("viscosity_switch"))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
