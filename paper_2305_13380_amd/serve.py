"""Continuous-batching request loop over the sphx C-ABI.

Requests are independent periodic particle sets of different sizes arriving
on a clock. A dispatcher admits them in arrival order as soon as a slot is
free and their device footprint (inputs, outputs and the library workspace,
``sphx_workspace_bytes``) fits in the HBM budget; a request that does not fit
waits (it is never started to fail with out-of-memory). Each slot owns one
library context and one HIP stream and runs its request's whole step
(upload, grid build, task build, h iteration, force, download) on that
stream, so the work of requests in different slots overlaps on the device.

Every request is computed by the same kernels on its own grid, with no data
shared between requests, so its results are bitwise the same alone and in
the mix. ``n_slots=1`` is the plain per-call form: one request at a time.

With ``batch_particles`` set, a free slot takes every request that has
arrived and waits (in arrival order, up to that many particles and the HBM
budget) as one batch: the requests' particles are concatenated into one grid
of independent particle sets (``sphx_grid_build_sets``), and one step runs
the h iteration, ghost and force of all of them, so a queue of small
requests costs the launches and readbacks of one step instead of one step
each. No leaf or task joins two sets and each set's sums are reduced on
their own, so every request's results are still bitwise those of the
request alone.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .sphx import DENS_F32, FORCE_F32, GHOST_F32


@dataclass
class Result:
    rid: int
    n: int
    arrival: float
    start: float = 0.0
    done: float = 0.0
    passes: int = 0
    interactions: int = 0
    status: int = 0
    outputs: Optional[dict] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def request_bytes(ctx, n: int) -> int:
    """Device bytes a request of n particles holds while it runs: its inputs
    (FP64 positions, FP32 fields, activity mask), a private copy of h, the
    caller-owned outputs and the library workspace."""
    inputs = n * (3 * 8 + 8 * 4 + 1) + n * 4
    outputs = n * (len(DENS_F32) * 4 + 4 + len(GHOST_F32) * 4 + 1 + len(FORCE_F32) * 4 + 4) + 256
    return inputs + outputs + ctx.workspace_bytes(n)


def _run_one(sphx, ctx, req, stream, keep, res: Result):
    """One whole request on ``stream``: (upload,) grid, tasks, h iteration,
    ghost, force and FP64 sums, then (optionally) the download. A request
    given as device arrays is not modified: its h is copied first."""
    import torch
    with torch.cuda.stream(stream):
        if isinstance(req, sphx.DeviceParticles):
            t = dict(req.t)
            t["h"] = req.t["h"].clone()
            dp = sphx.DeviceParticles(t, req.n)
        else:
            dp = sphx.DeviceParticles.from_set(req, "cuda:0")
        out = sphx.Outputs(dp.n, "cuda:0")
        grid = sphx.Grid(ctx, dp, stream)
        tasks = sphx.Tasks(ctx, grid, dp, stream)
        try:
            st, info = sphx.step(ctx, grid, tasks, dp, out, stream)
            res.status = st
            res.passes = info.passes
            # wait for the step's last kernels without the interpreter lock
            # (a tensor read would wait for them holding it, and stall the
            # other slots' launches meanwhile)
            stream.synchronize()
            res.interactions = int(out.d["nngb"].to(torch.int64).sum()
                                   + out.f["nforce"].to(torch.int64).sum())
            if keep:
                host = {k: v.cpu() for k, v in {**out.d, **out.g, **out.f}.items()}
                host["h"] = dp.t["h"].cpu()
                host["sums"] = out.sums.cpu()
            stream.synchronize()
            if keep:
                res.outputs = {k: v.numpy() for k, v in host.items()}
        finally:
            tasks.close()
            grid.close()
            del dp, out


def _run_batch(sphx, ctx, reqs, stream, keep, results: List[Result]):
    """Several requests as one batch on ``stream``: their particles
    concatenated (new arrays: the requests' own are not modified), one grid of
    independent sets, tasks, one step; each request's interaction count (and,
    optionally, its outputs) taken from its slice."""
    import torch
    with torch.cuda.stream(stream):
        parts = [r if isinstance(r, sphx.DeviceParticles)
                 else sphx.DeviceParticles.from_set(r, "cuda:0") for r in reqs]
        dp, off = sphx.DeviceParticles.concat(parts)
        out = sphx.Outputs(dp.n, "cuda:0", n_sets=len(parts))
        grid = sphx.Grid(ctx, dp, stream, sets=off)
        tasks = sphx.Tasks(ctx, grid, dp, stream)
        try:
            st, info = sphx.step(ctx, grid, tasks, dp, out, stream)
            stream.synchronize()  # (without the interpreter lock)
            per = (out.d["nngb"].to(torch.int64) + out.f["nforce"].to(torch.int64))
            csum = torch.cat([torch.zeros(1, dtype=torch.int64, device=per.device),
                              torch.cumsum(per, 0)])
            ends = torch.as_tensor(off, dtype=torch.int64, device=per.device)
            counts = (csum[ends[1:]] - csum[ends[:-1]]).cpu().tolist()
            for b, res in enumerate(results):
                res.status = st
                res.passes = info.passes
                res.interactions = int(counts[b])
                if keep:
                    a, e = off[b], off[b + 1]
                    host = {k: v[a:e].cpu() for k, v in {**out.d, **out.g, **out.f}.items()}
                    host["h"] = dp.t["h"][a:e].cpu()
                    host["sums"] = out.sums[6 * b:6 * b + 6].cpu()
                    res.outputs = {k: v.numpy() for k, v in host.items()}
            stream.synchronize()
        finally:
            tasks.close()
            grid.close()
            del dp, out


class Server:
    """Admits requests as slots and HBM budget free up; K slots run at once."""

    def __init__(self, n_slots: int = 8, budget_bytes: Optional[int] = None, params=None,
                 keep_outputs: bool = False, batch_particles: Optional[int] = None):
        import torch
        from paper_2305_13380_amd import sphx
        self.sphx = sphx
        self.n_slots = int(n_slots)
        self.keep = keep_outputs
        self.batch_particles = batch_particles  # None: one request per slot
        free, _total = torch.cuda.mem_get_info()
        self.budget = int(budget_bytes) if budget_bytes is not None else int(0.5 * free)
        self.ctxs = [sphx.Context(params, 0) for _ in range(self.n_slots)]
        self.streams = [torch.cuda.Stream() for _ in range(self.n_slots)]
        self.peak_bytes = 0     # largest admitted footprint in flight at once
        self.peak_running = 0   # largest number of requests running at once

    def close(self):
        for c in self.ctxs:
            c.close()

    def run(self, requests, get_particles: Callable[[int], object]) -> List[Result]:
        """requests: list of (rid, arrival_seconds, n), arrivals ascending.
        The particles of request k come from get_particles(k), as a ParticleSet
        (uploaded by the request itself) or as DeviceParticles already in HBM.
        Returns results in request order; times are seconds from the start."""
        if self.batch_particles:
            return self._run_batched(requests, get_particles)
        import torch
        torch.cuda.synchronize()  # device inputs written on other streams are complete
        lock = threading.Condition()
        free_slots = list(range(self.n_slots))
        used = [0]
        running = [0]
        results = [Result(rid, n, arr) for rid, arr, n in requests]
        threads = []
        t0 = time.perf_counter()

        def worker(slot, k, need):
            r = results[k]
            try:
                ps = get_particles(k)
                r.start = time.perf_counter() - t0
                _run_one(self.sphx, self.ctxs[slot], ps, self.streams[slot], self.keep, r)
            except Exception as e:  # reported, never silent
                r.error = "%s: %s" % (type(e).__name__, e)
            r.done = time.perf_counter() - t0
            with lock:
                free_slots.append(slot)
                used[0] -= need
                running[0] -= 1
                lock.notify_all()

        for k, (rid, arr, n) in enumerate(requests):
            need = request_bytes(self.ctxs[0], n)
            if need > self.budget:
                results[k].error = "request of %d particles needs %d bytes > budget %d" % (
                    n, need, self.budget)
                results[k].done = results[k].start = arr
                continue
            now = time.perf_counter() - t0
            if arr > now:
                time.sleep(arr - now)
            with lock:
                while not free_slots or used[0] + need > self.budget:
                    lock.wait()
                slot = free_slots.pop(0)
                used[0] += need
                running[0] += 1
                self.peak_bytes = max(self.peak_bytes, used[0])
                self.peak_running = max(self.peak_running, running[0])
            th = threading.Thread(target=worker, args=(slot, k, need), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        return results


    def _run_batched(self, requests, get_particles) -> List[Result]:
        """run() with batches (batch_particles set): a free slot takes the
        requests that have arrived and wait, in arrival order, while they fit
        in batch_particles particles and the HBM budget, as one step over a
        grid of independent sets; a request alone larger than batch_particles
        runs as a batch of one."""
        import torch
        torch.cuda.synchronize()
        lock = threading.Condition()
        free_slots = list(range(self.n_slots))
        used = [0]
        running = [0]
        results = [Result(rid, n, arr) for rid, arr, n in requests]
        threads = []
        t0 = time.perf_counter()
        # a batch's footprint is taken as the sum of its requests' (inputs,
        # outputs, workspace): the batch's copy of their inputs, its outputs
        # and its grid's workspace for all of them
        need_of = [request_bytes(self.ctxs[0], n) for _, _, n in requests]

        def worker(slot, ks, need):
            rs = [results[k] for k in ks]
            try:
                parts = [get_particles(k) for k in ks]
                start = time.perf_counter() - t0
                for r in rs:
                    r.start = start
                if len(ks) == 1:  # (a batch of one needs no concatenation)
                    _run_one(self.sphx, self.ctxs[slot], parts[0], self.streams[slot],
                             self.keep, rs[0])
                else:
                    _run_batch(self.sphx, self.ctxs[slot], parts, self.streams[slot], self.keep,
                               rs)
            except Exception as e:  # reported, never silent
                for r in rs:
                    r.error = "%s: %s" % (type(e).__name__, e)
            done = time.perf_counter() - t0
            for r in rs:
                r.done = done
            with lock:
                free_slots.append(slot)
                used[0] -= need
                running[0] -= len(ks)
                lock.notify_all()

        pending = []  # arrived, not started (request indices, arrival order)
        k_next = 0
        while k_next < len(requests) or pending:
            now = time.perf_counter() - t0
            while k_next < len(requests) and requests[k_next][1] <= now:
                k = k_next
                k_next += 1
                if need_of[k] > self.budget:
                    results[k].error = "request of %d particles needs %d bytes > budget %d" % (
                        requests[k][2], need_of[k], self.budget)
                    results[k].done = results[k].start = requests[k][1]
                    continue
                pending.append(k)
            if not pending:
                time.sleep(max(0.0, requests[k_next][1] - now))
                continue
            with lock:
                while not free_slots or used[0] + need_of[pending[0]] > self.budget:
                    lock.wait()
                # the batch: the waiting requests in arrival order, while they fit
                ks, parts_n, need = [], 0, 0
                while pending and len(ks) < 65536:
                    k = pending[0]
                    n = requests[k][2]
                    if ks and (parts_n + n > self.batch_particles or
                               used[0] + need + need_of[k] > self.budget):
                        break
                    ks.append(pending.pop(0))
                    parts_n += n
                    need += need_of[k]
                slot = free_slots.pop(0)
                used[0] += need
                running[0] += len(ks)
                self.peak_bytes = max(self.peak_bytes, used[0])
                self.peak_running = max(self.peak_running, running[0])
            th = threading.Thread(target=worker, args=(slot, ks, need), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        return results

def percentiles(results: List[Result]):
    lat = np.array([r.latency for r in results if r.error is None])
    if lat.size == 0:
        return {}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}
