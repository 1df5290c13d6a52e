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


class Server:
    """Admits requests as slots and HBM budget free up; K slots run at once."""

    def __init__(self, n_slots: int = 8, budget_bytes: Optional[int] = None, params=None,
                 keep_outputs: bool = False):
        import torch
        from paper_2305_13380_amd import sphx
        self.sphx = sphx
        self.n_slots = int(n_slots)
        self.keep = keep_outputs
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


def percentiles(results: List[Result]):
    lat = np.array([r.latency for r in results if r.error is None])
    if lat.size == 0:
        return {}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}
