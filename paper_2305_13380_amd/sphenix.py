"""Multi-step SPHENIX runs on the GPU (Section 3.3 with the kick-drift-kick
leapfrog of Section 2.4 and the step limiter of Section 3.4), sequencing the
library's calls; every operation on particle data runs in its kernels.

One global step (the smallest limited CFL step of the particles) and every
particle active. With the GDF flavour (Appendix A) the switch follows that
flavour's shock detector, held between steps, and the conduction parameter
is the one its step forms. Per step: half kick; drift, with v and u predicted to the
end of the drift by the previous derivatives; a new grid and task list, the
h iteration, ghost and force pass (sphx_step) with the viscosity and
conduction parameters of the step before; the viscosity switch; the gradient
loop; the conduction parameter; the second half kick; the next step size.
"""
from dataclasses import dataclass, field
from typing import Callable, List, Optional


@dataclass
class RunState:
    t: float = 0.0
    steps: int = 0
    hist: List[tuple] = field(default_factory=list)  # (t, dt, passes, rebuilds)


class SphenixRun:
    """State of a run on device: the particles (positions FP64, the rest
    FP32, as the library takes them) and the last step's outputs."""

    def __init__(self, ps, params=None, device="cuda:0", c_cfl=0.1, delta=4.0,
                 dt_max: Optional[float] = None):
        import torch
        from paper_2305_13380_amd import sphx
        self.sphx = sphx
        # a new grid of the same set every step: its builds reuse the last
        # grid's buffers instead of allocating, and no step is captured (a
        # captured step replays only on the grid it was recorded for)
        p = sphx.default_params() if params is None else type(params).from_buffer_copy(params)
        p.recycle_workspace = 1
        p.graph_passes = 0
        self.ctx = sphx.Context(p, 0)
        self.dp = sphx.DeviceParticles.from_set(ps, device)
        self.out = sphx.Outputs(ps.n, device)
        self.n = ps.n
        self.c_cfl, self.delta, self.dt_max = float(c_cfl), float(delta), dt_max
        f = lambda: torch.empty(ps.n, dtype=torch.float32, device=device)
        self.v_pred = (f(), f(), f())
        self.u_pred = f()
        self.state = RunState()
        self.grid = self.tasks = None
        # the GDF flavour (Appendix A): its switch follows its shock detector
        # D (held between steps) and its conduction parameter is formed
        # inside the step
        self.gdf = p.flavour == sphx.FLAVOURS["gdf"]
        self._evaluate()
        self.D = self._detector() if self.gdf else None
        self.dt = self._next_dt()

    # the particle set the library reads: positions and the predicted v, u
    def _view(self, v, u):
        t = dict(self.dp.t)
        t["vx"], t["vy"], t["vz"] = v
        t["u"] = u
        return self.sphx.DeviceParticles(t, self.n)

    def _evaluate(self, v=None, u=None):
        sphx = self.sphx
        parts = self.dp if v is None else self._view(v, u)
        if self.tasks is not None:
            self.tasks.close()
            self.grid.close()
        self.grid = sphx.Grid(self.ctx, parts)
        self.tasks = sphx.Tasks(self.ctx, self.grid, parts)
        st, info = sphx.step(self.ctx, self.grid, self.tasks, parts, self.out)
        self.parts = parts
        self.info = info
        return st, info

    def _detector(self):
        _, _, D = self.sphx.gdf(self.ctx, self.grid, self.tasks, self.parts, self.out.d["rho"],
                                detector=True)
        return D

    def _next_dt(self):
        dt, mn = self.sphx.timestep(self.ctx, self.grid, self.tasks, self.parts,
                                    self.out.f["v_sig"], self.c_cfl, self.delta)
        d = float(mn.item())
        return min(d, self.dt_max) if self.dt_max is not None else d

    def step(self):
        sphx, t, o = self.sphx, self.dp.t, self.out
        dt = self.dt
        v = (t["vx"], t["vy"], t["vz"])
        a = (o.f["ax"], o.f["ay"], o.f["az"])
        sphx.kick(self.ctx, v, t["u"], a, o.f["du_dt"], 0.5 * dt)
        sphx.drift(self.ctx, self.dp, dt)
        sphx.kick(self.ctx, v, t["u"], a, o.f["du_dt"], 0.5 * dt, v_out=self.v_pred,
                  u_out=self.u_pred)
        div_old = o.g["div_v"].clone()
        st, info = self._evaluate(self.v_pred, self.u_pred)
        if st < 0:
            raise RuntimeError("step failed")
        if self.gdf:
            D = self._detector()
            sphx.gdf_alpha_v_update(self.ctx, t["alpha_v"], self.D, D, o.g["c"], t["h"],
                                    o.f["v_sig"], o.g["balsara"], dt)
            self.D = D
        else:
            sphx.alpha_v_update(self.ctx, t["alpha_v"], div_old, o.g["div_v"], o.g["c"],
                                t["h"], o.f["v_sig"], dt)
            lap, vc, avmax = sphx.gradient(self.ctx, self.grid, self.tasks, self.parts, o)
            sphx.alpha_c_update(self.ctx, t["alpha_c"], lap, self.u_pred, t["h"], vc, avmax,
                                dt)
        sphx.kick(self.ctx, v, t["u"], a, o.f["du_dt"], 0.5 * dt)
        self.state.t += dt
        self.state.steps += 1
        self.state.hist.append((self.state.t, dt, info.passes, info.task_rebuilds))
        self.dt = self._next_dt()
        return self.state

    def run(self, n_steps, callback: Optional[Callable] = None):
        for k in range(n_steps):
            self.step()
            if callback is not None:
                callback(k, self)
        return self.state

    def close(self):
        if self.tasks is not None:
            self.tasks.close()
            self.grid.close()
            self.tasks = self.grid = None
        self.ctx.close()


def _main():
    """A SPHENIX run of the 64^3 Sedov box (one unit of energy in the central
    particles): python -m paper_2305_13380_amd.sphenix [--steps N]
    [--flavour energy|gdf]."""
    import argparse
    import sys
    import time
    import torch
    from paper_2305_13380_amd import inputs
    ap = argparse.ArgumentParser(description=_main.__doc__.split("\n")[0])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--flavour", default="energy", choices=["energy", "gdf"])
    a = ap.parse_args()
    from paper_2305_13380_amd import sphx
    ps = inputs.config_sedov(2)
    ps.alpha_v[:] = 0.1
    ps.alpha_c[:] = 0.0
    run = SphenixRun(ps, sphx.default_params(flavour=a.flavour), c_cfl=0.1)
    for _ in range(a.warmup):
        run.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.run(a.steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / max(a.steps, 1) * 1e3
    print("sphenix (%s): %d steps, %.3f ms per step, t = %.4g" % (a.flavour, a.steps, ms,
                                                                 run.state.t),
          file=sys.stderr, flush=True)
    run.close()


if __name__ == "__main__":
    _main()
