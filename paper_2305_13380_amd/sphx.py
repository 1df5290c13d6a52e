"""ctypes binding of libsphx.so (the C-ABI declared in include/sphx.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels. PyTorch provides device memory (tensors) and streams. Importing
this module loads the library and raises if it has not been built: there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphx.so")

OK = 0
E_INVALID, E_OOM, E_HIP, E_STATE = -1, -2, -3, -4
W_NOT_CONVERGED, W_H_CLAMPED, W_REBUILD = 1, 2, 4
COUNTERS = 4


class SphxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("sphx status %d: %s" % (status, msg))
        self.status = status


class Params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("periodic", C.c_int32), ("max_iter", C.c_int32),
                ("gamma_k", C.c_double), ("eta", C.c_double), ("h_tol", C.c_double),
                ("h_max", C.c_double), ("gamma_gas", C.c_double), ("beta_v", C.c_double),
                ("eps_balsara", C.c_double), ("skin", C.c_double), ("leaf_max", C.c_int32),
                ("neighbour_lists", C.c_int32), ("density_tile", C.c_int32),
                ("density_waves", C.c_int32), ("force_tile", C.c_int32),
                ("force_waves", C.c_int32), ("graph_passes", C.c_int32),
                ("density_balance", C.c_int32), ("kernel", C.c_int32), ("flavour", C.c_int32),
                ("recycle_workspace", C.c_int32)]


# Smoothing kernels (SPHX_KERNEL_* of sphx.h), by name.
KERNELS = {"wendland_c2": 0, "wendland_c4": 1, "wendland_c6": 2, "cubic_spline": 3,
           "quartic_spline": 4, "quintic_spline": 5}


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in (
        "x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "alpha_v", "alpha_c", "active")]


class DensityOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in (
        "rho", "rho_dh", "n", "n_dh", "div_sum", "curl_x", "curl_y", "curl_z", "nngb",
        "P_hat", "P_hat_dh")]


class GhostOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in (
        "f", "P", "c", "balsara", "A", "div_v", "curl_v", "converged")]


class ForceOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ax", "ay", "az", "du_dt", "v_sig", "nforce")]


class StepInfo(C.Structure):
    _fields_ = [("passes", C.c_int32), ("task_rebuilds", C.c_int32), ("unconverged", C.c_int32),
                ("clamped", C.c_int32), ("n_leaves", C.c_int64), ("n_tasks", C.c_int64),
                ("list_builds", C.c_int32), ("list_fallback", C.c_int32),
                ("list_entries", C.c_int64), ("pairs_cellpair", C.c_int64),
                ("pairs_list", C.c_int64), ("captured_passes", C.c_int32),
                ("task_relayouts", C.c_int32)]


SYMBOLS = ("sphx_params_default", "sphx_ctx_create", "sphx_ctx_destroy", "sphx_workspace_bytes",
           "sphx_grid_build", "sphx_grid_destroy", "sphx_tasks_build", "sphx_tasks_destroy",
           "sphx_iter_reset", "sphx_density", "sphx_ghost", "sphx_force", "sphx_step",
           "sphx_grid_leaves", "sphx_tasks_count", "sphx_last_error", "sphx_profile_enable",
           "sphx_profile_read", "sphx_autotune", "sphx_params_set_kernel", "sphx_fof",
           "sphx_gravity", "sphx_alpha_v_update", "sphx_force_noalloc", "sphx_gradient",
           "sphx_alpha_c_update", "sphx_timestep", "sphx_kick", "sphx_drift",
           "sphx_probe_read", "sphx_grid_build_sets", "sphx_gdf", "sphx_gdf_alpha_v_update")

_LIB = None


def _load():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsphx.so is not built (%s); run python paper_2305_13380_amd/build.py"
                          % LIB_PATH)
    # torch ships its own HIP runtime under the same soname. Loading torch
    # first makes the loader bind the library to that runtime, so the streams
    # and memory torch hands over belong to the runtime the library calls;
    # loaded the other way round the process would hold two HIP runtimes.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    P = C.POINTER
    L.sphx_params_default.argtypes = [P(Params)]
    L.sphx_params_set_kernel.argtypes = [P(Params), i32]
    L.sphx_params_set_kernel.restype = i32
    L.sphx_fof.argtypes = [vp, P(Particles), C.c_double, vp, vp, vp, vp]
    L.sphx_fof.restype = i32
    L.sphx_gravity.argtypes = [vp, P(Particles)] + [C.c_double] * 4 + [vp] * 6
    L.sphx_gravity.restype = i32
    L.sphx_alpha_v_update.argtypes = [vp, i64] + [vp] * 5 + [C.c_double, vp, vp]
    L.sphx_alpha_v_update.restype = i32
    L.sphx_params_default.restype = None
    L.sphx_ctx_create.argtypes = [P(Params), C.c_int, P(vp)]
    L.sphx_ctx_destroy.argtypes = [vp]
    L.sphx_ctx_destroy.restype = None
    L.sphx_workspace_bytes.argtypes = [P(Params), i64]
    L.sphx_workspace_bytes.restype = C.c_size_t
    L.sphx_grid_build.argtypes = [vp, P(Particles), vp, P(vp)]
    L.sphx_grid_build_sets.argtypes = [vp, P(Particles), P(C.c_int64), i32, vp, P(vp)]
    L.sphx_grid_destroy.argtypes = [vp]
    L.sphx_grid_destroy.restype = None
    L.sphx_tasks_build.argtypes = [vp, vp, P(Particles), vp, P(vp)]
    L.sphx_tasks_destroy.argtypes = [vp]
    L.sphx_tasks_destroy.restype = None
    L.sphx_iter_reset.argtypes = [vp, vp, P(Particles), vp]
    L.sphx_density.argtypes = [vp, vp, vp, P(Particles), P(DensityOut), vp, vp]
    L.sphx_ghost.argtypes = [vp, vp, vp, P(Particles), P(DensityOut), P(GhostOut), vp, i32, vp]
    L.sphx_force.argtypes = [vp, vp, vp, P(Particles), P(DensityOut), P(GhostOut), P(ForceOut),
                             vp, vp]
    L.sphx_force_noalloc.argtypes = L.sphx_force.argtypes
    L.sphx_gradient.argtypes = [vp, vp, vp, P(Particles), vp, vp, vp, vp, vp, vp]
    L.sphx_gdf.argtypes = [vp, vp, vp, P(Particles), vp, vp, vp, vp, vp]
    L.sphx_gdf_alpha_v_update.argtypes = [vp, i64] + [vp] * 7 + [C.c_double, vp, vp]
    L.sphx_probe_read.argtypes = [vp, P(C.c_uint64), i32]
    L.sphx_probe_read.restype = i32
    L.sphx_alpha_c_update.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, C.c_double, vp, vp]
    L.sphx_timestep.argtypes = [vp, vp, vp, P(Particles), vp, C.c_double, C.c_double, vp, vp,
                                vp]
    L.sphx_kick.argtypes = [vp, i64] + [vp] * 9 + [C.c_double] + [vp] * 5
    L.sphx_drift.argtypes = [vp, i64] + [vp] * 6 + [C.c_double, vp]
    L.sphx_step.argtypes = [vp, vp, P(vp), P(Particles), P(DensityOut), P(GhostOut),
                            P(ForceOut), vp, vp, P(StepInfo)]
    L.sphx_autotune.argtypes = [vp, vp, vp, P(Particles), P(DensityOut), P(GhostOut),
                                P(ForceOut), i32, P(Params), vp]
    L.sphx_autotune.restype = i32
    L.sphx_grid_leaves.argtypes = [vp]
    L.sphx_grid_leaves.restype = i64
    L.sphx_tasks_count.argtypes = [vp]
    L.sphx_tasks_count.restype = i64
    L.sphx_profile_enable.argtypes = [vp, i32]
    L.sphx_profile_enable.restype = i32
    L.sphx_profile_read.argtypes = [vp, i32, P(C.c_double), P(i64)]
    L.sphx_profile_read.restype = i32
    L.sphx_last_error.argtypes = []
    L.sphx_last_error.restype = C.c_char_p
    for name in ("sphx_ctx_create", "sphx_grid_build", "sphx_grid_build_sets",
                 "sphx_tasks_build", "sphx_iter_reset",
                 "sphx_density", "sphx_ghost", "sphx_force", "sphx_step", "sphx_force_noalloc",
                 "sphx_gradient", "sphx_alpha_c_update", "sphx_timestep", "sphx_kick",
                 "sphx_drift", "sphx_gdf", "sphx_gdf_alpha_v_update"):
        getattr(L, name).restype = i32
    _LIB = L
    return L


lib = _load()


def last_error() -> str:
    return lib.sphx_last_error().decode()


def _check(status):
    if status < 0:
        raise SphxError(status, last_error())
    return status


FLAVOURS = {"energy": 0, "entropy": 1, "phantom": 2,  # SPHX_FLAVOUR_*
            "pressure_energy": 3, "anarchy_pu": 4, "gdf": 5}


def default_params(**kw) -> Params:
    """The library's defaults with fields overridden by keyword; kernel= takes
    a name of KERNELS (or its number) and sets the kernel's gamma_k too;
    flavour= takes a name of FLAVOURS (or the number)."""
    p = Params()
    lib.sphx_params_default(C.byref(p))
    if isinstance(kw.get("flavour"), str):
        kw = dict(kw, flavour=FLAVOURS[kw["flavour"]])
    if "kernel" in kw:
        k = kw["kernel"]
        k = KERNELS[k] if isinstance(k, str) else int(k)
        _check(lib.sphx_params_set_kernel(C.byref(p), k))
    for k, v in kw.items():
        if k == "kernel":
            continue
        if k == "box":
            p.box = (C.c_double * 3)(*v)
        else:
            setattr(p, k, v)
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    handle = None

    def __init__(self, params: Optional[Params] = None, device: int = 0):
        self.params = params if params is not None else default_params()
        self.device = device
        h = C.c_void_p()
        _check(lib.sphx_ctx_create(C.byref(self.params), device, C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle and lib is not None:  # lib is None at interpreter shutdown
            lib.sphx_ctx_destroy(self.handle)
        self.handle = None

    __del__ = close

    def profile(self, enable: bool):
        _check(lib.sphx_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self, kernel: int):
        """(total milliseconds, launches) of kernel 0 (density) or 1 (force)."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib.sphx_profile_read(self.handle, kernel, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def workspace_bytes(self, n: int) -> int:
        return int(lib.sphx_workspace_bytes(C.byref(self.params), int(n)))


@dataclass
class DeviceParticles:
    """Device-resident particle arrays (torch tensors) and their C view."""
    t: dict
    n: int

    @classmethod
    def from_set(cls, ps, device="cuda"):
        import torch
        t = {}
        for k in ("x", "y", "z"):
            t[k] = torch.from_numpy(np.ascontiguousarray(getattr(ps, k), np.float64)).to(device)
        for k in ("vx", "vy", "vz", "m", "u", "h", "alpha_v", "alpha_c"):
            t[k] = torch.from_numpy(np.ascontiguousarray(getattr(ps, k), np.float32)).to(device)
        t["active"] = None if ps.active is None else torch.from_numpy(
            np.ascontiguousarray(ps.active, np.uint8)).to(device)
        return cls(t, ps.n)

    @classmethod
    def concat(cls, parts):
        """The particle sets `parts` one after another in new arrays (a batch
        for sphx_grid_build_sets) and their n_sets + 1 offsets. The activity
        mask is kept if any set has one (the others count as all active)."""
        import torch
        t = {}
        for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "alpha_v", "alpha_c"):
            t[k] = torch.cat([p.t[k] for p in parts])
        if any(p.t["active"] is not None for p in parts):
            t["active"] = torch.cat([
                p.t["active"] if p.t["active"] is not None else
                torch.ones((p.n,), dtype=torch.uint8, device=p.t["x"].device) for p in parts])
        else:
            t["active"] = None
        off = [0]
        for p in parts:
            off.append(off[-1] + p.n)
        return cls(t, off[-1]), off

    def view(self) -> Particles:
        p = Particles()
        p.n = self.n
        for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "alpha_v", "alpha_c", "active"):
            setattr(p, k, _ptr(self.t[k]))
        return p


DENS_F32 = ("rho", "rho_dh", "n", "n_dh", "div_sum", "curl_x", "curl_y", "curl_z")
DENS_PE = ("P_hat", "P_hat_dh")  # the pressure-energy flavour's extra outputs
GHOST_F32 = ("f", "P", "c", "balsara", "A", "div_v", "curl_v")
FORCE_F32 = ("ax", "ay", "az", "du_dt", "v_sig")


class Outputs:
    """Caller-owned output arrays for the density, ghost and force passes
    (pressure=True: also the smoothed pressure and its h-derivative)."""

    def __init__(self, n, device="cuda", pressure=False, n_sets=1):
        import torch
        f = lambda: torch.full((n,), float("nan"), dtype=torch.float32, device=device)
        self.d = {k: f() for k in DENS_F32 + (DENS_PE if pressure else ())}
        self.d["nngb"] = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.g = {k: f() for k in GHOST_F32}
        self.g["converged"] = torch.zeros((n,), dtype=torch.uint8, device=device)
        self.f = {k: f() for k in FORCE_F32}
        self.f["nforce"] = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.counters = torch.zeros((COUNTERS,), dtype=torch.int32, device=device)
        # six FP64 conservation sums per particle set (sphx_grid_build_sets)
        self.sums = torch.zeros((6 * n_sets,), dtype=torch.float64, device=device)

    def dens_view(self):
        o = DensityOut()
        for k in DENS_F32 + ("nngb",) + DENS_PE:
            setattr(o, k, _ptr(self.d.get(k)))
        return o

    def ghost_view(self):
        o = GhostOut()
        for k in GHOST_F32 + ("converged",):
            setattr(o, k, _ptr(self.g[k]))
        return o

    def force_view(self):
        o = ForceOut()
        for k in FORCE_F32 + ("nforce",):
            setattr(o, k, _ptr(self.f[k]))
        return o


class Grid:
    handle = None

    def __init__(self, ctx: Context, parts: DeviceParticles, stream=None, sets=None):
        """sets: None (one particle set), or the n_sets + 1 offsets of the
        independent sets held in `parts` (sphx_grid_build_sets)."""
        self.ctx = ctx
        self.pv = parts.view()
        h = C.c_void_p()
        if sets is None:
            self.n_sets = 1
            _check(lib.sphx_grid_build(ctx.handle, C.byref(self.pv), _stream(stream),
                                       C.byref(h)))
        else:
            off = (C.c_int64 * len(sets))(*[int(v) for v in sets])
            self.n_sets = len(sets) - 1
            _check(lib.sphx_grid_build_sets(ctx.handle, C.byref(self.pv), off, self.n_sets,
                                            _stream(stream), C.byref(h)))
        self.handle = h

    @property
    def n_leaves(self):
        return int(lib.sphx_grid_leaves(self.handle))

    def close(self):
        if self.handle and lib is not None:  # lib is None at interpreter shutdown
            lib.sphx_grid_destroy(self.handle)
        self.handle = None

    __del__ = close


class Tasks:
    handle = None

    def __init__(self, ctx: Context, grid: Grid, parts: DeviceParticles, stream=None):
        self.ctx = ctx
        self.grid = grid
        self.handle = C.c_void_p()
        self.build(parts, stream)

    def build(self, parts: DeviceParticles, stream=None):
        pv = parts.view()
        _check(lib.sphx_tasks_build(self.ctx.handle, self.grid.handle, C.byref(pv),
                                    _stream(stream), C.byref(self.handle)))

    @property
    def count(self):
        return int(lib.sphx_tasks_count(self.handle))

    def close(self):
        if self.handle and lib is not None:  # lib is None at interpreter shutdown
            lib.sphx_tasks_destroy(self.handle)
        self.handle = None

    __del__ = close


def iter_reset(ctx, grid, parts, stream=None):
    pv = parts.view()
    return _check(lib.sphx_iter_reset(ctx.handle, grid.handle, C.byref(pv), _stream(stream)))


def density(ctx, grid, tasks, parts, out: Outputs, counters=True, stream=None):
    pv = parts.view()
    dv = out.dens_view()
    return _check(lib.sphx_density(ctx.handle, grid.handle, tasks.handle, C.byref(pv),
                                   C.byref(dv), _ptr(out.counters) if counters else None,
                                   _stream(stream)))


def ghost(ctx, grid, tasks, parts, out: Outputs, final_pass=False, counters=True, stream=None):
    pv = parts.view()
    dv, gv = out.dens_view(), out.ghost_view()
    return _check(lib.sphx_ghost(ctx.handle, grid.handle, tasks.handle, C.byref(pv), C.byref(dv),
                                 C.byref(gv), _ptr(out.counters) if counters else None,
                                 1 if final_pass else 0, _stream(stream)))


def force(ctx, grid, tasks, parts, out: Outputs, sums=True, stream=None):
    pv = parts.view()
    dv, gv, fv = out.dens_view(), out.ghost_view(), out.force_view()
    return _check(lib.sphx_force(ctx.handle, grid.handle, tasks.handle, C.byref(pv), C.byref(dv),
                                 C.byref(gv), C.byref(fv), _ptr(out.sums) if sums else None,
                                 _stream(stream)))


def force_noalloc(ctx, grid, tasks, parts, out: Outputs, sums=True, stream=None):
    """sphx_force_noalloc: the force pass with its partial sums in the
    library's fixed device workspace (no allocation)."""
    pv = parts.view()
    dv, gv, fv = out.dens_view(), out.ghost_view(), out.force_view()
    return _check(lib.sphx_force_noalloc(ctx.handle, grid.handle, tasks.handle, C.byref(pv),
                                         C.byref(dv), C.byref(gv), C.byref(fv),
                                         _ptr(out.sums) if sums else None, _stream(stream)))


def step(ctx, grid, tasks: Tasks, parts, out: Outputs, stream=None):
    pv = parts.view()
    dv, gv, fv = out.dens_view(), out.ghost_view(), out.force_view()
    info = StepInfo()
    st = _check(lib.sphx_step(ctx.handle, grid.handle, C.byref(tasks.handle), C.byref(pv),
                              C.byref(dv), C.byref(gv), C.byref(fv), _ptr(out.sums),
                              _stream(stream), C.byref(info)))
    return st, info


def fixed_h_pass(ctx, grid, tasks, parts, out: Outputs, stream=None):
    """Density at the current h, ghost finalisation without changing h (one
    final pass), force: the three loops at a fixed h."""
    iter_reset(ctx, grid, parts, stream)
    out.counters.zero_()
    density(ctx, grid, tasks, parts, out, stream=stream)
    ghost(ctx, grid, tasks, parts, out, final_pass=True, stream=stream)
    force(ctx, grid, tasks, parts, out, stream=stream)


def fof(ctx, parts, b, sizes=True, stream=None):
    """Friends-of-friends groups at linking length b (sphx_fof): returns
    (group, group_size or None, counts) as device tensors: group[i] is the
    smallest index of i's group, counts = [groups, linked pairs] (int64)."""
    import torch
    dev = parts.t["x"].device
    group = torch.empty(parts.n, dtype=torch.int32, device=dev)
    gsize = torch.empty(parts.n, dtype=torch.int32, device=dev) if sizes else None
    counts = torch.empty(2, dtype=torch.int64, device=dev)
    pv = parts.view()
    _check(lib.sphx_fof(ctx.handle, C.byref(pv), float(b), _ptr(group), _ptr(gsize),
                        _ptr(counts), _stream(stream)))
    return group, gsize, counts


def gravity(ctx, parts, G, H, r_s, r_p2p, potential=True, pairs=None, stream=None):
    """Short-range softened gravity by direct summation (sphx_gravity):
    returns device tensors (ax, ay, az, pot or None); `pairs`, a device int64
    tensor of one element, receives the number of pairs summed."""
    import torch
    dev = parts.t["x"].device
    a = [torch.empty(parts.n, dtype=torch.float32, device=dev) for _ in range(3)]
    pot = torch.empty(parts.n, dtype=torch.float32, device=dev) if potential else None
    pv = parts.view()
    _check(lib.sphx_gravity(ctx.handle, C.byref(pv), float(G), float(H), float(r_s),
                            float(r_p2p), _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(pot),
                            _ptr(pairs), _stream(stream)))
    return a[0], a[1], a[2], pot


def alpha_v_update(ctx, alpha_v, div_old, div_new, c, h, v_sig, dt, stream=None):
    """SPHENIX viscosity switch (sphx_alpha_v_update): updates the FP32
    device tensor alpha_v in place."""
    _check(lib.sphx_alpha_v_update(ctx.handle, int(alpha_v.numel()), _ptr(div_old),
                                   _ptr(div_new), _ptr(c), _ptr(h), _ptr(v_sig), float(dt),
                                   _ptr(alpha_v), _stream(stream)))
    return alpha_v


def probe_read(ctx, clear=True):
    """Neighbour-loop counters of a measurement build (sphx_probe_read):
    (probe build?, [lane slots, receiver-lane tests, accepted pairs,
    compute-loop lane slots, entries they evaluated])."""
    v = (C.c_uint64 * 5)()
    st = _check(lib.sphx_probe_read(ctx.handle, v, 1 if clear else 0))
    return st == 0, [int(x) for x in v]


def gradient(ctx, grid, tasks, parts, out: Outputs, stream=None):
    """SPHENIX gradient loop (sphx_gradient) after a step: returns device
    tensors (lap_u, v_c, alpha_v_max); entries of inactive particles are
    left as allocated (NaN)."""
    import torch
    dev = parts.t["x"].device
    res = [torch.full((parts.n,), float("nan"), dtype=torch.float32, device=dev)
           for _ in range(3)]
    pv = parts.view()
    _check(lib.sphx_gradient(ctx.handle, grid.handle, tasks.handle, C.byref(pv),
                             _ptr(out.d["rho"]), _ptr(out.g["P"]), _ptr(res[0]), _ptr(res[1]),
                             _ptr(res[2]), _stream(stream)))
    return tuple(res)


def gdf(ctx, grid, tasks, parts, rho, f=None, alpha_c=None, stream=None, detector=False):
    """The GDF flavour's correction f and conduction parameter alpha_c
    (sphx_gdf) from the particles' h and the device tensor rho: returns
    device tensors (f, alpha_c), and the shock detector D as a third with
    detector=True, written for the active particles (given tensors are
    filled in place; new ones start as NaN)."""
    import torch
    dev = parts.t["x"].device
    if f is None:
        f = torch.full((parts.n,), float("nan"), dtype=torch.float32, device=dev)
    if alpha_c is None:
        alpha_c = torch.full((parts.n,), float("nan"), dtype=torch.float32, device=dev)
    D = (torch.full((parts.n,), float("nan"), dtype=torch.float32, device=dev)
         if detector else None)
    pv = parts.view()
    _check(lib.sphx_gdf(ctx.handle, grid.handle, tasks.handle, C.byref(pv), _ptr(rho),
                        _ptr(f), _ptr(alpha_c), _ptr(D), _stream(stream)))
    return (f, alpha_c, D) if detector else (f, alpha_c)


def gdf_alpha_v_update(ctx, alpha_v, D_old, D_new, c, h, v_sig, balsara, dt, active=None,
                       stream=None):
    """The GDF viscosity switch over a step dt (sphx_gdf_alpha_v_update):
    updates the FP32 device tensor alpha_v in place."""
    _check(lib.sphx_gdf_alpha_v_update(ctx.handle, int(alpha_v.numel()), _ptr(D_old),
                                       _ptr(D_new), _ptr(c), _ptr(h), _ptr(v_sig),
                                       _ptr(balsara), _ptr(active), float(dt), _ptr(alpha_v),
                                       _stream(stream)))
    return alpha_v


def alpha_c_update(ctx, alpha_c, lap_u, u, h, v_c, alpha_v_max, dt, active=None, stream=None):
    """SPHENIX conduction parameter over a step dt (sphx_alpha_c_update):
    updates the FP32 device tensor alpha_c in place."""
    _check(lib.sphx_alpha_c_update(ctx.handle, int(alpha_c.numel()), _ptr(lap_u), _ptr(u),
                                   _ptr(h), _ptr(v_c), _ptr(alpha_v_max), _ptr(active),
                                   float(dt), _ptr(alpha_c), _stream(stream)))
    return alpha_c


def timestep(ctx, grid, tasks, parts, v_sig, c_cfl, delta=4.0, stream=None):
    """Step sizes (sphx_timestep): returns device tensors (dt of every active
    particle, the smallest of them as one FP32 element)."""
    import torch
    dev = parts.t["x"].device
    dt = torch.full((parts.n,), float("nan"), dtype=torch.float32, device=dev)
    mn = torch.empty(1, dtype=torch.float32, device=dev)
    pv = parts.view()
    _check(lib.sphx_timestep(ctx.handle, grid.handle, tasks.handle, C.byref(pv), _ptr(v_sig),
                             float(c_cfl), float(delta), _ptr(dt), _ptr(mn), _stream(stream)))
    return dt, mn


def kick(ctx, v, u, a, du, dt_half, v_out=None, u_out=None, active=None, stream=None):
    """Half kick (sphx_kick): v, a are sequences of three FP32 device
    tensors; in place unless v_out/u_out are given."""
    v_out = v if v_out is None else v_out
    u_out = u if u_out is None else u_out
    _check(lib.sphx_kick(ctx.handle, int(u.numel()), _ptr(v[0]), _ptr(v[1]), _ptr(v[2]), _ptr(u),
                         _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(du), _ptr(active),
                         float(dt_half), _ptr(v_out[0]), _ptr(v_out[1]), _ptr(v_out[2]),
                         _ptr(u_out), _stream(stream)))
    return v_out, u_out


def drift(ctx, parts, dt, stream=None):
    """Drift (sphx_drift) of the particles' FP64 positions, in place."""
    t = parts.t
    _check(lib.sphx_drift(ctx.handle, parts.n, _ptr(t["x"]), _ptr(t["y"]), _ptr(t["z"]),
                          _ptr(t["vx"]), _ptr(t["vy"]), _ptr(t["vz"]), float(dt),
                          _stream(stream)))


def autotune(ctx, grid, tasks, parts, out: Outputs, reps=3, stream=None) -> Params:
    """Loop shapes timed on this grid (sphx_autotune); returns the tuned
    parameters (create contexts from them to use the shapes)."""
    pv, dv, gv, fv = parts.view(), out.dens_view(), out.ghost_view(), out.force_view()
    tuned = Params()
    _check(lib.sphx_autotune(ctx.handle, grid.handle, tasks.handle, C.byref(pv), C.byref(dv),
                             C.byref(gv), C.byref(fv), int(reps), C.byref(tuned),
                             _stream(stream)))
    return tuned
