"""The oracle: a plain FP64 CPU reference for the SPH neighbour loops.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package. It never imports the library
package and the library never imports it; the seeded input generators are the
only code both use, and they hold none of the method's arithmetic.

The arithmetic lives in ``sph_oracle.c`` (one plain loop per definition of the
paper's Section 3). This module marshals arrays, drives the per-particle
Newton-Raphson iteration on the smoothing length, and produces neighbour
candidate lists:

* ``mode="brute"`` -- every receiver is tested against every particle.
* ``mode="tree"``  -- a scipy k-d tree supplies an ascending superset of the
  neighbours (radius padded by 1e-9 relative); the C code applies the same
  exact membership test as in brute mode, so both modes are bit-identical.

Parity note: every function here is pinned by the tests in
``tests/test_oracle_*.py`` against closed forms, invariants and brute force.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import build as _build

_LIB = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _nullable(p):
    """ctypes argtype that accepts None or a contiguous array."""
    class _N:
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return p.from_param(obj)
    return _N


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.or_wc2_array.argtypes = [C.c_int64, _dp, _dp, C.c_double, _dp, _dp, _dp]
        L.or_wc2_array.restype = None
        L.or_kernel_array.argtypes = [C.c_int, C.c_int64, _dp, _dp, C.c_double, _dp, _dp, _dp]
        L.or_kernel_array.restype = None
        L.or_density.argtypes = ([C.c_int64] + [_dp] * 8 + [_dp, C.c_int, C.c_double, C.c_int,
                                 C.c_int64,
                                 _nullable(_ip), _nullable(_ip), _nullable(_ip)] + [_dp] * 8 + [_ip])
        L.or_density.restype = C.c_int64
        L.or_h_update.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                  _dp, _dp, _dp, _i32p]
        L.or_h_update.restype = None
        L.or_ghost.argtypes = ([C.c_int64] + [_dp] * 8 + [C.c_double, C.c_double] + [_dp] * 7
                               + [C.c_int] + [_nullable(_dp)] * 4)
        L.or_ghost.restype = None
        L.or_force.argtypes = ([C.c_int64] + [_dp] * 16 + [_dp, C.c_int, C.c_double, C.c_int,
                               C.c_double,
                               C.c_int64, _nullable(_ip), _nullable(_ip), _nullable(_ip)]
                               + [_dp] * 5 + [_ip, C.c_int, C.c_double, _nullable(_dp),
                                              _nullable(_dp)])
        L.or_force.restype = C.c_int64
        L.or_pressure.argtypes = ([C.c_int64] + [_dp] * 7 + [C.c_int, C.c_double, C.c_int,
                                  C.c_double, C.c_int64, _nullable(_ip), _nullable(_ip),
                                  _nullable(_ip), _dp, _dp])
        L.or_pressure.restype = None
        L.or_sums.argtypes = [C.c_int64] + [_dp] * 8 + [_dp]
        L.or_sums.restype = None
        L.or_fof.argtypes = ([C.c_int64] + [_dp] * 4 + [C.c_int, C.c_double, _nullable(_ip),
                             _nullable(_ip), _ip])
        L.or_fof.restype = C.c_int64
        L.or_grav_pair_array.argtypes = [C.c_int64, _dp, C.c_double, C.c_double, _dp, _dp]
        L.or_grav_pair_array.restype = None
        L.or_gravity.argtypes = ([C.c_int64] + [_dp] * 5 + [C.c_int] + [C.c_double] * 4
                                 + [C.c_int64, _nullable(_ip), _nullable(_ip), _nullable(_ip)]
                                 + [_dp] * 5)
        L.or_gravity.restype = C.c_int64
        L.or_alpha_v_update.argtypes = ([C.c_int64] + [_dp] * 5 + [C.c_double] * 4 + [_dp])
        L.or_alpha_v_update.restype = None
        L.or_gradient.argtypes = ([C.c_int64] + [_dp] * 12 + [_dp, C.c_int, C.c_double, C.c_int,
                                  C.c_int64, _nullable(_ip), _nullable(_ip), _nullable(_ip)]
                                  + [_dp] * 3 + [_nullable(_dp)])
        L.or_gradient.restype = C.c_int64
        L.or_gdf.argtypes = ([C.c_int64] + [_dp] * 10 + [C.c_int, C.c_double, C.c_int,
                             C.c_double, C.c_int64, _nullable(_ip), _nullable(_ip),
                             _nullable(_ip), _dp, _dp])
        L.or_gdf_detector.argtypes = ([C.c_int64] + [_dp] * 10 + [C.c_int, C.c_double,
                                      C.c_int, C.c_double, C.c_int64, _nullable(_ip),
                                      _nullable(_ip), _nullable(_ip), _dp])
        L.or_gdf_detector.restype = None
        L.or_gdf_alpha_v_update.argtypes = [C.c_int64] + [_dp] * 6 + [C.c_double,
                                                                      C.c_double, _dp]
        L.or_gdf_alpha_v_update.restype = None
        L.or_gdf.restype = None
        L.or_alpha_c_update.argtypes = ([C.c_int64] + [_dp] * 5 + [C.c_double] * 6 + [_dp])
        L.or_alpha_c_update.restype = None
        L.or_dt_cfl.argtypes = [C.c_int64, _dp, _dp, C.c_double, C.c_double, _dp]
        L.or_dt_cfl.restype = None
        L.or_dt_limit.argtypes = ([C.c_int64] + [_dp] * 5 + [_dp, C.c_int, C.c_double,
                                  C.c_double, C.c_int64, _nullable(_ip), _nullable(_ip),
                                  _nullable(_ip), _dp])
        L.or_dt_limit.restype = C.c_int64
        L.or_kick.argtypes = [C.c_int64] + [_dp] * 8 + [C.c_double]
        L.or_kick.restype = None
        L.or_drift.argtypes = [C.c_int64] + [_dp] * 6 + [C.c_double, _dp, C.c_int]
        L.or_drift.restype = None
        _LIB = L
    return _LIB


# The kernels Section 3.1 lists, by the id the C code takes, with the square
# of gamma_k = H / h for h = twice the kernel's standard deviation (the
# smoothing length is the same for every kernel: only the cut-off moves).
# Exact fractions: sigma^2 = (1/3) int r^2 W dV is rational for these
# piecewise polynomials; the tests recompute them from the kernels' shapes.
KERNELS = {
    "wendland_c2": (0, (15, 4)),
    "wendland_c4": (1, (39, 8)),
    "wendland_c6": (2, (6, 1)),
    "cubic_spline": (3, (10, 3)),
    "quartic_spline": (4, (375, 92)),
    "quintic_spline": (5, (135, 28)),
}


def kernel_gamma(name: str) -> float:
    """gamma_k of a kernel: H / h with h twice its standard deviation."""
    p, q = KERNELS[name][1]
    return math.sqrt(p / q)


@dataclass
class Params:
    """Method parameters, with the paper's values where it gives them."""

    box: tuple = (1.0, 1.0, 1.0)
    periodic: bool = True
    # H = gamma_k h; sqrt(15)/2 makes h twice the kernel's standard deviation.
    gamma_k: float = math.sqrt(15.0) / 2.0
    kernel: str = "wendland_c2"    # a key of KERNELS (with_kernel sets gamma_k)
    eta: float = 1.2348
    gamma_gas: float = 5.0 / 3.0   # ratio of specific heats (Section 8, gas gamma 5/3)
    beta_v: float = 3.0            # signal-velocity constant (Section 3.2)
    eps_b: float = 1e-4            # Balsara switch regulariser (Section 3.2)
    h_tol: float = 1e-4            # relative Newton-Raphson tolerance (Section 3.1)
    max_iter: int = 30
    h_max: Optional[float] = None  # default: min(box) / (3 gamma_k) * (1 - 1e-6)
    # "energy": density-energy (u is the internal energy, with conduction);
    # "entropy": density-entropy, the Gadget2 flavour of Section 3.2 (the u
    # array holds the adiabat A, no conduction, du/dt becomes dA/dt);
    # "phantom": the Phantom-like flavour of Appendix A (density-energy, fixed
    # alpha_c = 1, conduction speed without the velocity term; its viscosity
    # switch decays with ell = 0.25);
    # "pressure_energy": pressure-smoothed SPH of Appendix A (the smoothed
    # pressure P_hat from u, factors f_ij, density-flavour viscosity, no
    # conduction; u > 0 everywhere);
    # "anarchy_pu": Anarchy-PU of Appendix A (pressure-energy plus conduction
    # with the mean alpha_c and speed c_i + c_j + mu; its conduction parameter
    # evolves with beta_c = 0.01 and no shock limiter, its viscosity switch
    # with ell = 0.25)
    # "gdf": the Gasoline-2-like flavour of Appendix A (geometric density
    # average force: both pressures over rho_i rho_j on the mean gradient,
    # the GDF correction f and the dimensional conduction parameter from the
    # shear tensor, both from gdf(); the density flavours' viscosity)
    flavour: str = "energy"

    def flavour_id(self) -> int:
        return {"energy": 0, "entropy": 1, "phantom": 2, "pressure_energy": 3,
                "anarchy_pu": 4, "gdf": 5}[self.flavour]

    def smoothed_pressure(self) -> bool:
        return self.flavour in ("pressure_energy", "anarchy_pu")

    def hmax(self) -> float:
        if self.h_max is not None:
            return float(self.h_max)
        return min(self.box) / (3.0 * self.gamma_k) * (1.0 - 1e-6)

    @classmethod
    def with_kernel(cls, name: str, **kw):
        """Parameters for another kernel of the family, with its own gamma_k."""
        return cls(kernel=name, gamma_k=kernel_gamma(name), **kw)

    def kernel_id(self) -> int:
        return KERNELS[self.kernel][0]


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _pos(ps):
    return _f64(ps.x), _f64(ps.y), _f64(ps.z)


def _recv_arr(recv, n):
    if recv is None:
        return None, n
    r = np.ascontiguousarray(np.asarray(recv, dtype=np.int64))
    return r, int(r.shape[0])


def kernel(name, r, h, gamma_k=None):
    """Vectorised W, dW/dr, dW/dh of a kernel of KERNELS (its own gamma_k
    unless given)."""
    g = kernel_gamma(name) if gamma_k is None else float(gamma_k)
    r = _f64(np.atleast_1d(r))
    h = _f64(np.broadcast_to(np.asarray(h, dtype=np.float64), r.shape))
    w = np.empty_like(r)
    d1 = np.empty_like(r)
    d2 = np.empty_like(r)
    lib().or_kernel_array(KERNELS[name][0], r.shape[0], r, h, g, w, d1, d2)
    return w, d1, d2


def wc2(r, h, gamma_k=Params.gamma_k):
    """Vectorised W, dW/dr, dW/dh of the Wendland C2 kernel."""
    r = _f64(np.atleast_1d(r))
    h = _f64(np.broadcast_to(np.asarray(h, dtype=np.float64), r.shape))
    w = np.empty_like(r)
    d1 = np.empty_like(r)
    d2 = np.empty_like(r)
    lib().or_wc2_array(r.shape[0], r, h, float(gamma_k), w, d1, d2)
    return w, d1, d2


# ---------------------------------------------------------------------------
# Candidate lists (k-d tree supersets; the C code decides membership).
# ---------------------------------------------------------------------------

def _wrapped_positions(ps, periodic):
    p = np.stack(_pos(ps), axis=1)
    if periodic:
        b = np.asarray(ps.box, dtype=np.float64)
        p = np.mod(p, b)
        p = np.where(p >= b, p - b, p)
    return p


_TREE_CACHE = {}


def _tree(p, ps, periodic, cache=True):
    """k-d tree over positions p; the tree over a whole particle set is kept
    for reuse while the set's position arrays are the same objects."""
    from scipy.spatial import cKDTree
    key = None
    if cache and p.shape[0] == ps.n:
        key = (id(ps.x), id(ps.y), id(ps.z), ps.n, bool(periodic), tuple(ps.box),
               float(ps.x[: 8].sum() + ps.y[-8:].sum() + ps.z[ps.n // 2]))
        hit = _TREE_CACHE.get("last")
        if hit is not None and hit[0] == key:
            return hit[1]
    t = cKDTree(p, boxsize=np.asarray(ps.box, dtype=np.float64) if periodic else None)
    if key is not None:
        _TREE_CACHE["last"] = (key, t)
    return t


def _pairs(lists, k_offset=0):
    lens = np.fromiter((len(l) for l in lists), count=len(lists), dtype=np.int64)
    if lens.sum() == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    idx = np.concatenate([np.asarray(l, dtype=np.int64) for l in lists if len(l)])
    k = np.repeat(np.arange(len(lists), dtype=np.int64) + k_offset, lens)
    return k, idx


def _csr(k, idx, nrecv, n):
    key = np.unique(k * np.int64(n) + idx)
    kk = key // n
    jj = key - kk * n
    off = np.zeros(nrecv + 1, np.int64)
    np.add.at(off, kk + 1, 1)
    off = np.cumsum(off)
    return np.ascontiguousarray(off), np.ascontiguousarray(jj)


_PAD = 1.0 + 1e-9


def density_candidates(ps, h, params: Params, recv):
    """Ascending superset of {j : |x_i - x_j| < H_i} for each receiver."""
    p = _wrapped_positions(ps, params.periodic)
    tree = _tree(p, ps, params.periodic)
    ri = np.arange(ps.n) if recv is None else np.asarray(recv)
    H = params.gamma_k * np.asarray(h, dtype=np.float64)
    ks, js = [], []
    chunk = 65536
    for s in range(0, len(ri), chunk):
        sl = ri[s:s + chunk]
        lists = tree.query_ball_point(p[sl], H[sl] * _PAD, return_sorted=True)
        k, j = _pairs(lists, s)
        ks.append(k)
        js.append(j)
    return _csr(np.concatenate(ks), np.concatenate(js), len(ri), ps.n)


def force_candidates(ps, h, params: Params, recv):
    """Ascending superset of {j : |x_i - x_j| < max(H_i, H_j)}: the H_i part
    from one tree query, the H_j part from trees over bands of H (factor 2)."""
    p = _wrapped_positions(ps, params.periodic)
    H = params.gamma_k * np.asarray(h, dtype=np.float64)
    ri = np.arange(ps.n) if recv is None else np.asarray(recv)
    tree = _tree(p, ps, params.periodic)
    ks, js = [], []
    chunk = 65536
    for s in range(0, len(ri), chunk):
        sl = ri[s:s + chunk]
        k, j = _pairs(tree.query_ball_point(p[sl], H[sl] * _PAD, return_sorted=True), s)
        ks.append(k)
        js.append(j)
    lo = float(H.min())
    band = np.floor(np.log2(H / lo)).astype(np.int64)
    for b in np.unique(band):
        members = np.nonzero(band == b)[0]
        sub = _tree(p[members], ps, params.periodic, cache=False)
        rb = float(H[members].max()) * _PAD
        for s in range(0, len(ri), chunk):
            sl = ri[s:s + chunk]
            lists = sub.query_ball_point(p[sl], rb)
            k, j = _pairs(lists, s)
            ks.append(k)
            js.append(members[j])
    return _csr(np.concatenate(ks), np.concatenate(js), len(ri), ps.n)


def _resolve_mode(mode, n):
    if mode == "auto":
        return "brute" if n <= 8192 else "tree"
    return mode


# ---------------------------------------------------------------------------
# The passes.
# ---------------------------------------------------------------------------

def density(ps, h, params: Params, recv=None, mode="auto"):
    """Density sums at the given h for the receivers (Section 3.1)."""
    mode = _resolve_mode(mode, ps.n)
    h = _f64(h)
    r, nrecv = _recv_arr(recv, ps.n)
    off = idx = None
    if mode == "tree":
        off, idx = density_candidates(ps, h, params, r)
    out = {k: np.zeros(nrecv) for k in ("rho", "rho_dh", "n", "n_dh", "div_sum",
                                        "curl_x", "curl_y", "curl_z")}
    nngb = np.zeros(nrecv, np.int64)
    x, y, z = _pos(ps)
    total = lib().or_density(ps.n, x, y, z, _f64(ps.vx), _f64(ps.vy), _f64(ps.vz), _f64(ps.m), h,
                             _f64(ps.box), int(params.periodic), float(params.gamma_k),
                             params.kernel_id(), nrecv, r,
                             off, idx, out["rho"], out["rho_dh"], out["n"], out["n_dh"],
                             out["div_sum"], out["curl_x"], out["curl_y"], out["curl_z"], nngb)
    out["nngb"] = nngb
    out["total"] = int(total)
    if params.smoothed_pressure():
        out["P_hat"], out["P_hat_dh"] = np.zeros(nrecv), np.zeros(nrecv)
        lib().or_pressure(ps.n, x, y, z, _f64(ps.m), _f64(ps.u), h, _f64(ps.box),
                          int(params.periodic), float(params.gamma_k), params.kernel_id(),
                          float(params.gamma_gas), nrecv, r, off, idx, out["P_hat"],
                          out["P_hat_dh"])
    return out


def pressure(ps, h, params: Params, recv=None, mode="auto"):
    """Smoothed pressure and its h-derivative at the given h (or_pressure,
    Appendix A)."""
    mode = _resolve_mode(mode, ps.n)
    h = _f64(h)
    r, nrecv = _recv_arr(recv, ps.n)
    off = idx = None
    if mode == "tree":
        off, idx = density_candidates(ps, h, params, r)
    P, P_dh = np.zeros(nrecv), np.zeros(nrecv)
    x, y, z = _pos(ps)
    lib().or_pressure(ps.n, x, y, z, _f64(ps.m), _f64(ps.u), h, _f64(ps.box),
                      int(params.periodic), float(params.gamma_k), params.kernel_id(),
                      float(params.gamma_gas), nrecv, r, off, idx, P, P_dh)
    return P, P_dh


def h_update(h, nd, nd_dh, params: Params, lo=None, hi=None):
    """One safeguarded Newton-Raphson step per particle (or_h_update). lo/hi
    are the per-particle bracket (largest h with G < 0, smallest with G > 0),
    updated in place; None starts without one."""
    h = _f64(h)
    lo = np.zeros(h.shape[0]) if lo is None else lo
    hi = np.full(h.shape[0], np.inf) if hi is None else hi
    assert lo.dtype == np.float64 and hi.dtype == np.float64
    assert lo.flags.c_contiguous and hi.flags.c_contiguous
    hn = np.empty_like(h)
    conv = np.empty(h.shape[0], np.int32)
    lib().or_h_update(h.shape[0], h, _f64(nd), _f64(nd_dh), float(params.eta),
                      float(params.h_tol), float(params.hmax()), lo, hi, hn, conv)
    return hn, conv.astype(bool)


def ghost(dens, u, h, params: Params):
    """Pressure, sound speed, f-factor, Balsara switch and A = f P / rho^2
    (pressure-energy: P = P_hat and A the grad-h term F of its f_ij)."""
    n = dens["rho"].shape[0]
    out = {k: np.zeros(n) for k in ("f", "P", "c", "balsara", "A", "div_v", "curl_v")}
    extra = ([_f64(dens[k]) for k in ("n", "n_dh", "P_hat", "P_hat_dh")]
             if params.smoothed_pressure() else [None] * 4)
    lib().or_ghost(n, _f64(dens["rho"]), _f64(dens["rho_dh"]), _f64(dens["div_sum"]),
                   _f64(dens["curl_x"]), _f64(dens["curl_y"]), _f64(dens["curl_z"]), _f64(u),
                   _f64(h), float(params.gamma_gas), float(params.eps_b), out["f"], out["P"],
                   out["c"], out["balsara"], out["A"], out["div_v"], out["curl_v"],
                   params.flavour_id(), *extra)
    return out


def solve_h(ps, params: Params, recv=None, mode="auto", h0=None):
    """Per-particle Newton-Raphson on n(h) h^3 = eta^3 (Section 3.1).

    Each receiver iterates independently (its sums depend only on its own h).
    Returns the final h (the one the returned sums were evaluated at), the
    density sums there, a converged flag and the number of passes used.
    """
    mode = _resolve_mode(mode, ps.n)
    ri = np.arange(ps.n) if recv is None else np.asarray(recv, dtype=np.int64)
    nr = ri.shape[0]
    h_all = _f64(ps.h if h0 is None else h0).copy()
    h_all = np.minimum(h_all, params.hmax())
    h = h_all[ri].copy()
    conv = np.zeros(nr, bool)
    dens = None
    todo = np.arange(nr)
    iters = np.zeros(nr, np.int32)
    lo = np.zeros(nr)          # bracket of the root, per receiver
    hi = np.full(nr, np.inf)
    passes = 0
    while todo.size and passes < params.max_iter:
        passes += 1
        h_all[ri[todo]] = h[todo]
        d = density(ps, h_all, params, recv=ri[todo], mode=mode)
        if dens is None:
            dens = {k: np.zeros(nr, dtype=v.dtype) for k, v in d.items() if k != "total"}
        for k, v in d.items():
            if k != "total":
                dens[k][todo] = v
        iters[todo] += 1
        lo_t, hi_t = lo[todo], hi[todo]
        hn, c = h_update(h[todo], d["n"], d["n_dh"], params, lo_t, hi_t)
        lo[todo], hi[todo] = lo_t, hi_t
        conv[todo] = c
        last = passes == params.max_iter
        # A receiver still unconverged after the last allowed pass keeps the
        # h its sums were evaluated at.
        if not last:
            h[todo] = hn
        todo = todo[~c]
    return h, dens, conv, iters, passes


def force(ps, h, gst, dens_rho, params: Params, recv=None, mode="auto", cand=None):
    """Accelerations, du/dt and signal velocity for the receivers (Sections
    3.2, 3.3). ``gst`` and ``dens_rho`` hold every particle's ghost state
    (only neighbours' entries are read)."""
    mode = _resolve_mode(mode, ps.n)
    h = _f64(h)
    r, nrecv = _recv_arr(recv, ps.n)
    off = idx = None
    if mode == "tree":
        off, idx = cand if cand is not None else force_candidates(ps, h, params, r)
    out = {k: np.zeros(nrecv) for k in ("ax", "ay", "az", "du", "vsig", "du_energy")}
    nf = np.zeros(nrecv, np.int64)
    x, y, z = _pos(ps)
    total = lib().or_force(ps.n, x, y, z, _f64(ps.vx), _f64(ps.vy), _f64(ps.vz), _f64(ps.m),
                           _f64(ps.u), h, _f64(dens_rho), _f64(gst["P"]), _f64(gst["c"]),
                           _f64(gst["f"]), _f64(gst["balsara"]), _f64(ps.alpha_v),
                           _f64(ps.alpha_c), _f64(ps.box), int(params.periodic),
                           float(params.gamma_k), params.kernel_id(), float(params.beta_v),
                           nrecv, r, off, idx,
                           out["ax"], out["ay"], out["az"], out["du"], out["vsig"], nf,
                           params.flavour_id(), float(params.gamma_gas),
                           out["du_energy"],
                           _f64(gst["A"]) if params.smoothed_pressure() else None)
    out["nforce"] = nf
    out["total"] = int(total)
    return out


def sums(m, vx, vy, vz, ax, ay, az, du):
    out = np.zeros(6)
    lib().or_sums(len(m), _f64(m), _f64(vx), _f64(vy), _f64(vz), _f64(ax), _f64(ay), _f64(az),
                  _f64(du), out)
    return out


def force_needed(ps, h, params: Params, recv, mode="auto", cand=None):
    """Receivers plus every particle inside their force neighbourhoods."""
    mode = _resolve_mode(mode, ps.n)
    if recv is None:
        return np.arange(ps.n)
    if mode == "brute":
        return np.arange(ps.n)
    off, idx = cand if cand is not None else force_candidates(
        ps, _f64(h), params, np.asarray(recv, np.int64))
    return np.unique(np.concatenate([np.asarray(recv, np.int64), idx]))


def fixed_h_step(ps, params: Params, recv=None, mode="auto", h=None):
    """Density, ghost and force at the given (input) h, no iteration.

    Density and ghost are evaluated for the receivers and everything in their
    force neighbourhoods; the force for the receivers only. Entries of
    particles outside that set are NaN so any stray read shows up.
    """
    h = _f64(ps.h if h is None else h)
    cand = None
    if recv is not None and _resolve_mode(mode, ps.n) == "tree":
        cand = force_candidates(ps, h, params, np.asarray(recv, np.int64))
    need = force_needed(ps, h, params, recv, mode, cand=cand)
    d = density(ps, h, params, recv=need, mode=mode)
    g = ghost(d, _f64(ps.u)[need], h[need], params)
    full = {k: np.full(ps.n, np.nan) for k in ("P", "c", "f", "balsara", "A")}
    rho = np.full(ps.n, np.nan)
    for k in full:
        full[k][need] = g[k]
    rho[need] = d["rho"]
    fo = force(ps, h, full, rho, params, recv=recv, mode=mode, cand=cand)
    ri = np.arange(ps.n) if recv is None else np.asarray(recv, np.int64)
    pos = np.searchsorted(need, ri)
    res = {"h": h[ri]}
    for k, v in d.items():
        if k != "total":
            res[k] = v[pos]
    for k, v in g.items():
        res[k] = v[pos]
    for k, v in fo.items():
        if k != "total":
            res[k] = v
    res["n_dens_total"] = int(res["nngb"].sum())
    res["n_force_total"] = fo["total"]
    return res


def nr_step(ps, params: Params, mode="auto"):
    """Full step on every particle: h iteration with its density passes,
    ghost, force and the global sums."""
    h, dens, conv, iters, passes = solve_h(ps, params, mode=mode)
    g = ghost(dens, ps.u, h, params)
    fo = force(ps, h, g, dens["rho"], params, mode=mode)
    res = {"h": h, "converged": conv, "iters": iters, "passes": passes}
    res.update({k: v for k, v in dens.items()})
    res.update(g)
    res.update({k: v for k, v in fo.items() if k != "total"})
    res["sums"] = sums(ps.m, ps.vx, ps.vy, ps.vz, fo["ax"], fo["ay"], fo["az"], fo["du"])
    res["n_dens_total"] = int(dens["nngb"].sum())
    res["n_force_total"] = fo["total"]
    return res


# ---------------------------------------------------------------------------
# Friends-of-friends groups (Section 9.1).
# ---------------------------------------------------------------------------

def fof_link_length(ps, frac=0.2):
    """frac times the mean inter-particle separation (V / N)^(1/3)."""
    vol = float(np.prod(np.asarray(ps.box, dtype=np.float64)))
    return frac * (vol / ps.n) ** (1.0 / 3.0)


def fof(ps, b, periodic=True, mode="auto"):
    """Friends-of-friends groups at linking length b (or_fof): returns
    (group, links) with group[i] the smallest index of i's group and links the
    number of linked pairs. Tree mode takes candidates from a k-d tree within
    b (padded); the C code applies the exact test, so both modes agree."""
    mode = _resolve_mode(mode, ps.n)
    off = idx = None
    if mode == "tree":
        p = _wrapped_positions(ps, periodic)
        tree = _tree(p, ps, periodic)
        ks, js = [], []
        chunk = 65536
        for s in range(0, ps.n, chunk):
            lists = tree.query_ball_point(p[s:s + chunk], b * _PAD, return_sorted=True)
            k, j = _pairs(lists, s)
            ks.append(k)
            js.append(j)
        off, idx = _csr(np.concatenate(ks), np.concatenate(js), ps.n, ps.n)
    group = np.empty(ps.n, np.int64)
    x, y, z = _pos(ps)
    links = lib().or_fof(ps.n, x, y, z, _f64(ps.box), int(periodic), float(b) * float(b),
                         off, idx, group)
    return group, int(links)


# ---------------------------------------------------------------------------
# Short-range softened gravity by direct summation (Sections 4.1 and 4.4).
# ---------------------------------------------------------------------------

def grav_pair(r, H, rs=0.0):
    """(phi_s, k/r) of or_grav_pair for an array of separations."""
    r = _f64(np.atleast_1d(r))
    phi = np.empty_like(r)
    kr = np.empty_like(r)
    lib().or_grav_pair_array(r.shape[0], r, float(H), float(rs), phi, kr)
    return phi, kr


def gravity(ps, G, H, rs, rp2p, periodic=True, recv=None, mode="auto"):
    """Accelerations, potential and term scale of or_gravity for the
    receivers (all particles when recv is None), over j != i with
    r_ij < rp2p."""
    mode = _resolve_mode(mode, ps.n)
    r, nrecv = _recv_arr(recv, ps.n)
    off = idx = None
    if mode == "tree":
        p = _wrapped_positions(ps, periodic)
        tree = _tree(p, ps, periodic)
        ri = np.arange(ps.n) if recv is None else np.asarray(recv)
        ks, js = [], []
        chunk = 65536
        for s in range(0, len(ri), chunk):
            lists = tree.query_ball_point(p[ri[s:s + chunk]], rp2p * _PAD, return_sorted=True)
            k, j = _pairs(lists, s)
            ks.append(k)
            js.append(j)
        off, idx = _csr(np.concatenate(ks), np.concatenate(js), len(ri), ps.n)
    out = {k: np.zeros(nrecv) for k in ("ax", "ay", "az", "pot", "scale")}
    x, y, z = _pos(ps)
    total = lib().or_gravity(ps.n, x, y, z, _f64(ps.m), _f64(ps.box), int(periodic), float(G),
                             float(H), float(rs), float(rp2p), nrecv, r, off, idx, out["ax"],
                             out["ay"], out["az"], out["pot"], out["scale"])
    out["pairs"] = int(total)
    return out


# ---------------------------------------------------------------------------
# SPHENIX viscosity switch (Section 3.3).
# ---------------------------------------------------------------------------

SPHENIX_ALPHA_V_MAX = 2.0   # Section 3.3: maximal viscosity parameter
SPHENIX_ELL = 0.05          # Section 3.3: viscosity decay length
PHANTOM_ELL = 0.25          # Appendix A: the Phantom-like flavour's decay length


def alpha_v_update(alpha, div_old, div_new, c, h, vsig, dt, params: Params,
                   alpha_max=SPHENIX_ALPHA_V_MAX, ell=SPHENIX_ELL):
    """New alpha_V of every particle after a step dt (or_alpha_v_update)."""
    a = _f64(alpha).copy()
    n = a.shape[0]
    lib().or_alpha_v_update(n, _f64(div_old), _f64(div_new), _f64(c), _f64(h), _f64(vsig),
                            float(dt), float(params.gamma_k), float(alpha_max), float(ell), a)
    return a


# ---------------------------------------------------------------------------
# The rest of SPHENIX (Section 3.3) and the time integration (Sections 2.4,
# 3.4).
# ---------------------------------------------------------------------------

SPHENIX_BETA_C = 1.0        # Section 3.3: conduction source strength
ANARCHY_BETA_C = 0.01       # Appendix A: Anarchy-PU's conduction source strength
ANARCHY_ELL = 0.25          # Appendix A: Anarchy-PU's viscosity decay length


def switch_constants(params: Params):
    """(ell, beta_c, alpha_V,max of the shock limiter) of a flavour's
    viscosity switch and conduction parameter; alpha_V,max = inf leaves only
    the plain cap alpha_c <= alpha_c,max (Anarchy-PU has no shock limiter)."""
    if params.flavour == "anarchy_pu":
        return ANARCHY_ELL, ANARCHY_BETA_C, math.inf
    if params.flavour == "phantom":
        return PHANTOM_ELL, SPHENIX_BETA_C, SPHENIX_ALPHA_V_MAX
    return SPHENIX_ELL, SPHENIX_BETA_C, SPHENIX_ALPHA_V_MAX
SPHENIX_ALPHA_C_MIN = 0.0   # Section 3.3: smallest conduction parameter
SPHENIX_ALPHA_C_MAX = 1.0   # Section 3.3: constant of the shock limiter
DT_LIMIT_DELTA = 4.0        # Section 3.4: largest step ratio between neighbours


def gradient(ps, h, rho, P, params: Params, recv=None, mode="auto", c=None):
    """SPHENIX gradient loop (or_gradient): Laplacian of u, conduction speed
    and the largest neighbouring alpha_V for the receivers. rho and P hold
    every particle's values (only neighbours' entries are read); c, every
    particle's sound speed, is required by (and only read for) Anarchy-PU."""
    if params.flavour == "anarchy_pu":
        assert c is not None, "Anarchy-PU's conduction speed needs the sound speeds"
    else:
        c = None
    mode = _resolve_mode(mode, ps.n)
    h = _f64(h)
    r, nrecv = _recv_arr(recv, ps.n)
    off = idx = None
    if mode == "tree":
        off, idx = density_candidates(ps, h, params, r)
    out = {k: np.zeros(nrecv) for k in ("lap_u", "vc", "avmax")}
    x, y, z = _pos(ps)
    total = lib().or_gradient(ps.n, x, y, z, _f64(ps.vx), _f64(ps.vy), _f64(ps.vz), _f64(ps.m),
                              _f64(ps.u), h, _f64(rho), _f64(P), _f64(ps.alpha_v), _f64(ps.box),
                              int(params.periodic), float(params.gamma_k), params.kernel_id(),
                              nrecv, r, off, idx, out["lap_u"], out["vc"], out["avmax"],
                              None if c is None else _f64(c))
    out["total"] = int(total)
    return out


# Conduction constant of the GDF flavour (Appendix A).
GDF_C = 0.03


def gdf(ps, h, rho, params: Params, recv=None, mode="auto"):
    """The GDF flavour's correction f and conduction parameter alpha_c
    (or_gdf) for the receivers, from every particle's h and rho."""
    mode = _resolve_mode(mode, ps.n)
    h = _f64(h)
    r, nrecv = _recv_arr(recv, ps.n)
    off = idx = None
    if mode == "tree":
        off, idx = density_candidates(ps, h, params, r)
    f = np.zeros(nrecv)
    ac = np.zeros(nrecv)
    x, y, z = _pos(ps)
    lib().or_gdf(ps.n, x, y, z, _f64(ps.vx), _f64(ps.vy), _f64(ps.vz), _f64(ps.m), h,
                 _f64(rho), _f64(ps.box), int(params.periodic), float(params.gamma_k),
                 params.kernel_id(), float(GDF_C), nrecv, r, off, idx, f, ac)
    return f, ac


def gdf_detector(ps, h, params: Params, recv=None, mode="auto"):
    """The GDF shock detector D of the receivers (or_gdf_detector)."""
    mode = _resolve_mode(mode, ps.n)
    h = _f64(h)
    r, nrecv = _recv_arr(recv, ps.n)
    off = idx = None
    if mode == "tree":
        off, idx = density_candidates(ps, h, params, r)
    D = np.zeros(nrecv)
    x, y, z = _pos(ps)
    lib().or_gdf_detector(ps.n, x, y, z, _f64(ps.vx), _f64(ps.vy), _f64(ps.vz), _f64(ps.m),
                          _f64(ps.u), h, _f64(ps.box), int(params.periodic),
                          float(params.gamma_k), params.kernel_id(), float(params.gamma_gas),
                          nrecv, r, off, idx, D)
    return D


def gdf_alpha_v_update(alpha, D_old, D_new, c, h, vsig, B, dt, alpha_max=SPHENIX_ALPHA_V_MAX):
    """New GDF viscosity parameter of every particle after a step dt
    (or_gdf_alpha_v_update; alpha_max read as SPHENIX's, which the paper
    does not restate for this flavour)."""
    a = _f64(alpha).copy()
    lib().or_gdf_alpha_v_update(a.shape[0], _f64(D_old), _f64(D_new), _f64(c), _f64(h),
                                _f64(vsig), _f64(B), float(dt), float(alpha_max), a)
    return a


def alpha_c_update(alpha, lap_u, u, h, vc, avmax, dt, params: Params,
                   beta_c=SPHENIX_BETA_C, a_min=SPHENIX_ALPHA_C_MIN, a_max=SPHENIX_ALPHA_C_MAX,
                   av_max=SPHENIX_ALPHA_V_MAX):
    """New alpha_c of every particle after a step dt (or_alpha_c_update)."""
    a = _f64(alpha).copy()
    lib().or_alpha_c_update(a.shape[0], _f64(lap_u), _f64(u), _f64(h), _f64(vc), _f64(avmax),
                            float(dt), float(params.gamma_k), float(beta_c), float(a_min),
                            float(a_max), float(av_max), a)
    return a


def dt_cfl(h, vsig, params: Params, c_cfl):
    h = _f64(h)
    dt = np.empty_like(h)
    lib().or_dt_cfl(h.shape[0], h, _f64(vsig), float(params.gamma_k), float(c_cfl), dt)
    return dt


def dt_limit(ps, h, dt, params: Params, delta=DT_LIMIT_DELTA, recv=None, mode="auto"):
    """Each receiver's step capped at delta times the smallest step of its
    force-loop neighbours (or_dt_limit)."""
    mode = _resolve_mode(mode, ps.n)
    h = _f64(h)
    r, nrecv = _recv_arr(recv, ps.n)
    off = idx = None
    if mode == "tree":
        off, idx = force_candidates(ps, h, params, r)
    out = np.zeros(nrecv)
    x, y, z = _pos(ps)
    lib().or_dt_limit(ps.n, x, y, z, h, _f64(dt), _f64(ps.box), int(params.periodic),
                      float(params.gamma_k), float(delta), nrecv, r, off, idx, out)
    return out


def kick(v, u, a, du, dt_half):
    """Half kick in place: v (3 x n) += a dt/2, u += du/dt dt/2."""
    lib().or_kick(u.shape[0], v[0], v[1], v[2], u, _f64(a[0]), _f64(a[1]), _f64(a[2]), _f64(du),
                  float(dt_half))


def drift(pos, v, dt, box, periodic=True):
    """Drift in place: pos (3 x n) += v dt, wrapped into the box."""
    lib().or_drift(pos.shape[1], pos[0], pos[1], pos[2], _f64(v[0]), _f64(v[1]), _f64(v[2]),
                   float(dt), _f64(box), int(periodic))


def sphenix_run(ps, params: Params, n_steps, c_cfl=0.2, delta=DT_LIMIT_DELTA, mode="auto",
                dt_max=None, callback=None):
    """Kick-drift-kick integration with one global step (the smallest
    limited CFL step; every particle active). Per step: half kick, drift
    (with v and u predicted to the end of the drift by the previous
    derivatives), h iteration, ghost and force with the viscosity and
    conduction parameters of the step before, then the viscosity switch, the
    gradient loop and the conduction parameter, the second half kick and the
    next step size. Returns the final state and the list of (t, dt)."""
    n = ps.n
    pos = np.stack([_f64(ps.x), _f64(ps.y), _f64(ps.z)]).copy()
    v = np.stack([_f64(ps.vx), _f64(ps.vy), _f64(ps.vz)]).copy()
    u = _f64(ps.u).copy()
    q = ps.copy()

    def evaluate(h0, vp=None, up=None):
        for k, a in zip(("x", "y", "z"), pos):
            setattr(q, k, np.ascontiguousarray(a))
        q.vx, q.vy, q.vz = (np.ascontiguousarray(a) for a in (v if vp is None else vp))
        q.u = (u if up is None else up).copy()
        h, _, conv, _, _ = solve_h(q, params, mode=mode, h0=h0)
        r = fixed_h_step(q, params, mode=mode, h=h)
        return h, r

    h, r = evaluate(_f64(ps.h))
    alpha_v = _f64(ps.alpha_v).copy()
    alpha_c = _f64(ps.alpha_c).copy()
    dt = float(dt_limit(q, h, dt_cfl(h, r["vsig"], params, c_cfl), params, delta, mode=mode).min())
    if dt_max is not None:
        dt = min(dt, dt_max)
    t = 0.0
    hist = []
    for step in range(n_steps):
        a = (r["ax"], r["ay"], r["az"])
        kick(v, u, a, r["du"], 0.5 * dt)
        drift(pos, v, dt, ps.box, params.periodic)
        div_old = r["div_v"]
        q.alpha_v, q.alpha_c = alpha_v.copy(), alpha_c.copy()
        # the forces at the end of the drift see v and u predicted to that
        # time with the derivatives of the step before (the half-step values
        # would make the energy equation first order in dt)
        vp = v + 0.5 * dt * np.stack(a)
        up = u + 0.5 * dt * r["du"]
        h, r = evaluate(h, vp, up)
        ell, beta_c, av_lim = switch_constants(params)
        alpha_v = alpha_v_update(alpha_v, div_old, r["div_v"], r["c"], h, r["vsig"], dt, params,
                                 ell=ell)
        q.alpha_v = alpha_v.copy()
        g = gradient(q, h, r["rho"], r["P"], params, mode=mode, c=r["c"])
        alpha_c = alpha_c_update(alpha_c, g["lap_u"], up, h, g["vc"], g["avmax"], dt, params,
                                 beta_c=beta_c, av_max=av_lim)
        kick(v, u, (r["ax"], r["ay"], r["az"]), r["du"], 0.5 * dt)
        t += dt
        hist.append((t, dt))
        if callback is not None:
            callback(step, t, pos, v, u, h, r)
        dt = float(dt_limit(q, h, dt_cfl(h, r["vsig"], params, c_cfl), params, delta,
                            mode=mode).min())
        if dt_max is not None:
            dt = min(dt, dt_max)
    return dict(pos=pos, v=v, u=u, h=h, alpha_v=alpha_v, alpha_c=alpha_c, t=t, hist=hist,
                last=r)
