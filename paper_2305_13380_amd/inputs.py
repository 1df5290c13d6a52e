"""Seeded synthetic particle sets for the SPH neighbour-loop workloads.

This module is the only code shared by the HIP path and the CPU oracle. It
draws particle-carried inputs (positions, velocities, masses, internal
energies, smoothing-length guesses, dissipation coefficients, activity flags)
and nothing else: it holds no kernel, no density or force arithmetic and no
smoothing-length solve.

All sets live in a periodic box whose lower corner is the origin. Positions are
float64; every other particle-carried quantity is float32, which is the layout
the library's C-ABI takes (structure of arrays, one contiguous array per
field). Particles are returned in a seeded random order so that the spatial
sort on the device has real work to do.

The workloads stand in for the paper's cosmological and test-problem boxes
(which are not available here):

* ``lattice_box``   -- a cubic lattice with per-axis uniform jitter; the
  uniform-density case and the Sedov blast start from it.
* ``lognormal_box`` -- particles sampled from a lognormal density field built
  from a Gaussian random field with power spectrum P(k) ~ k^-2, giving density
  contrasts of 10^4 and more, i.e. the uneven, clustered neighbourhoods the
  nested-grid design of the paper (Section 2) is meant for.
* ``serving_stream`` -- many independent boxes of log-uniform size arriving on
  a Poisson clock.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator, Optional

import numpy as np

# Smoothing-scale parameter of the workloads (the paper's eta, Section 3.1).
ETA = 1.2348

F32_FIELDS = ("vx", "vy", "vz", "m", "u", "h", "alpha_v", "alpha_c")
F64_FIELDS = ("x", "y", "z")


@dataclass
class ParticleSet:
    """Structure-of-arrays particle set in a periodic box ``[0, box)^3``."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray
    u: np.ndarray
    h: np.ndarray
    alpha_v: np.ndarray
    alpha_c: np.ndarray
    active: Optional[np.ndarray] = None
    box: tuple = (1.0, 1.0, 1.0)
    eta: float = ETA
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def positions(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def copy(self) -> "ParticleSet":
        kw = {k: getattr(self, k).copy() for k in F64_FIELDS + F32_FIELDS}
        return ParticleSet(**kw, active=None if self.active is None else self.active.copy(),
                           box=tuple(self.box), eta=self.eta, name=self.name, meta=dict(self.meta))

    def subset(self, idx: np.ndarray) -> "ParticleSet":
        kw = {k: np.ascontiguousarray(getattr(self, k)[idx]) for k in F64_FIELDS + F32_FIELDS}
        act = None if self.active is None else np.ascontiguousarray(self.active[idx])
        return ParticleSet(**kw, active=act, box=tuple(self.box), eta=self.eta,
                           name=self.name + "[subset]", meta=dict(self.meta))


def _finish(pos, vel, m, u, h, rng, box, name, meta, alpha=True, active=None) -> ParticleSet:
    n = pos.shape[0]
    order = rng.permutation(n)
    pos = pos[order]
    vel = vel[order]
    u = np.broadcast_to(u, (n,))[order] if np.ndim(u) else np.full(n, u)
    h = np.broadcast_to(h, (n,))[order] if np.ndim(h) else np.full(n, h)
    if alpha:
        # Per-particle viscosity and conduction coefficients: the paper evolves
        # them in time (Section 3.3) with maxima 2 and 1; here they are inputs.
        av = rng.uniform(0.1, 2.0, n)
        ac = rng.uniform(0.0, 1.0, n)
    else:
        av = np.full(n, 0.8)
        ac = np.zeros(n)
    if active is not None:
        active = np.ascontiguousarray(active[order].astype(np.uint8))
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    f64 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return ParticleSet(
        x=f64(pos[:, 0]), y=f64(pos[:, 1]), z=f64(pos[:, 2]),
        vx=f32(vel[:, 0]), vy=f32(vel[:, 1]), vz=f32(vel[:, 2]),
        m=f32(np.full(n, m)), u=f32(u), h=f32(h), alpha_v=f32(av), alpha_c=f32(ac),
        active=active, box=tuple(float(b) for b in box), name=name, meta=meta)


def lattice_positions(n_side: int, rng: np.random.Generator, jitter: float = 0.1,
                      box: float = 1.0) -> np.ndarray:
    """Cubic lattice with points at cell centres, each coordinate jittered by
    U(-jitter*d, +jitter*d) with d the lattice spacing."""
    d = box / n_side
    g = (np.arange(n_side) + 0.5) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if jitter:
        pos = pos + rng.uniform(-jitter * d, jitter * d, size=pos.shape)
    return np.mod(pos, box)


def lattice_box(n_side: int, seed: int, *, jitter: float = 0.1, u="const", sigma_v: float = 0.01,
                eta: float = ETA, name: str = "lattice", alpha: bool = True) -> ParticleSet:
    """Jittered lattice in the unit box, equal masses 1/N, h = eta * spacing.

    ``u``: ``"const"`` gives u = 1, ``"logu"`` gives u = 10^U(-1, 1).
    """
    rng = np.random.default_rng(seed)
    pos = lattice_positions(n_side, rng, jitter)
    n = pos.shape[0]
    vel = rng.normal(0.0, sigma_v, size=(n, 3)) if sigma_v > 0 else np.zeros((n, 3))
    uu = 10.0 ** rng.uniform(-1.0, 1.0, n) if u == "logu" else 1.0
    h = eta / n_side
    return _finish(pos, vel, 1.0 / n, uu, h, rng, (1.0,) * 3, name,
                   {"n_side": n_side, "seed": seed, "jitter": jitter}, alpha=alpha)


def sedov_box(n_side: int = 64, seed: int = 2, *, n_hot: int = 32, eta: float = ETA) -> ParticleSet:
    """Sedov blast set-up: jittered lattice at rest, u = 1e-6 everywhere except
    the ``n_hot`` particles nearest the box centre (minimum-image distance, ties
    by index), which share one unit of energy: u = 1 / (n_hot * m)."""
    rng = np.random.default_rng(seed)
    pos = lattice_positions(n_side, rng, 0.1)
    n = pos.shape[0]
    d = pos - 0.5
    d -= np.round(d)
    r2 = np.einsum("ij,ij->i", d, d)
    hot = np.lexsort((np.arange(n), r2))[:n_hot]
    m = 1.0 / n
    u = np.full(n, 1e-6)
    u[hot] = 1.0 / (n_hot * m)
    vel = np.zeros((n, 3))
    return _finish(pos, vel, m, u, eta / n_side, rng, (1.0,) * 3, "sedov",
                   {"n_side": n_side, "seed": seed, "n_hot": n_hot})


def gaussian_field(n_mesh: int, rng: np.random.Generator, slope: float = -2.0) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian random field on a periodic n_mesh^3
    mesh with power spectrum P(k) ~ k^slope (the k = 0 mode removed)."""
    g = rng.standard_normal((n_mesh,) * 3)
    gk = np.fft.rfftn(g)
    k1 = np.fft.fftfreq(n_mesh) * n_mesh
    kz = np.fft.rfftfreq(n_mesh) * n_mesh
    k2 = k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)  # sqrt(P(k)) = k^(slope/2)
    g = np.fft.irfftn(gk * amp, s=(n_mesh,) * 3, axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_positions(n_mesh: int, n_part: int, sigma: float, rng: np.random.Generator):
    """Positions drawn from rho ~ exp(sigma*g - sigma^2/2): multinomial counts
    per mesh cell, uniform inside each cell. Returns (pos, count_of_own_cell)."""
    g = gaussian_field(n_mesh, rng)
    rho = np.exp(sigma * g - 0.5 * sigma * sigma).ravel()
    p = rho / rho.sum()
    counts = rng.multinomial(n_part, p)
    cell = np.repeat(np.arange(n_mesh ** 3, dtype=np.int64), counts)
    iz = cell % n_mesh
    iy = (cell // n_mesh) % n_mesh
    ix = cell // (n_mesh * n_mesh)
    ijk = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    pos = (ijk + rng.uniform(0.0, 1.0, size=ijk.shape)) / n_mesh
    pos = np.mod(pos, 1.0)
    return pos, counts[cell]


def lognormal_box(n_mesh: int, n_part: int, sigma: float, seed: int, *, eta: float = ETA,
                  sigma_v: float = 0.01, name: str = "lognormal", time_bins=None) -> ParticleSet:
    """Clustered box: lognormal density field (Gaussian field with P(k) ~ k^-2),
    u = 10^U(-1, 1), v ~ N(0, sigma_v), equal masses 1/N.

    The smoothing-length guess is eta * (mesh-cell volume / its count)^(1/3),
    floored at a quarter mesh spacing and capped at box/6.

    ``time_bins``: optional probabilities of time bins 0, 1, 2, ...; a particle
    is active when its bin is 0 (an odd step of the power-of-two timeline of
    the paper's Section 2.4 activates only the shortest bin).
    """
    rng = np.random.default_rng(seed)
    pos, cnt = lognormal_positions(n_mesh, n_part, sigma, rng)
    n = pos.shape[0]
    dm = 1.0 / n_mesh
    h = eta * dm * np.power(cnt.astype(np.float64), -1.0 / 3.0)
    h = np.clip(h, 0.25 * dm, 1.0 / 6.0)
    u = 10.0 ** rng.uniform(-1.0, 1.0, n)
    vel = rng.normal(0.0, sigma_v, size=(n, 3))
    active = None
    if time_bins is not None:
        bins = rng.choice(len(time_bins), size=n, p=np.asarray(time_bins, dtype=np.float64))
        active = bins == 0
    return _finish(pos, vel, 1.0 / n, u, h, rng, (1.0,) * 3, name,
                   {"n_mesh": n_mesh, "sigma": sigma, "seed": seed}, active=active)


def uniform_random_box(n: int, seed: int, *, eta: float = ETA, sigma_v: float = 0.01,
                       u="logu", name: str = "poisson") -> ParticleSet:
    """Poisson (uniform random) positions: a ragged, unstructured case."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(n, 3))
    vel = rng.normal(0.0, sigma_v, size=(n, 3))
    uu = 10.0 ** rng.uniform(-1.0, 1.0, n) if u == "logu" else 1.0
    h = eta * n ** (-1.0 / 3.0)
    return _finish(pos, vel, 1.0 / n, uu, h, rng, (1.0,) * 3, name, {"seed": seed})


# ---------------------------------------------------------------------------
# The five named workloads.
# ---------------------------------------------------------------------------

def config_small(seed: int = 1, u: str = "const") -> ParticleSet:
    """4,096 particles: 16^3 lattice jittered by 0.1 spacing, u = 1 (or
    log-uniform), v ~ N(0, 0.01)."""
    return lattice_box(16, seed, u=u, name="lattice16")


def config_sedov(seed: int = 2, n_side: int = 64) -> ParticleSet:
    """Sedov blast: 64^3 = 262,144 particles."""
    return sedov_box(n_side, seed)


def config_clustered(seed: int = 3, n_mesh: int = 128) -> ParticleSet:
    """Clustered box: 128^3 = 2,097,152 particles, sigma_ln(rho) = 2."""
    return lognormal_box(n_mesh, n_mesh ** 3, 2.0, seed, name="clustered%d" % n_mesh)


def config_large(seed: int = 5, n_mesh: int = 256) -> ParticleSet:
    """Large clustered box: 256^3 particles, sigma = 2.5, ~10% active."""
    return lognormal_box(n_mesh, n_mesh ** 3, 2.5, seed, name="large%d" % n_mesh,
                         time_bins=(0.1, 0.2, 0.3, 0.4))


@dataclass
class Request:
    rid: int
    arrival: float
    particles: ParticleSet


def serving_sizes(n_req: int = 512, seed: int = 4, lo: float = 3.0, hi: float = 6.0):
    rng = np.random.default_rng(seed)
    sizes = np.round(10.0 ** rng.uniform(lo, hi, n_req)).astype(np.int64)
    lattice = rng.uniform(size=n_req) < 0.5
    return sizes, lattice


def serving_request(k: int, size: int, lattice: bool, seed: int = 4) -> ParticleSet:
    """Request k of the serving stream: a jittered lattice with n = round(N^(1/3))
    per side, or a lognormal box on an n^3 mesh with sigma = 2."""
    s = seed * 1_000_003 + k
    ns = max(4, int(round(size ** (1.0 / 3.0))))
    if lattice:
        return lattice_box(ns, s, u="logu", name="req%d-lattice" % k)
    return lognormal_box(ns, int(size), 2.0, s, name="req%d-lognormal" % k)


def serving_stream(rate: float, n_req: int = 512, seed: int = 4, lo: float = 3.0,
                   hi: float = 6.0) -> Iterator[Request]:
    """Poisson arrivals at ``rate`` requests/s; sizes log-uniform in [10^lo, 10^hi]."""
    sizes, lattice = serving_sizes(n_req, seed, lo, hi)
    rng = np.random.default_rng(seed + 7919)
    t = 0.0
    for k in range(n_req):
        t += rng.exponential(1.0 / rate)
        yield Request(k, t, serving_request(k, int(sizes[k]), bool(lattice[k]), seed))
