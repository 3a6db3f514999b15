"""Seeded synthetic particle sets (shared by the tests, the oracle runs and the benchmark).

This module holds no part of the tree method: it only draws positions, velocities,
masses and softenings.  The paper's own initial conditions (a Milky-Way model built with
an external generator, section "Disk galaxy simulation") are not available, so Plummer
spheres, a clustered Plummer system and ensembles of Plummer spheres stand in for them.

Plummer sampling follows Aarseth, Henon & Wielen (1974): radius from the inverted
cumulative mass profile, speed from the isotropic distribution function by rejection.
Units G = 1.  Every generator is a pure function of its seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ParticleSet:
    """Structure-of-arrays particle set in FP64, optionally split into independent systems."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray
    eps: np.ndarray
    sys_off: np.ndarray = field(default=None)  # int64 [S+1]; None = one system

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_sys(self) -> int:
        return 1 if self.sys_off is None else int(self.sys_off.shape[0] - 1)

    def offsets(self) -> np.ndarray:
        if self.sys_off is None:
            return np.array([0, self.n], dtype=np.int64)
        return self.sys_off

    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def vel(self) -> np.ndarray:
        return np.stack([self.vx, self.vy, self.vz], axis=1)


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)


def _plummer_radii(rng: np.random.Generator, n: int, rmax: float) -> np.ndarray:
    """Radii of a unit Plummer sphere (a = 1) from M(<r) = r^3/(1+r^2)^{3/2}, redrawn above rmax."""
    out = np.empty(n)
    filled = 0
    while filled < n:
        k = n - filled
        u = rng.uniform(0.0, 1.0, k)
        u = u[u > 0.0]
        r = 1.0 / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        r = r[np.isfinite(r) & (r <= rmax)]
        take = min(r.shape[0], n - filled)
        out[filled:filled + take] = r[:take]
        filled += take
    return out


def _plummer_speed_fraction(rng: np.random.Generator, n: int) -> np.ndarray:
    """q = v / v_esc drawn from g(q) = q^2 (1 - q^2)^{7/2} by rejection under the bound 0.1."""
    out = np.empty(n)
    filled = 0
    while filled < n:
        k = 2 * (n - filled) + 64
        q = rng.uniform(0.0, 1.0, k)
        y = rng.uniform(0.0, 0.1, k)
        ok = q[y < q * q * (1.0 - q * q) ** 3.5]
        take = min(ok.shape[0], n - filled)
        out[filled:filled + take] = ok[:take]
        filled += take
    return out


def plummer_raw(rng: np.random.Generator, n: int, a: float = 1.0, mass: float = 1.0,
                rtrunc: float = 20.0):
    """Positions and velocities of an n-particle Plummer sphere (scale a, total mass `mass`,
    radii truncated at rtrunc * a), not yet shifted to the centre-of-mass frame."""
    r = _plummer_radii(rng, n, rtrunc) * a
    pos = _isotropic(rng, n) * r[:, None]
    q = _plummer_speed_fraction(rng, n)
    # escape speed of the Plummer potential -G M / sqrt(r^2 + a^2)
    vesc = np.sqrt(2.0 * mass) * (r * r + a * a) ** (-0.25)
    vel = _isotropic(rng, n) * (q * vesc)[:, None]
    return pos, vel


def _com_shift(pos, vel, m):
    mt = m.sum()
    pos -= (m[:, None] * pos).sum(axis=0) / mt
    vel -= (m[:, None] * vel).sum(axis=0) / mt


def _pack(pos, vel, m, eps, sys_off=None) -> ParticleSet:
    c = np.ascontiguousarray
    return ParticleSet(c(pos[:, 0]), c(pos[:, 1]), c(pos[:, 2]),
                       c(vel[:, 0]), c(vel[:, 1]), c(vel[:, 2]),
                       c(m), c(eps), sys_off)


def plummer(n: int, seed: int, eps: float, a: float = 1.0, mass: float = 1.0,
            rtrunc: float = 20.0) -> ParticleSet:
    """Equal-mass Plummer sphere in its centre-of-mass frame, uniform softening eps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, vel = plummer_raw(rng, n, a, mass, rtrunc)
    m = np.full(n, mass / n)
    _com_shift(pos, vel, m)
    return _pack(pos, vel, m, np.full(n, float(eps)))


def clustered(n_background: int = 1 << 23, n_clusters: int = 64, n_per_cluster: int = 1 << 17,
              seed: int = 3, eps: float = 1e-3, a_bg: float = 1.0, a_cl: float = 0.02,
              rtrunc: float = 20.0) -> ParticleSet:
    """Plummer background (scale a_bg, half the mass) with n_clusters embedded Plummer
    sub-clusters (scale a_cl, equal shares of the other half) whose centres are uniform in
    the unit sphere; all particles have equal mass and the system has total mass 1.
    Sub-clusters carry no bulk velocity; the whole set is shifted to its centre-of-mass frame."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = n_background + n_clusters * n_per_cluster
    m_bg = 0.5
    m_cl = 0.5 / n_clusters
    pos = np.empty((n, 3))
    vel = np.empty((n, 3))
    p, v = plummer_raw(rng, n_background, a_bg, m_bg, rtrunc)
    pos[:n_background] = p
    vel[:n_background] = v
    # centres uniform in the unit ball
    cu = rng.uniform(0.0, 1.0, n_clusters) ** (1.0 / 3.0)
    centres = _isotropic(rng, n_clusters) * cu[:, None]
    off = n_background
    for k in range(n_clusters):
        p, v = plummer_raw(rng, n_per_cluster, a_cl, m_cl, rtrunc)
        pos[off:off + n_per_cluster] = p + centres[k]
        vel[off:off + n_per_cluster] = v
        off += n_per_cluster
    m = np.full(n, 1.0 / n)
    _com_shift(pos, vel, m)
    return _pack(pos, vel, m, np.full(n, float(eps)))


def ensemble(n_sys: int = 512, seed: int = 4, nmin: int = 1024, nmax: int = 65536,
             rtrunc: float = 20.0) -> ParticleSet:
    """n_sys independent unit Plummer spheres (G = M = a = 1) laid end to end in one SoA set.
    System s draws its size log-uniformly in [nmin, nmax] from the ensemble seed and its
    particles from its own stream (seed + s); softening eps_s = 4 / N_s^{1/3}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_sys))).astype(np.int64)
    sys_off = np.zeros(n_sys + 1, dtype=np.int64)
    sys_off[1:] = np.cumsum(sizes)
    n = int(sys_off[-1])
    pos = np.empty((n, 3))
    vel = np.empty((n, 3))
    m = np.empty(n)
    eps = np.empty(n)
    for s in range(n_sys):
        ns = int(sizes[s])
        r = np.random.Generator(np.random.PCG64(seed + s))
        p, v = plummer_raw(r, ns, 1.0, 1.0, rtrunc)
        ms = np.full(ns, 1.0 / ns)
        _com_shift(p, v, ms)
        a, b = sys_off[s], sys_off[s + 1]
        pos[a:b] = p
        vel[a:b] = v
        m[a:b] = ms
        eps[a:b] = 4.0 / ns ** (1.0 / 3.0)
    return _pack(pos, vel, m, eps, sys_off)


def concat(sets) -> ParticleSet:
    """Lay several particle sets end to end as independent systems."""
    sizes = [s.n for s in sets]
    sys_off = np.zeros(len(sets) + 1, dtype=np.int64)
    sys_off[1:] = np.cumsum(sizes)
    cat = lambda name: np.ascontiguousarray(np.concatenate([getattr(s, name) for s in sets]))
    return ParticleSet(cat("x"), cat("y"), cat("z"), cat("vx"), cat("vy"), cat("vz"),
                       cat("m"), cat("eps"), sys_off)


def uniform_cube(n: int, seed: int, eps: float, side: float = 1.0) -> ParticleSet:
    """Uniform random points in a cube, at rest (small tests and edge cases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.uniform(-0.5 * side, 0.5 * side, (n, 3))
    vel = np.zeros((n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    return _pack(pos, vel, m, np.full(n, float(eps)))


def multisection(ps: ParticleSet, nx: int, ny: int, nz: int):
    """The particles of a one-system set regrouped into nx * ny * nz domains laid end to end
    as systems: equal-count slabs along x, each slab cut into equal-count columns along y,
    each column into equal-count blocks along z (stable order, ties by index).  An input
    layout for exchange-list tests and benchmarks (the domains stand in for processes); the
    paper's sampling-based decomposition is not this.  Returns (domain set, order), order[k]
    = the original index of the k-th particle of the domain set."""
    if ps.n_sys != 1:
        raise ValueError("multisection takes a one-system set")
    n = ps.n
    order = np.argsort(ps.x, kind="stable")
    pieces = []
    for sx in np.array_split(order, nx):
        sx = sx[np.argsort(ps.y[sx], kind="stable")]
        for sy in np.array_split(sx, ny):
            sy = sy[np.argsort(ps.z[sy], kind="stable")]
            pieces.extend(np.array_split(sy, nz))
    order = np.concatenate(pieces).astype(np.int64)
    sys_off = np.zeros(len(pieces) + 1, dtype=np.int64)
    sys_off[1:] = np.cumsum([len(p) for p in pieces])
    take = lambda a: np.ascontiguousarray(a[order])
    dom = ParticleSet(take(ps.x), take(ps.y), take(ps.z), take(ps.vx), take(ps.vy), take(ps.vz),
                      take(ps.m), take(ps.eps), sys_off)
    assert sys_off[-1] == n
    return dom, order


def subset(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct particle indices out of n, ascending (error-measurement subsets)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if k >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


# Workloads of the benchmark configurations, named by what they are.
def workload(name: str) -> ParticleSet:
    if name == "plummer4k":          # N = 4096, eps = 1/64, seed 1
        return plummer(4096, seed=1, eps=1.0 / 64.0)
    if name == "plummer1m":          # N = 2^20, eps = 1/256, seed 2
        return plummer(1 << 20, seed=2, eps=1.0 / 256.0)
    if name == "clustered16m":       # N = 2^24 clustered, eps = 1e-3, seed 3
        return clustered(seed=3)
    if name == "ensemble512":        # 512 Plummer spheres, N_s log-uniform in [1024, 65536]
        return ensemble(seed=4)
    raise KeyError(name)
