"""FP64 CPU oracle for the Barnes-Hut gravity hot path (Iwasawa et al., FDPS).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline
leg may import this package; the GPU library never does, and nothing in the product path
may fall back to it.  It shares no code with the GPU library.

Two parts:
  O-D  `direct`      softened FP64 direct summation (equation ParticleParticleNbody, G = 1),
                     the exact quantity the tree approximates;
  O-T  `build_tree`, `make_groups`, `walk`, `tree_force`
                     a plain serial tree that fixes keys, order, cells, groups and lists
                     (the readings are documented in oracle.c next to each step).
Plus the multisection domain decomposition with cost-weighted sampling (`decompose`,
section "Domain decomposition"), the exchange lists between domains (`exchange`, section "Exchange of particles and
superparticles") with the force from received lists (`list_force`), the leapfrog of the
sample program (`kdk`), energy and error diagnostics, and the list-length models (equations
nlist_long and n_list_long).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _LIB = C.CDLL(_build.LIB)
        _declare(_LIB)
    return _LIB


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _declare(L):
    vp, i64, i32, f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.or_direct.argtypes = [i64, i64, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp]
    L.or_set_threads.argtypes = [C.c_int]
    L.or_set_threads.restype = C.c_int
    L.or_keys.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    L.or_interleave.argtypes = [C.c_uint32] * 3
    L.or_interleave.restype = C.c_uint64
    L.or_deinterleave.argtypes = [i64, vp, vp]
    L.or_sort.argtypes = [i64, vp, vp, vp]
    L.or_build_cells.argtypes = [i64, vp, vp, i32]
    L.or_build_cells.restype = vp
    L.or_cells_count.argtypes = [vp]
    L.or_cells_count.restype = i64
    L.or_cells_system.argtypes = [vp, i64, vp]
    L.or_cells_export.argtypes = [vp] + [vp] * 7
    L.or_cells_free.argtypes = [vp]
    L.or_moments.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
    L.or_groups.argtypes = [vp, i64, i32]
    L.or_groups.restype = vp
    L.or_groups_count.argtypes = [vp]
    L.or_groups_count.restype = i64
    L.or_groups_export.argtypes = [vp, vp, vp, vp]
    L.or_groups_free.argtypes = [vp]
    L.or_group_geometry.argtypes = [i64] + [vp] * 11
    L.or_walk.argtypes = [vp, i64, vp, vp, vp, vp, f64, vp]
    L.or_walk.restype = vp
    L.or_walk_export.argtypes = [vp, vp, vp]
    L.or_walk_free.argtypes = [vp]
    L.or_force.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp]
    L.or_exchange.argtypes = [vp, i64, vp, vp, vp, f64, vp]
    L.or_exchange.restype = vp
    L.or_wendland_c6.argtypes = [f64, f64]
    L.or_wendland_c6.restype = f64
    L.or_density_brute.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, f64, vp, vp]
    L.or_cell_hmax.argtypes = [vp, vp, vp]
    L.or_short_walk.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, vp, vp]
    L.or_short_walk.restype = vp
    L.or_density_lists.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i32, f64, vp, vp]
    L.or_s2_cutoff.argtypes = [f64]
    L.or_s2_cutoff.restype = f64
    L.or_direct_cutoff.argtypes = [i64, vp, vp, vp, vp, vp, vp, f64, vp]
    L.or_walk_cutoff.argtypes = [vp, i64, vp, vp, vp, f64, f64, vp, vp]
    L.or_walk_cutoff.restype = vp
    L.or_force_cutoff.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, f64, vp]
    L.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.or_splitmix64.restype = C.c_uint64
    L.or_dd_sample.argtypes = [i64, vp, vp, C.c_uint64, vp]
    L.or_dd_multisection.argtypes = [i64, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
    L.or_dd_multisection.restype = i32
    L.or_dd_assign.argtypes = [i64, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ----------------------------------------------------------------------------------------
# O-D
def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops from now on; returns the previous maximum."""
    return int(lib().or_set_threads(int(n)))


def direct(ps, targets=None) -> np.ndarray:
    """Direct-sum {ax, ay, az, phi} on the target particles (user indices), each against the
    particles of its own system only.  Returns an array [len(targets), 4]."""
    L = lib()
    off = ps.offsets()
    if targets is None:
        targets = np.arange(ps.n, dtype=np.int64)
    targets = _c(targets, np.int64)
    out = np.zeros((targets.shape[0], 4))
    sys_of = np.searchsorted(off, targets, side="right") - 1
    x, y, z, m, e = (_c(getattr(ps, k), np.float64) for k in ("x", "y", "z", "m", "eps"))
    for s in np.unique(sys_of):
        sel = np.nonzero(sys_of == s)[0]
        t = _c(targets[sel], np.int64)
        ax, ay, az, pot = (np.zeros(t.shape[0]) for _ in range(4))
        L.or_direct(int(off[s]), int(off[s + 1]), _p(x), _p(y), _p(z), _p(m), _p(e),
                    t.shape[0], _p(t), _p(ax), _p(ay), _p(az), _p(pot))
        out[sel, 0], out[sel, 1], out[sel, 2], out[sel, 3] = ax, ay, az, pot
    return out


# ----------------------------------------------------------------------------------------
# O-T
def interleave(qx: int, qy: int, qz: int) -> int:
    return int(lib().or_interleave(qx, qy, qz))


def deinterleave(keys: np.ndarray) -> np.ndarray:
    keys = _c(keys, np.uint64)
    q = np.zeros((keys.shape[0], 3), dtype=np.uint32)
    lib().or_deinterleave(keys.shape[0], _p(keys), _p(q))
    return q


def keys(ps):
    """Root cube {ox, oy, oz, Lr} per system and the 63-bit key of every particle."""
    off = _c(ps.offsets(), np.int64)
    S = off.shape[0] - 1
    cube = np.zeros((S, 4))
    key = np.zeros(ps.n, dtype=np.uint64)
    x, y, z = (_c(getattr(ps, k), np.float64) for k in ("x", "y", "z"))
    lib().or_keys(S, _p(off), _p(x), _p(y), _p(z), _p(cube), _p(key))
    return cube, key


def sort(ps, key) -> np.ndarray:
    off = _c(ps.offsets(), np.int64)
    perm = np.zeros(ps.n, dtype=np.uint32)
    key = _c(key, np.uint64)
    lib().or_sort(off.shape[0] - 1, _p(off), _p(key), _p(perm))
    return perm


class Tree:
    """Keys, order, cells and moments of one particle set (all systems)."""

    def __init__(self, ps, n_leaf: int = 8, moments: bool = True):
        L = lib()
        self.ps = ps
        self.n_leaf = n_leaf
        self.off = _c(ps.offsets(), np.int64)
        self.n_sys = self.off.shape[0] - 1
        self.cube, self.key = keys(ps)
        self.perm = sort(ps, self.key)
        p = self.perm.astype(np.int64)
        self.skey = _c(self.key[p], np.uint64)
        self.sx, self.sy, self.sz, self.sm, self.seps = (
            _c(getattr(ps, k)[p], np.float64) for k in ("x", "y", "z", "m", "eps"))
        h = L.or_build_cells(self.n_sys, _p(self.off), _p(self.skey), n_leaf)
        try:
            nc = L.or_cells_count(h)
            self.level = np.zeros(nc, np.int32)
            self.prefix = np.zeros(nc, np.uint64)
            self.begin, self.count, self.first_child, self.nchild, self.parent, self.csys = (
                np.zeros(nc, np.uint32) for _ in range(6))
            L.or_cells_export(h, _p(self.level), _p(self.prefix), _p(self.begin),
                              _p(self.count), _p(self.first_child), _p(self.nchild),
                              _p(self.parent))
            L.or_cells_system(h, self.n_sys, _p(self.csys))
            self._h = h
        except Exception:
            L.or_cells_free(h)
            raise
        self.mom = None
        if moments:
            self.compute_moments()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_cells_free(h)
            self._h = None

    @property
    def n_cells(self) -> int:
        return int(self.level.shape[0])

    def compute_moments(self):
        self.mom = np.zeros((self.n_cells, 10))
        lib().or_moments(self.n_cells, _p(self.begin), _p(self.count), _p(self.sx),
                         _p(self.sy), _p(self.sz), _p(self.sm), _p(self.mom))
        return self.mom


def build_tree(ps, n_leaf: int = 8, moments: bool = True) -> Tree:
    return Tree(ps, n_leaf, moments)


class Groups:
    def __init__(self, tree: Tree, n_group: int):
        L = lib()
        self.n_group = n_group
        h = L.or_groups(tree._h, tree.n_sys, n_group)
        ng = L.or_groups_count(h)
        self.cell, self.begin, self.count = (np.zeros(ng, np.uint32) for _ in range(3))
        L.or_groups_export(h, _p(self.cell), _p(self.begin), _p(self.count))
        L.or_groups_free(h)
        self.qmin = np.zeros((ng, 3), np.uint32)
        self.qmax = np.zeros((ng, 3), np.uint32)
        self.centre = np.zeros((ng, 3))
        L.or_group_geometry(ng, _p(self.cell), _p(self.begin), _p(self.count), _p(tree.level),
                            _p(tree.prefix), _p(tree.skey), _p(tree.csys), _p(tree.cube),
                            _p(self.qmin), _p(self.qmax), _p(self.centre))
        self.root = _c(tree.csys[self.cell], np.uint32)   # roots are cells 0..S-1

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])


def make_groups(tree: Tree, n_group: int) -> Groups:
    return Groups(tree, n_group)


def group_features(tree: Tree, grp: Groups) -> np.ndarray:
    """The eight per-group inputs of the list-length network, [G, 8] in FP64.  The paper models
    only the mean list length (equation nlist_long, from the group size, the opening angle and
    the particle count); these are cheap per-group stand-ins for its terms.  With the group's
    integer box [qmin, qmax] (grid units, 2^21 per root side), its cell c at level l_c and
    p = the parent of c (c itself for a root) at level l_p:
      0 ln n_i                               1 ln(1 + max_a (qmax_a - qmin_a))
      2 ln(1 + |box centre - root centre|),  box centre (qmin + qmax + 1) / 2, root centre 2^20
      3 ln(M_p / M_system)                   4 ln(side_p / side_root) = -l_p ln 2
      5 l_c                                  6 ln(count_p / (side_p / side_root)^3)
      7 log2 N_system"""
    if tree.mom is None:
        tree.compute_moments()
    G = grp.n
    X = np.zeros((G, 8))
    off = tree.off
    for g in range(G):
        c = int(grp.cell[g])
        p = int(tree.parent[c])
        if p == 0xFFFFFFFF:
            p = c
        s = int(tree.csys[c])
        lo = grp.qmin[g].astype(np.float64)
        hi = grp.qmax[g].astype(np.float64)
        centre = 0.5 * (lo + hi + 1.0) - 2.0 ** 20
        lp = int(tree.level[p])
        X[g, 0] = math.log(int(grp.count[g]))
        X[g, 1] = math.log(1.0 + float(np.max(hi - lo)))
        X[g, 2] = math.log(1.0 + math.sqrt(float(centre @ centre)))
        X[g, 3] = math.log(tree.mom[p, 0] / tree.mom[s, 0])
        X[g, 4] = -lp * math.log(2.0)
        X[g, 5] = float(tree.level[c])
        X[g, 6] = math.log(int(tree.count[p])) + 3.0 * lp * math.log(2.0)
        X[g, 7] = math.log2(int(off[s + 1] - off[s]))
    return X


class Lists:
    """Interaction lists of selected groups, CSR: EPJ (sorted particle positions) and SPJ
    (cell ids), each in depth-first walk order."""

    def __init__(self, tree: Tree, grp: Groups, theta: float, sel=None):
        L = lib()
        self.tree, self.grp = tree, grp
        self.sel = _c(np.arange(grp.n) if sel is None else sel, np.int64)
        k = self.sel.shape[0]
        counts = np.zeros(2 * k, np.int64)
        self._h = L.or_walk(tree._h, k, _p(self.sel), _p(grp.root), _p(grp.qmin),
                            _p(grp.qmax), float(theta), _p(counts))
        self.n_epj = counts[0::2].copy()
        self.n_spj = counts[1::2].copy()
        self.epj_off = np.concatenate([[0], np.cumsum(self.n_epj)]).astype(np.int64)
        self.spj_off = np.concatenate([[0], np.cumsum(self.n_spj)]).astype(np.int64)
        self.epj = np.zeros(int(self.epj_off[-1]), np.uint32)
        self.spj = np.zeros(int(self.spj_off[-1]), np.uint32)
        L.or_walk_export(self._h, _p(self.epj), _p(self.spj))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_walk_free(h)
            self._h = None

    def group_lists(self, k: int):
        return (self.epj[self.epj_off[k]:self.epj_off[k + 1]],
                self.spj[self.spj_off[k]:self.spj_off[k + 1]])

    def force(self, quad: bool) -> np.ndarray:
        """{ax, ay, az, phi} at every sorted position covered by the selected groups
        (rows of unselected groups stay NaN)."""
        t, g = self.tree, self.grp
        if t.mom is None:
            t.compute_moments()
        acc = np.full((t.ps.n, 4), np.nan)
        lib().or_force(self._h, _p(self.sel), _p(g.begin), _p(g.count), _p(t.sx), _p(t.sy),
                       _p(t.sz), _p(t.sm), _p(t.seps), _p(t.mom), 1 if quad else 0, _p(acc))
        return acc


def walk(tree: Tree, grp: Groups, theta: float, sel=None) -> Lists:
    return Lists(tree, grp, theta, sel)


def tree_force(ps, theta: float, n_leaf: int = 8, n_group: int = 64, quad: bool = True):
    """Whole O-T evaluation; returns {ax, ay, az, phi} in the user's original order."""
    t = build_tree(ps, n_leaf)
    g = make_groups(t, n_group)
    lists = walk(t, g, theta)
    acc_sorted = lists.force(quad)
    acc = np.empty_like(acc_sorted)
    acc[t.perm.astype(np.int64)] = acc_sorted
    return acc


# ----------------------------------------------------------------------------------------
# Leapfrog (predict = half kick + drift, correct = half kick, as in the sample program),
# energy and error diagnostics.
def kick(v: np.ndarray, a: np.ndarray, dt: float):
    v += (0.5 * dt) * a


def drift(x: np.ndarray, v: np.ndarray, dt: float):
    x += dt * v


def energy(ps, pot: np.ndarray):
    """Kinetic, potential (1/2 sum m phi, per-particle phi from `pot`) and total."""
    K = 0.5 * float(np.sum(ps.m * (ps.vx ** 2 + ps.vy ** 2 + ps.vz ** 2)))
    W = 0.5 * float(np.sum(ps.m * pot))
    return K, W, K + W


class ExchangeLists:
    """Exchange lists between the domains of a particle set (each system is one domain with
    its own local tree; section "Exchange of particles and superparticles", long-range
    mode): for every ordered pair (sender s, receiver r != s), pairs ordered by sender then
    receiver, the sender's particles (EPJ, sorted positions) and cells (SPJ, cell ids)
    that r needs.  The reading is documented at or_exchange in oracle.c."""

    def __init__(self, tree: Tree, theta: float):
        L = lib()
        self.tree, self.theta = tree, theta
        ns = tree.n_sys
        off, ps = tree.off, tree.ps
        if ns < 2 or np.any(np.diff(off) == 0):
            raise ValueError("exchange lists need at least two non-empty domains")
        blo = np.zeros((ns, 3))
        bhi = np.zeros((ns, 3))
        for s in range(ns):
            sl = slice(off[s], off[s + 1])
            for a, k in enumerate(("x", "y", "z")):
                v = getattr(ps, k)[sl]
                blo[s, a], bhi[s, a] = v.min(), v.max()
        self.blo, self.bhi = blo, bhi
        self.pairs = [(s, r) for s in range(ns) for r in range(ns) if r != s]
        k = len(self.pairs)
        counts = np.zeros(2 * k, np.int64)
        self._h = L.or_exchange(tree._h, ns, _p(_c(tree.cube, np.float64)), _p(_c(blo, np.float64)),
                                _p(_c(bhi, np.float64)), float(theta), _p(counts))
        self.n_epj = counts[0::2].copy()
        self.n_spj = counts[1::2].copy()
        self.epj_off = np.concatenate([[0], np.cumsum(self.n_epj)]).astype(np.int64)
        self.spj_off = np.concatenate([[0], np.cumsum(self.n_spj)]).astype(np.int64)
        self.epj = np.zeros(int(self.epj_off[-1]), np.uint32)
        self.spj = np.zeros(int(self.spj_off[-1]), np.uint32)
        L.or_walk_export(self._h, _p(self.epj), _p(self.spj))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_walk_free(h)
            self._h = None

    def index(self, s: int, r: int) -> int:
        return self.pairs.index((s, r))

    def pair_lists(self, s: int, r: int):
        k = self.index(s, r)
        return (self.epj[self.epj_off[k]:self.epj_off[k + 1]],
                self.spj[self.spj_off[k]:self.spj_off[k + 1]])

    def received(self, r: int):
        """Everything domain r receives: (EPJ sorted positions, SPJ cell ids)."""
        es, ss = [], []
        for s in range(self.tree.n_sys):
            if s != r:
                e, c = self.pair_lists(s, r)
                es.append(e)
                ss.append(c)
        return np.concatenate(es), np.concatenate(ss)


def exchange(tree: Tree, theta: float) -> ExchangeLists:
    return ExchangeLists(tree, theta)


def list_force(x, y, z, eps, jx, jy, jz, jm, mom, quad: bool = True, self_mask=None):
    """{ax, ay, az, phi} on the targets (x, y, z, eps) from particles (jx, jy, jz, jm) and
    superparticles (rows of `mom`: M, X, Y, Z, Qxx, Qyy, Qzz, Qxy, Qxz, Qyz), FP64, with the
    particle term of equation ParticleParticleNbody and the quadrupole superparticle term
    (the Taylor expansion of 1/r about the centre of mass to second order, softened like
    equation ParticleSuperparticleNbody); pairs at zero separation contribute nothing (the
    self term)."""
    out = np.zeros((x.shape[0], 4))
    e2 = (eps * eps)[:, None]
    if jx.shape[0]:
        dx, dy, dz = jx[None, :] - x[:, None], jy[None, :] - y[:, None], jz[None, :] - z[:, None]
        d2 = dx * dx + dy * dy + dz * dz
        same = d2 == 0.0
        ri = 1.0 / np.sqrt(d2 + e2)
        mri = np.where(same, 0.0, jm[None, :] * ri)
        mri3 = mri * ri * ri
        out[:, 0] += np.sum(mri3 * dx, axis=1)
        out[:, 1] += np.sum(mri3 * dy, axis=1)
        out[:, 2] += np.sum(mri3 * dz, axis=1)
        out[:, 3] -= np.sum(mri, axis=1)
    if mom.shape[0]:
        M, X, Y, Z = (mom[:, k][None, :] for k in range(4))
        rx, ry, rz = x[:, None] - X, y[:, None] - Y, z[:, None] - Z
        R2 = rx * rx + ry * ry + rz * rz + e2
        Ri = 1.0 / np.sqrt(R2)
        Ri2, Ri3 = Ri * Ri, Ri * Ri * Ri
        ax, ay, az, ph = -M * Ri3 * rx, -M * Ri3 * ry, -M * Ri3 * rz, -M * Ri
        if quad:
            Qxx, Qyy, Qzz, Qxy, Qxz, Qyz = (mom[:, k][None, :] for k in range(4, 10))
            qx = Qxx * rx + Qxy * ry + Qxz * rz
            qy = Qxy * rx + Qyy * ry + Qyz * rz
            qz = Qxz * rx + Qyz * ry + Qzz * rz
            rqr = rx * qx + ry * qy + rz * qz
            Ri5 = Ri3 * Ri2
            ax = ax + Ri5 * qx - 2.5 * rqr * Ri5 * Ri2 * rx
            ay = ay + Ri5 * qy - 2.5 * rqr * Ri5 * Ri2 * ry
            az = az + Ri5 * qz - 2.5 * rqr * Ri5 * Ri2 * rz
            ph = ph - 0.5 * rqr * Ri5
        out[:, 0] += ax.sum(axis=1)
        out[:, 1] += ay.sum(axis=1)
        out[:, 2] += az.sum(axis=1)
        out[:, 3] += ph.sum(axis=1)
    return out


# ----------------------------------------------------------------------------------------
# Short-range neighbour lists and SPH density (readings at or_density_brute in oracle.c)

CUT_FIXED, CUT_SCATTER, CUT_GATHER, CUT_SYMMETRIC = 0, 1, 2, 3


def wendland_c6(r: float, H: float) -> float:
    return lib().or_wendland_c6(float(r), float(H))


def density_brute(ps, h, mode: int, r_cut: float = 0.0):
    """(rho, n_ngb) of every particle by all pairs of its system, caller's order."""
    rho = np.zeros(ps.n)
    n = np.zeros(ps.n, np.uint32)
    hh = None if h is None else _c(h, np.float64)
    lib().or_density_brute(ps.n_sys, _p(_c(ps.offsets(), np.int64)), _p(_c(ps.x, np.float64)),
                           _p(_c(ps.y, np.float64)), _p(_c(ps.z, np.float64)),
                           _p(_c(ps.m, np.float64)), None if hh is None else _p(hh), int(mode),
                           float(r_cut), _p(rho), _p(n))
    return rho, n


class ShortLists:
    """Candidate neighbour lists of every group (sorted particle positions) for one cutoff
    mode, and the density / neighbour count they give."""

    def __init__(self, tree: Tree, grp: Groups, h, mode: int, r_cut: float = 0.0):
        L = lib()
        self.tree, self.grp, self.mode, self.r_cut = tree, grp, int(mode), float(r_cut)
        self.sh = None if h is None else _c(np.asarray(h)[tree.perm.astype(np.int64)], np.float64)
        self.hmax = None
        if mode in (CUT_SCATTER, CUT_SYMMETRIC):
            self.hmax = np.zeros(tree.n_cells)
            L.or_cell_hmax(tree._h, _p(self.sh), _p(self.hmax))
        rg = np.full(grp.n, self.r_cut)
        if mode in (CUT_GATHER, CUT_SYMMETRIC):
            rg = np.array([self.sh[b:b + c].max() for b, c in zip(grp.begin, grp.count)])
        self.rg = _c(rg, np.float64)
        counts = np.zeros(grp.n, np.int64)
        self._h = L.or_short_walk(tree._h, grp.n, _p(grp.root), _p(grp.qmin), _p(grp.qmax),
                                  self.mode, _p(self.rg),
                                  None if self.hmax is None else _p(self.hmax),
                                  _p(_c(tree.cube, np.float64)), _p(counts))
        self.n_epj = counts
        self.epj_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        self.epj = np.zeros(int(self.epj_off[-1]), np.uint32)
        dummy = np.zeros(1, np.uint32)
        L.or_walk_export(self._h, _p(self.epj), _p(dummy))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_walk_free(h)
            self._h = None

    def group_list(self, k: int):
        return self.epj[self.epj_off[k]:self.epj_off[k + 1]]

    def density(self):
        """(rho, n_ngb) at sorted positions."""
        t, g = self.tree, self.grp
        rho = np.full(t.ps.n, np.nan)
        n = np.zeros(t.ps.n, np.uint32)
        lib().or_density_lists(self._h, _p(g.begin), _p(g.count), _p(t.sx), _p(t.sy), _p(t.sz),
                               _p(t.sm), None if self.sh is None else _p(self.sh), self.mode,
                               self.r_cut, _p(rho), _p(n))
        return rho, n


def short_lists(tree: Tree, grp: Groups, h, mode: int, r_cut: float = 0.0) -> ShortLists:
    return ShortLists(tree, grp, h, mode, r_cut)


def nlist_short_model(n_grp: float, r_cut: float, mean_spacing: float) -> float:
    """Short-range interaction-list length, equation nlist_short of section "Tree traverse
    and interaction calculation"."""
    return (n_grp ** (1.0 / 3.0) - 1.0 + 2.0 * r_cut / mean_spacing) ** 3


# ----------------------------------------------------------------------------------------
# Tree part of TreePM: monopole tree force with the S2 cutoff (readings at or_s2_cutoff)

def s2_cutoff(xi: float) -> float:
    return lib().or_s2_cutoff(float(xi))


def direct_cutoff(ps, r_cut: float) -> np.ndarray:
    """Acceleration of every particle (caller's order, n x 3) from all pairs of its system."""
    acc = np.zeros((ps.n, 3))
    lib().or_direct_cutoff(ps.n_sys, _p(_c(ps.offsets(), np.int64)), _p(_c(ps.x, np.float64)),
                           _p(_c(ps.y, np.float64)), _p(_c(ps.z, np.float64)),
                           _p(_c(ps.m, np.float64)), _p(_c(ps.eps, np.float64)), float(r_cut),
                           _p(acc))
    return acc


class CutoffLists:
    """Lists of every group for the cutoff walk (EPJ sorted positions, SPJ cell ids) and the
    monopole cutoff force they give."""

    def __init__(self, tree: Tree, grp: Groups, theta: float, r_cut: float):
        L = lib()
        self.tree, self.grp, self.r_cut = tree, grp, float(r_cut)
        counts = np.zeros(2 * grp.n, np.int64)
        self._h = L.or_walk_cutoff(tree._h, grp.n, _p(grp.root), _p(grp.qmin), _p(grp.qmax),
                                   float(theta), self.r_cut, _p(_c(tree.cube, np.float64)),
                                   _p(counts))
        self.n_epj = counts[0::2].copy()
        self.n_spj = counts[1::2].copy()
        self.epj_off = np.concatenate([[0], np.cumsum(self.n_epj)]).astype(np.int64)
        self.spj_off = np.concatenate([[0], np.cumsum(self.n_spj)]).astype(np.int64)
        self.epj = np.zeros(int(self.epj_off[-1]), np.uint32)
        self.spj = np.zeros(int(self.spj_off[-1]), np.uint32)
        L.or_walk_export(self._h, _p(self.epj), _p(self.spj))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_walk_free(h)
            self._h = None

    def group_lists(self, k: int):
        return (self.epj[self.epj_off[k]:self.epj_off[k + 1]],
                self.spj[self.spj_off[k]:self.spj_off[k + 1]])

    def force(self) -> np.ndarray:
        """Acceleration at sorted positions (n x 3)."""
        t, g = self.tree, self.grp
        if t.mom is None:
            t.compute_moments()
        acc = np.zeros((t.ps.n, 3))
        lib().or_force_cutoff(self._h, _p(g.begin), _p(g.count), _p(t.sx), _p(t.sy), _p(t.sz),
                              _p(t.sm), _p(t.seps), _p(t.mom), self.r_cut, _p(acc))
        return acc


def cutoff_lists(tree: Tree, grp: Groups, theta: float, r_cut: float) -> CutoffLists:
    return CutoffLists(tree, grp, theta, r_cut)


def exchange_list_model(n: float, theta: float, n_p: float) -> float:
    """Total exchange-list length of one domain of n particles among n_p cubic domains,
    equation n_list_long of section "Exchange of particles and superparticles"."""
    return (14.0 * n ** (2.0 / 3.0) / theta + 21.0 * math.pi * n ** (1.0 / 3.0) / theta ** 2
            + 28.0 * math.pi / (3.0 * theta ** 3)
            * math.log2(theta / 2.8 * ((n * n_p) ** (1.0 / 3.0) - n ** (1.0 / 3.0))))


# ----------------------------------------------------------------------------------------
# Domain decomposition (section "Domain decomposition"): multisection with sampling
def splitmix64(seed: int, ctr: int) -> int:
    """Output number ctr (0-based) of SplitMix64 seeded with seed."""
    return int(lib().or_splitmix64(seed & (2 ** 64 - 1), ctr))


def dd_factor(n: int):
    """(n_x, n_y, n_z) for n domains: integers close to n^(1/3) -- among the factorisations
    n_x >= n_y >= n_z, the one with the smallest n_x - n_z, then the smallest n_x - n_y."""
    best = None
    for nz in range(1, n + 1):
        if n % nz:
            continue
        for ny in range(nz, n // nz + 1):
            if (n // nz) % ny:
                continue
            nx = n // nz // ny
            if nx < ny:
                continue
            k = (nx - nz, nx - ny)
            if best is None or k < best[0]:
                best = (k, (nx, ny, nz))
    return best[1]


def dd_sample_counts(n_p, cost, n_sample: int) -> np.ndarray:
    """Samples drawn by each current domain: proportional to its cost, so that a sample
    stands for the same work everywhere (the sampling rate is the cost per particle).
    k_p = floor(n_sample * T_p / sum T) in FP64 (the sum taken in domain order), 0 for an
    empty domain; T_p = cost[p], or the particle count when cost is None."""
    n_p = [int(v) for v in n_p]
    T = [float(v) for v in (n_p if cost is None else cost)]
    total = 0.0
    for t in T:
        total += t
    return np.array([0 if n_p[p] == 0 else int(math.floor(float(n_sample) * T[p] / total))
                     for p in range(len(n_p))], dtype=np.int64)


def dd_sample(off, k, seed: int) -> np.ndarray:
    """Particle index of every sample (domains in order, k[p] samples each)."""
    off = _c(off, np.int64)
    k = _c(k, np.int64)
    idx = np.zeros(max(int(k.sum()), 1), np.uint32)
    lib().or_dd_sample(len(k), _p(off), _p(k), seed & (2 ** 64 - 1), _p(idx))
    return idx[:int(k.sum())]


def dd_multisection(sx, sy, sz, nx: int, ny: int, nz: int):
    """Faces (bx [nx+1], by [nx, ny+1], bz [nx, ny, nz+1]) and the domain of every sample."""
    K = len(sx)
    bx = np.zeros(nx + 1)
    by = np.zeros((nx, ny + 1))
    bz = np.zeros((nx, ny, nz + 1))
    cell = np.zeros(max(K, 1), np.uint32)
    r = lib().or_dd_multisection(K, _p(_c(sx, np.float64)), _p(_c(sy, np.float64)),
                                 _p(_c(sz, np.float64)), nx, ny, nz, _p(bx), _p(by), _p(bz),
                                 _p(cell))
    if r != 0:
        raise ValueError("fewer samples than domains")
    return bx, by, bz, cell[:K]


def dd_assign(x, y, z, nx: int, ny: int, nz: int, bx, by, bz) -> np.ndarray:
    """Destination domain of every particle."""
    n = len(x)
    dest = np.zeros(max(n, 1), np.uint32)
    lib().or_dd_assign(n, _p(_c(x, np.float64)), _p(_c(y, np.float64)), _p(_c(z, np.float64)),
                       nx, ny, nz, _p(_c(bx, np.float64)), _p(_c(by, np.float64)),
                       _p(_c(bz, np.float64)), _p(dest))
    return dest[:n]


def dd_exchange(dest, src, n_dom: int, n_src: int):
    """The exchange of particles: the new order (particles grouped by destination; within a
    destination by source domain, then by position, i.e. a stable grouping), the send
    counts [source, destination] and the offsets of the new domains."""
    dest = np.asarray(dest, np.int64)
    order = np.argsort(dest, kind="stable").astype(np.uint32)
    counts = np.zeros((n_src, n_dom), np.int64)
    np.add.at(counts, (np.asarray(src, np.int64), dest), 1)
    dom_off = np.concatenate([[0], np.cumsum(counts.sum(axis=0))]).astype(np.int64)
    return order, counts, dom_off


class Decomposition:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def decompose(ps, nx: int, ny: int, nz: int, n_sample: int, cost=None, seed: int = 0):
    """The whole decomposition of a particle set whose systems are the current domains:
    sample counts, samples, multisection, destinations and the exchange."""
    off = ps.offsets()
    n_p = np.diff(off)
    k = dd_sample_counts(n_p, cost, n_sample)
    idx = dd_sample(off, k, seed)
    bx, by, bz, cell = dd_multisection(ps.x[idx], ps.y[idx], ps.z[idx], nx, ny, nz)
    dest = dd_assign(ps.x, ps.y, ps.z, nx, ny, nz, bx, by, bz)
    src = np.repeat(np.arange(len(n_p)), n_p)
    order, counts, dom_off = dd_exchange(dest, src, nx * ny * nz, len(n_p))
    return Decomposition(k=k, idx=idx, bx=bx, by=by, bz=bz, cell=cell, dest=dest, order=order,
                         counts=counts, dom_off=dom_off)


def rms_rel_error(a: np.ndarray, a_ref: np.ndarray) -> float:
    """sqrt(mean_i |a_i - a_ref_i|^2 / |a_ref_i|^2) over the rows given (3 components)."""
    d = np.sum((a[:, :3] - a_ref[:, :3]) ** 2, axis=1)
    r = np.sum(a_ref[:, :3] ** 2, axis=1)
    return float(math.sqrt(np.mean(d / r)))


def nlist_model(n_grp: float, theta: float, n_total: float) -> float:
    """Mean interaction-list length of the long-range tree walk, equation nlist_long of
    section "Tree traverse and interaction calculation" (n n_p = total particle count)."""
    return (n_grp + 14.0 * n_grp ** (2.0 / 3.0) / theta
            + 21.0 * math.pi * n_grp ** (1.0 / 3.0) / theta ** 2
            + 28.0 * math.pi / (3.0 * theta ** 3)
            * math.log2(theta / 2.8 * (n_total ** (1.0 / 3.0) - n_grp ** (1.0 / 3.0))))
