"""Seeded random configurations of the short-range walk with the SPH density and of the TreePM
cutoff tree, against the oracle: distributions from smooth to coincident, one to three
systems, random n_leaf / n_group, all four cutoff modes with widely varying support radii,
random cutoff radii and opening angles.  Candidate and interaction lists bit-exact,
neighbour counts exact, densities to 1e-12; cutoff forces in FP64 against the oracle's on the
same lists to 1e-12 of each particle's Newtonian scale sum_j m_j / r_eff^2 (the cutoff can
leave a net force many orders below its terms, and evaluating the cutoff polynomial near
xi = 2 cancels, so a relative bound on the net force would measure round-off of zero)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1601_03138_amd import fdx as F
    c = F.Context(0)
    yield c
    c.close()


def _set(rng, seed):
    sets = []
    for s in range(int(rng.integers(1, 4))):
        n = int(rng.choice([1, int(rng.integers(2, 200)), int(rng.integers(200, 3000))]))
        kind = int(rng.integers(0, 4))
        if kind == 0:
            p = I.plummer(n, seed=seed * 10 + s, eps=0.01)
        elif kind == 1:
            p = I.uniform_cube(n, seed * 10 + s, 0.01)
        elif kind == 2:                         # coarse lattice: coincident particles
            q = rng.integers(-3, 4, size=(n, 3)).astype(np.float64) * 0.1
            p = I._pack(q, np.zeros((n, 3)), np.full(n, 1.0 / n), np.full(n, 0.01))
        else:                                   # two clumps far apart
            p = I.plummer(n, seed=seed * 10 + s, eps=0.01)
            p.x[n // 2:] += 100.0
        sets.append(p)
    return sets[0] if len(sets) == 1 else I.concat(sets)


@pytest.mark.parametrize("seed", range(12))
def test_random_sph_density(ctx, seed):
    rng = np.random.default_rng(2000 + seed)
    ps = _set(rng, seed)
    mode = int(rng.integers(0, 4))
    n_leaf = int(rng.choice([1, 4, 8, 32]))
    n_group = int(rng.choice([1, 16, 64, 300]))
    h = np.exp(rng.uniform(np.log(0.02), np.log(0.6), ps.n))
    r_cut = float(rng.uniform(0.03, 0.4))
    _say(f"[random sph {seed}] n={ps.n} sys={ps.n_sys} mode={mode} leaf={n_leaf} "
         f"group={n_group}")
    t = O.build_tree(ps, n_leaf, moments=False)
    g = O.make_groups(t, n_group)
    L = O.short_lists(t, g, h, mode, r_cut)
    rho_ref, n_ref = O.density_brute(ps, h, mode, r_cut)
    ctx.set_particles(ps)
    ctx.calc_density(mode, r_cut, h, n_leaf=n_leaf, n_group=n_group)
    ne, ns, epj, _ = ctx.lists()
    assert np.array_equal(ne.astype(np.int64), L.n_epj) and not ns.any()
    off = np.concatenate([[0], np.cumsum(ne.astype(np.int64))])
    for k in range(g.n):
        assert np.array_equal(np.sort(epj[off[k]:off[k + 1]]), np.sort(L.group_list(k)))
    rho, n = ctx.density()
    assert np.array_equal(n, n_ref)
    assert np.max(np.abs(rho - rho_ref) / rho_ref) <= 1e-12


def _newton_scale(t, g, L):
    """sum_j m_j / (r_ij^2 + eps_i^2) over each particle's lists (sorted order)."""
    pos = np.stack([t.sx, t.sy, t.sz], axis=1)
    out = np.zeros(pos.shape[0])
    for k in range(g.n):
        b, n = int(g.begin[k]), int(g.count[k])
        e, s = L.group_lists(k)
        xj = np.concatenate([pos[e.astype(np.int64)], t.mom[s.astype(np.int64), 1:4]])
        mj = np.concatenate([t.sm[e.astype(np.int64)], t.mom[s.astype(np.int64), 0]])
        d = xj[None, :, :] - pos[b:b + n, None, :]
        out[b:b + n] = np.sum(mj[None, :] / (np.sum(d * d, axis=2) + t.seps[b:b + n, None] ** 2),
                              axis=1)
    return out


@pytest.mark.parametrize("seed", range(12))
def test_random_treepm_cutoff(ctx, seed):
    rng = np.random.default_rng(3000 + seed)
    ps = _set(rng, seed)
    n_leaf = int(rng.choice([1, 4, 8, 32]))
    n_group = int(rng.choice([1, 16, 64, 300]))
    theta = float(rng.uniform(0.2, 1.0))
    r_cut = float(np.exp(rng.uniform(np.log(0.02), np.log(2.0))))
    _say(f"[random treepm {seed}] n={ps.n} sys={ps.n_sys} leaf={n_leaf} group={n_group} "
         f"theta={theta:.3f} r_cut={r_cut:.3f}")
    t = O.build_tree(ps, n_leaf)
    g = O.make_groups(t, n_group)
    L = O.cutoff_lists(t, g, theta, r_cut)
    ref = np.empty((ps.n, 3))
    ref[t.perm.astype(np.int64)] = L.force()
    ctx.set_particles(ps)
    ctx.calc_force_cutoff(theta, n_leaf, n_group, 0.0, r_cut)
    ne, ns, epj, spj = ctx.lists()
    assert np.array_equal(ne.astype(np.int64), L.n_epj)
    assert np.array_equal(ns.astype(np.int64), L.n_spj)
    oe = np.concatenate([[0], np.cumsum(ne.astype(np.int64))])
    os_ = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    for k in range(g.n):
        e_ref, s_ref = L.group_lists(k)
        assert np.array_equal(np.sort(epj[oe[k]:oe[k + 1]]), np.sort(e_ref))
        assert np.array_equal(np.sort(spj[os_[k]:os_[k + 1]]), np.sort(s_ref))
    a = ctx.forces()[:, :3]
    scale = np.empty(ps.n)
    scale[t.perm.astype(np.int64)] = _newton_scale(t, g, L)
    err = np.linalg.norm(a - ref, axis=1)
    assert np.all(err <= 1e-12 * scale)
    if np.any(ref != 0):
        assert np.sqrt(np.sum(err ** 2) / np.sum(ref ** 2)) <= 1e-12
