"""Comparison helpers for GPU-vs-oracle parity tests (test infrastructure)."""
import numpy as np

import oracle as O
from paper_1601_03138_amd import inputs as I

# FP64 kernel vs the oracle tree (same lists, different summation order): recursive summation
# of L terms errs by at most ~L u sum|t_j| with u = 2^-53.  With L <= 2e4 entries and the
# cancellation factor sum|t_j| / |a_i| below ~50 for these inputs, |da|/|a| <= 2e4 * 1.1e-16 *
# 50 ~ 1e-10 per particle; the rms over particles is far smaller.
F64_MAX_REL = 1e-9
F64_RMS_REL = 1e-11
# FP32 group-relative kernel vs the oracle tree: FP32 rounding (u = 6e-8) of coordinates,
# per-interaction arithmetic and tile sums, compensated across tiles: ~1e-6 rms.
F32_RMS_REL_VS_TREE = 3e-5
# The accuracy bar against FP64 direct summation at theta = 0.5 (quadrupole).
BAR_RMS_VS_DIRECT = 1e-3


def tree_ref(ps, n_leaf, n_group, theta):
    t = O.build_tree(ps, n_leaf)
    g = O.make_groups(t, n_group)
    lists = O.walk(t, g, theta)
    return t, g, lists


def check_tree(gpu_tree, t):
    assert np.array_equal(gpu_tree["cube"], t.cube)
    assert np.array_equal(gpu_tree["key"], t.skey)
    assert np.array_equal(gpu_tree["perm"], t.perm)
    for k in ("level", "prefix", "begin", "count", "first_child", "nchild", "parent"):
        got, want = gpu_tree[k], getattr(t, k)
        assert got.shape == want.shape, (k, got.shape, want.shape)
        assert np.array_equal(got, want.astype(got.dtype)), k


def check_moments(gpu_mom, t):
    """Bottom-up (GPU) vs per-cell direct (oracle) moments, FP64."""
    m, r = gpu_mom, t.mom
    Lr = t.cube[t.csys, 3]
    size = Lr / 2.0 ** t.level
    assert np.allclose(m[:, 0], r[:, 0], rtol=1e-13, atol=0)
    assert np.all(np.abs(m[:, 1:4] - r[:, 1:4]) <= 1e-13 * Lr[:, None] + 1e-12 * size[:, None])
    qscale = r[:, 0] * size * size + 1e-300
    assert np.all(np.abs(m[:, 4:] - r[:, 4:]) <= 1e-10 * qscale[:, None])


def check_groups(gg, g):
    for k in ("cell", "begin", "count"):
        assert np.array_equal(gg[k], getattr(g, k)), k
    assert np.array_equal(gg["qmin"], g.qmin)
    assert np.array_equal(gg["qmax"], g.qmax)
    assert np.array_equal(gg["centre"], g.centre)


def check_lists(gpu_lists, lists):
    ne, ns, epj, spj = gpu_lists
    assert np.array_equal(ne.astype(np.int64), lists.n_epj)
    assert np.array_equal(ns.astype(np.int64), lists.n_spj)
    oe = np.concatenate([[0], np.cumsum(ne.astype(np.int64))])
    os_ = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    for k in range(ne.shape[0]):
        e_ref, s_ref = lists.group_lists(k)
        assert np.array_equal(np.sort(epj[oe[k]:oe[k + 1]]), np.sort(e_ref))
        assert np.array_equal(np.sort(spj[os_[k]:os_[k + 1]]), np.sort(s_ref))


def rel_err(a, ref):
    d = np.linalg.norm(a[:, :3] - ref[:, :3], axis=1)
    r = np.linalg.norm(ref[:, :3], axis=1)
    return d / r


def pot_rel_err(a, ref):
    return np.abs(a[:, 3] - ref[:, 3]) / np.abs(ref[:, 3])


def fp32_error_bound(t, g, lists, ref_sorted):
    """Per-particle bound (sorted order) on the relative error of the FP32 group-relative
    kernel against the FP64 kernel on the same lists.  Coordinates relative to the group
    centre c are rounded to FP32 (unit roundoff u = 2^-24), so a pair separation d = x_j - x_i
    is off by at most sqrt(3) u (|x_i - c| + |x_j - c|); the pair force m d / r_eff^3 then
    moves by at most 3 |dd| / r_eff of its size, plus a few u of arithmetic:
        |da_i| <= sum_j m_j / r_eff^2 (3 sqrt(3) u (|x_i - c| + |x_j - c|) / r_eff + 8 u),
    superparticles taken as point masses at their centre of mass.  Returned as |da_i| / |a_i|
    (inf where a_i = 0).  It grows with the group's extent over its pair separations."""
    u = 2.0 ** -24
    pos = np.stack([t.sx, t.sy, t.sz], axis=1)
    out = np.full(t.sx.shape[0], np.inf)
    for k in range(g.n):
        b, n = int(g.begin[k]), int(g.count[k])
        c = g.centre[k]
        xi = pos[b:b + n] - c
        ni = np.linalg.norm(xi, axis=1)
        e, s = lists.group_lists(k)
        xj = np.concatenate([pos[e.astype(np.int64)], t.mom[s.astype(np.int64), 1:4]]) - c
        mj = np.concatenate([t.sm[e.astype(np.int64)], t.mom[s.astype(np.int64), 0]])
        nj = np.linalg.norm(xj, axis=1)
        d = xj[None, :, :] - xi[:, None, :]
        reff = np.sqrt(np.sum(d * d, axis=2) + (t.seps[b:b + n] ** 2)[:, None])
        dd = np.sqrt(3.0) * u * (ni[:, None] + nj[None, :])
        term = mj[None, :] / reff ** 2 * (3.0 * dd / reff + 8.0 * u)
        self_pair = np.zeros_like(term, dtype=bool)
        self_pair[:, :len(e)] = (e.astype(np.int64)[None, :] == np.arange(b, b + n)[:, None])
        term[self_pair] = 0.0
        amag = np.linalg.norm(ref_sorted[b:b + n, :3], axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            out[b:b + n] = np.where(amag > 0, term.sum(axis=1) / amag, np.inf)
    return out


def _random_set(rng, kind, n, seed):
    if kind == "plummer" or (kind == "clustered" and n < 400):
        return I.plummer(n, seed=seed, eps=float(rng.uniform(1e-3, 0.05)))
    if kind == "cube":
        return I.uniform_cube(n, seed, float(rng.uniform(1e-3, 0.05)))
    if kind == "clustered":
        k = max(1, n // 400)
        return I.clustered(n_background=n - k * 200, n_clusters=k, n_per_cluster=200, seed=seed,
                           eps=float(rng.uniform(1e-3, 0.02)))
    if kind == "lattice":                  # many coincident particles
        q = rng.integers(-3, 4, size=(n, 3)).astype(np.float64) * 0.25
        v = np.zeros((n, 3))
        return I._pack(q, v, np.full(n, 1.0 / n), np.full(n, 0.05))
    # two clumps 10^4 apart: a deep tree with a huge dynamic range
    p = I.plummer(n, seed=seed, eps=0.01)
    p.x[n // 2:] += 1.0e4
    return p


def random_case(seed):
    """Seeded random configuration: one to three systems of ragged sizes drawn from Plummer,
    uniform cube, clustered, coarse lattice (coincident particles) and two far-apart clumps,
    with random n_leaf, n_group, theta and moment order."""
    rng = np.random.default_rng(1000 + seed)
    kinds = ["plummer", "cube", "clustered", "lattice", "clumps"]
    n_sys = int(rng.integers(1, 4))
    sets = []
    for s in range(n_sys):
        n = int(rng.choice([1, 2, int(rng.integers(3, 300)), int(rng.integers(300, 4000))]))
        sets.append(_random_set(rng, kinds[int(rng.integers(0, len(kinds)))], n, seed * 10 + s))
    ps = sets[0] if n_sys == 1 else I.concat(sets)
    n_leaf = int(rng.choice([1, 2, 4, 8, 16, 32]))
    n_group = int(rng.choice([1, 7, 64, 200, 512]))
    theta = float(rng.uniform(0.2, 1.0))
    quad = bool(rng.integers(0, 2))
    return ps, n_leaf, n_group, theta, quad
