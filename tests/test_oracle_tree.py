"""Pins of the oracle's serial tree (O-T) against geometry, brute force, library routines,
closed forms and invariants."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I


def _pos_set(pos, m=None, eps=0.01):
    pos = np.asarray(pos, float)
    n = pos.shape[0]
    m = np.full(n, 1.0 / n) if m is None else np.asarray(m, float)
    return I._pack(pos.copy(), np.zeros((n, 3)), m.copy(), np.full(n, eps))


# ---------------------------------------------------------------------------------------
# keys
def test_root_cube_is_tight_power_of_two():
    for seed in range(5):
        ps = I.uniform_cube(500, seed, 0.01, side=0.37 * (seed + 1))
        cube, _ = O.keys(ps)
        o, Lr = cube[0, :3], cube[0, 3]
        L = max(ps.x.max() - ps.x.min(), ps.y.max() - ps.y.min(), ps.z.max() - ps.z.min())
        assert math.frexp(Lr)[0] == 0.5            # a power of two
        assert Lr >= L > Lr / 2
        assert np.array_equal(o, [ps.x.min(), ps.y.min(), ps.z.min()])


def test_grid_coordinates_locate_particles():
    ps = I.plummer(3000, seed=1, eps=0.01)
    cube, key = O.keys(ps)
    q = O.deinterleave(key)
    o, Lr = cube[0, :3], cube[0, 3]
    h = Lr / 2 ** 21
    for a, arr in enumerate((ps.x, ps.y, ps.z)):
        lo = o[a] + q[:, a] * h
        hi = o[a] + (q[:, a] + 1.0) * h
        top = q[:, a] == 2 ** 21 - 1
        assert np.all(lo <= arr + 1e-15 * abs(arr).max())
        assert np.all((arr < hi + 1e-15 * abs(arr).max()) | top)


def _octant_path(p, o, Lr, depth):
    """Octants visited by halving the root cube geometrically (no bit arithmetic)."""
    lo = np.array(o, float)
    size = Lr
    path = []
    for _ in range(depth):
        size /= 2
        mid = lo + size
        bx, by, bz = (p >= mid).astype(int)
        path.append(4 * bx + 2 * by + bz)
        lo = lo + size * np.array([bx, by, bz])
    return path


def test_key_order_is_geometric_octant_order():
    ps = I.uniform_cube(400, 4, 0.01)
    cube, key = O.keys(ps)
    o, Lr = cube[0, :3], cube[0, 3]
    paths = [tuple(_octant_path(np.array([ps.x[i], ps.y[i], ps.z[i]]), o, Lr, 21))
             for i in range(ps.n)]
    for d in (1, 2, 5, 21):
        # the top 3d key bits are the octant path to depth d, one octal digit per level
        top = key >> np.uint64(3 * (21 - d))
        val = [sum(int(p[k]) << (3 * (d - 1 - k)) for k in range(d)) for p in paths]
        assert np.array_equal(top.astype(np.int64), np.array(val, dtype=np.int64))


def test_interleave_round_trip():
    rng = np.random.default_rng(0)
    q = rng.integers(0, 2 ** 21, size=(200, 3), dtype=np.uint32)
    k = np.array([O.interleave(*map(int, r)) for r in q], dtype=np.uint64)
    assert np.all(k < np.uint64(2 ** 63))
    assert np.array_equal(O.deinterleave(k), q)


def test_sort_matches_library_stable_sort():
    ps = I.ensemble(n_sys=5, seed=2, nmin=100, nmax=900)
    _, key = O.keys(ps)
    # add exact duplicates to exercise the tie rule
    key[10:20] = key[5]
    perm = O.sort(ps, key)
    sys = np.searchsorted(ps.offsets(), np.arange(ps.n), side="right") - 1
    ref = np.lexsort((np.arange(ps.n), key, sys))
    assert np.array_equal(perm.astype(np.int64), ref)


# ---------------------------------------------------------------------------------------
# topology
def _brute_cells(skey, off, n_leaf):
    """All cells by definition: a level-l run of equal key prefixes is a cell when l == 0 or
    its parent run holds more than n_leaf particles (and the parent's level is < 21)."""
    cells = set()
    for s in range(len(off) - 1):
        b, e = int(off[s]), int(off[s + 1])
        cells.add((0, 0, b, e - b))
        for lv in range(1, 22):
            pre = skey[b:e] >> np.uint64(3 * (21 - lv))
            par = skey[b:e] >> np.uint64(3 * (22 - lv))
            for p in np.unique(pre):
                idx = np.nonzero(pre == p)[0]
                pidx = np.nonzero(par == (p >> np.uint64(3)))[0]
                if len(pidx) > n_leaf:
                    cells.add((lv, int(p), b + int(idx[0]), len(idx)))
    return cells


@pytest.mark.parametrize("n_leaf", [1, 4, 8])
def test_cells_match_brute_force(n_leaf):
    ps = I.concat([I.plummer(300, seed=3, eps=0.01), I.uniform_cube(200, 5, 0.01)])
    t = O.build_tree(ps, n_leaf=n_leaf, moments=False)
    got = set(zip(t.level.tolist(), t.prefix.tolist(), t.begin.tolist(), t.count.tolist()))
    assert got == _brute_cells(t.skey, t.off, n_leaf)
    assert len(got) == t.n_cells


def test_cell_invariants_and_bfs_order():
    ps = I.plummer(5000, seed=8, eps=0.01)
    t = O.build_tree(ps, n_leaf=8, moments=False)
    # breadth-first: level non-decreasing, begins ascending within a level
    assert np.all(np.diff(t.level) >= 0)
    for lv in np.unique(t.level):
        b = t.begin[t.level == lv]
        assert np.all(np.diff(b.astype(np.int64)) > 0)
    in_leaf = np.zeros(ps.n, int)
    for c in range(t.n_cells):
        nc = t.nchild[c]
        if nc:
            ch = np.arange(t.first_child[c], t.first_child[c] + nc)
            assert np.all(t.parent[ch] == c)
            assert np.all((t.prefix[ch] >> np.uint64(3)) == t.prefix[c])
            assert t.begin[ch[0]] == t.begin[c]
            assert np.sum(t.count[ch]) == t.count[c]
            assert np.all(t.begin[ch[1:]] == t.begin[ch[:-1]] + t.count[ch[:-1]])
            assert np.all(np.diff(t.prefix[ch].astype(np.int64)) > 0)
        else:
            assert t.count[c] <= 8 or t.level[c] == 21
            in_leaf[t.begin[c]:t.begin[c] + t.count[c]] += 1
    assert np.all(in_leaf == 1)


def test_cells_contain_their_particles_geometrically():
    ps = I.plummer(2000, seed=6, eps=0.01)
    t = O.build_tree(ps, moments=False)
    o, Lr = t.cube[0, :3], t.cube[0, 3]
    for c in range(0, t.n_cells, 7):
        lv = t.level[c]
        size = Lr / 2 ** lv
        corner = O.deinterleave(np.array([t.prefix[c] << np.uint64(3 * (21 - lv))]))[0]
        lo = o + corner * (Lr / 2 ** 21)
        sl = slice(t.begin[c], t.begin[c] + t.count[c])
        p = np.stack([t.sx[sl], t.sy[sl], t.sz[sl]], 1)
        assert np.all(p >= lo - 1e-12) and np.all(p <= lo + size + 1e-12)


def test_coincident_particles_make_deep_leaf():
    pos = np.zeros((12, 3))
    pos[:, 0] = 0.25
    pos[0] = [0.0, 0.0, 0.0]
    pos[1] = [1.0, 1.0, 1.0]
    t = O.build_tree(_pos_set(pos), n_leaf=8, moments=False)
    deep = np.nonzero(t.nchild == 0)[0]
    assert t.level.max() == 21
    big = deep[t.count[deep] > 8]
    assert len(big) == 1 and t.level[big[0]] == 21 and t.count[big[0]] == 10


# ---------------------------------------------------------------------------------------
# moments
def test_dumbbell_quadrupole_closed_form():
    # masses m1, m2 a distance s apart on the x axis: M = m1+m2, COM on the axis,
    # Q_xx = 2 mu s^2, Q_yy = Q_zz = -mu s^2 (mu = m1 m2 / M), off-diagonal 0
    m1, m2, s = 0.3, 0.7, 0.125
    pos = np.array([[0.1, 0.2, 0.3], [0.1 + s, 0.2, 0.3]])
    t = O.build_tree(_pos_set(pos, [m1, m2]), n_leaf=8)
    mo = t.mom[0]
    mu = m1 * m2 / (m1 + m2)
    assert mo[0] == pytest.approx(1.0)
    assert mo[1] == pytest.approx((0.1 * m1 + (0.1 + s) * m2), rel=1e-15)
    assert mo[4] == pytest.approx(2 * mu * s * s, rel=1e-13)
    assert mo[5] == pytest.approx(-mu * s * s, rel=1e-13)
    assert mo[6] == pytest.approx(-mu * s * s, rel=1e-13)
    assert np.allclose(mo[7:], 0, atol=1e-17)


def test_moments_traceless_and_parallel_axis():
    ps = I.plummer(3000, seed=2, eps=0.01)
    t = O.build_tree(ps)
    m = t.mom
    tr = m[:, 4] + m[:, 5] + m[:, 6]
    scale = np.abs(m[:, 4:7]).sum(axis=1) + 1e-300
    assert np.all(np.abs(tr) <= 1e-13 * scale)
    # parent = children shifted to the parent's centre of mass (parallel-axis theorem)
    for c in np.nonzero(t.nchild > 0)[0][:300]:
        ch = np.arange(t.first_child[c], t.first_child[c] + t.nchild[c])
        M = m[ch, 0].sum()
        X = (m[ch, 0, None] * m[ch, 1:4]).sum(0) / M
        Q = np.zeros(6)
        for k in ch:
            d = m[k, 1:4] - X
            d2 = d @ d
            Q += m[k, 4:10] + m[k, 0] * np.array([3 * d[0] ** 2 - d2, 3 * d[1] ** 2 - d2,
                                                  3 * d[2] ** 2 - d2, 3 * d[0] * d[1],
                                                  3 * d[0] * d[2], 3 * d[1] * d[2]])
        assert M == pytest.approx(m[c, 0], rel=1e-14)
        assert np.allclose(X, m[c, 1:4], rtol=1e-12, atol=1e-15)
        assert np.allclose(Q, m[c, 4:10], rtol=1e-10, atol=1e-12 * np.abs(Q).max())


def _spj_force_error(quad, size, rng):
    """Relative error of the force that one superparticle (a cluster of half-width `size`
    centred at (0.7, 0.7, 0.7)) exerts on a particle at the origin, eps = 0.  With the
    root cube [0, 1]^3 the cluster fills only octant 7, which the walk accepts whole."""
    n = 40
    cl = 0.7 + rng.uniform(-size, size, (n, 3))
    ms = rng.uniform(0.5, 1.5, n) / n
    pos = np.vstack([[[0.0, 0.0, 0.0]], cl])
    m = np.concatenate([[1e-30], ms])
    ps = _pos_set(pos, m, eps=0.0)
    exact = O.direct(ps, [0])[0]
    tr = O.build_tree(ps, n_leaf=1)
    assert tr.cube[0, 3] == 1.0
    g = O.make_groups(tr, 1)
    sel = [k for k in range(g.n) if tr.perm[g.begin[k]] == 0]
    lists = O.walk(tr, g, theta=0.5, sel=sel)
    epj, spj = lists.group_lists(0)
    assert epj.tolist() == [0] and len(spj) == 1 and tr.count[spj[0]] == n
    acc = lists.force(quad)
    return np.linalg.norm(acc[0, :3] - exact[:3]) / np.linalg.norm(exact[:3])


def _spj_potential_error(quad, size, rng):
    """Relative error of the potential of the same far superparticle at the origin (the
    particle's own list entry is itself, whose term is excluded), against the exact
    -sum_k m_k / |x_k| of the cluster's particles written out here."""
    n = 40
    cl = 0.7 + rng.uniform(-size, size, (n, 3))
    ms = rng.uniform(0.5, 1.5, n) / n
    pos = np.vstack([[[0.0, 0.0, 0.0]], cl])
    m = np.concatenate([[1e-30], ms])
    ps = _pos_set(pos, m, eps=0.0)
    exact = -float(np.sum(ms / np.linalg.norm(cl, axis=1)))
    tr = O.build_tree(ps, n_leaf=1)
    g = O.make_groups(tr, 1)
    sel = [k for k in range(g.n) if tr.perm[g.begin[k]] == 0]
    lists = O.walk(tr, g, theta=0.5, sel=sel)
    epj, spj = lists.group_lists(0)
    assert epj.tolist() == [0] and len(spj) == 1 and tr.count[spj[0]] == n
    return abs(lists.force(quad)[0, 3] - exact) / abs(exact)


def test_multipole_convergence_order():
    # with eps = 0 the monopole error of a far cell falls like (s/d)^2 and the quadrupole
    # error like (s/d)^3 (the dipole vanishes about the centre of mass)
    sizes = np.array([0.16, 0.08, 0.04, 0.02])
    em = [_spj_force_error(False, s, np.random.default_rng(1)) for s in sizes]
    eq = [_spj_force_error(True, s, np.random.default_rng(1)) for s in sizes]
    sm = np.polyfit(np.log(sizes), np.log(em), 1)[0]
    sq = np.polyfit(np.log(sizes), np.log(eq), 1)[0]
    assert sm == pytest.approx(2.0, abs=0.2)
    assert sq == pytest.approx(3.0, abs=0.2)
    assert all(q < m for q, m in zip(eq, em))


def test_multipole_potential_convergence_order():
    # the potential of a far cell: the monopole leaves the quadrupole term, an error falling
    # like (s/d)^2; with the quadrupole term the error is the octupole's, (s/d)^3.  A wrong
    # sign or factor of the quadrupole potential term leaves an (s/d)^2 error.
    sizes = np.array([0.16, 0.08, 0.04, 0.02])
    em = [_spj_potential_error(False, s, np.random.default_rng(2)) for s in sizes]
    eq = [_spj_potential_error(True, s, np.random.default_rng(2)) for s in sizes]
    sm = np.polyfit(np.log(sizes), np.log(em), 1)[0]
    sq = np.polyfit(np.log(sizes), np.log(eq), 1)[0]
    assert sm == pytest.approx(2.0, abs=0.2)
    assert sq == pytest.approx(3.0, abs=0.25)
    assert all(q < 0.2 * m for q, m in zip(eq, em))


# ---------------------------------------------------------------------------------------
# groups
@pytest.mark.parametrize("n_group", [1, 5, 16, 64, 300])
def test_groups_partition_and_maximal(n_group):
    ps = I.concat([I.plummer(2500, seed=4, eps=0.01), I.plummer(700, seed=5, eps=0.01)])
    t = O.build_tree(ps, n_leaf=8, moments=False)
    g = O.make_groups(t, n_group)
    assert np.all(np.diff(g.begin.astype(np.int64)) > 0)
    assert g.begin[0] == 0
    assert np.all(g.begin[1:] == g.begin[:-1] + g.count[:-1])
    assert int(g.begin[-1] + g.count[-1]) == ps.n
    assert np.all(g.count <= n_group) and np.all(g.count >= 1)
    for k in range(g.n):
        c = g.cell[k]
        if t.count[c] <= n_group:
            assert g.begin[k] == t.begin[c] and g.count[k] == t.count[c]
            assert c < t.n_sys or t.count[t.parent[c]] > n_group
        else:                           # a chunk of an over-full leaf
            assert t.nchild[c] == 0
    # the integer box bounds the members' grid coordinates tightly
    q = O.deinterleave(t.skey)
    for k in range(0, g.n, 5):
        sl = slice(g.begin[k], g.begin[k] + g.count[k])
        assert np.array_equal(q[sl].min(0), g.qmin[k])
        assert np.array_equal(q[sl].max(0), g.qmax[k])


# ---------------------------------------------------------------------------------------
# walk
def _ancestors(t, c):
    out = []
    while c >= t.n_sys:
        c = int(t.parent[c])
        out.append(c)
    return out


def test_walk_exact_cover_and_characterisation():
    ps = I.concat([I.plummer(1500, seed=12, eps=0.01), I.uniform_cube(600, 2, 0.01)])
    t = O.build_tree(ps, n_leaf=8, moments=False)
    g = O.make_groups(t, 32)
    theta = 0.5
    lists = O.walk(t, g, theta)
    off = t.off
    for k in range(g.n):
        epj, spj = lists.group_lists(k)
        s = int(t.csys[g.cell[k]])
        covered = np.zeros(ps.n, int)
        covered[epj] += 1
        for c in spj:
            covered[t.begin[c]:t.begin[c] + t.count[c]] += 1
        assert np.all(covered[off[s]:off[s + 1]] == 1)
        assert np.all(covered[:off[s]] == 0) and np.all(covered[off[s + 1]:] == 0)
        assert np.all(np.diff(epj.astype(np.int64)) > 0)
    # brute force: c is a superparticle of g iff c passes the test and no proper ancestor
    # does; a particle is in EPJ iff neither its leaf nor any ancestor passes.  Checked on a
    # sample of groups with the test evaluated from real-space geometry (the box spans the
    # members' grid cells; S^2 < theta^2 D^2).
    o_all, Lr_all = t.cube[:, :3], t.cube[:, 3]
    for k in range(0, g.n, 9):
        s = int(t.csys[g.cell[k]])
        o, Lr = o_all[s], Lr_all[s]
        h = Lr / 2 ** 21
        bmin = o + g.qmin[k] * h
        bmax = o + (g.qmax[k] + 1.0) * h
        cells = np.nonzero(t.csys == s)[0]
        ok = np.zeros(t.n_cells, bool)
        for c in cells:
            lv = t.level[c]
            size = Lr / 2 ** lv
            corner = O.deinterleave(np.array([t.prefix[c] << np.uint64(3 * (21 - lv))]))[0]
            cen = o + corner * h + size / 2
            dvec = np.maximum(0, np.maximum(bmin - cen, cen - bmax))
            ok[c] = size * size < theta * theta * (dvec @ dvec) * (1 - 1e-12)
        want_spj = sorted(int(c) for c in cells if ok[c] and not any(ok[a] for a in _ancestors(t, c)))
        epj, spj = lists.group_lists(k)
        assert sorted(spj.tolist()) == want_spj
        leaves = [c for c in cells if t.nchild[c] == 0 and t.count[c] > 0
                  and not ok[c] and not any(ok[a] for a in _ancestors(t, c))]
        want_epj = sorted(i for c in leaves for i in range(t.begin[c], t.begin[c] + t.count[c]))
        assert epj.tolist() == want_epj


def test_walk_box_test_is_conservative_for_every_member():
    ps = I.plummer(4000, seed=21, eps=0.01)
    t = O.build_tree(ps, moments=False)
    g = O.make_groups(t, 64)
    theta = 0.6
    lists = O.walk(t, g, theta)
    o, Lr = t.cube[0, :3], t.cube[0, 3]
    h = Lr / 2 ** 21
    for k in range(0, g.n, 4):
        _, spj = lists.group_lists(k)
        sl = slice(g.begin[k], g.begin[k] + g.count[k])
        p = np.stack([t.sx[sl], t.sy[sl], t.sz[sl]], 1)
        for c in spj[::5]:
            lv = t.level[c]
            size = Lr / 2 ** lv
            corner = O.deinterleave(np.array([t.prefix[c] << np.uint64(3 * (21 - lv))]))[0]
            cen = o + corner * h + size / 2
            d = np.linalg.norm(p - cen, axis=1)
            assert np.all(size < theta * d)


def test_theta_to_zero_is_direct_sum():
    ps = I.plummer(1500, seed=13, eps=0.02)
    a_d = O.direct(ps)
    a_t = O.tree_force(ps, theta=1e-7, n_leaf=8, n_group=16, quad=True)
    assert np.allclose(a_t, a_d, rtol=1e-12, atol=1e-13)


def test_tree_error_against_direct_sum():
    ps = I.plummer(8192, seed=14, eps=1 / 256)
    a_d = O.direct(ps)
    e_prev = None
    for theta in (0.3, 0.5, 0.7):
        a_q = O.tree_force(ps, theta, 8, 64, quad=True)
        e = O.rms_rel_error(a_q, a_d)
        if theta == 0.5:
            assert e <= 1e-3
            a_m = O.tree_force(ps, theta, 8, 64, quad=False)
            assert O.rms_rel_error(a_m, a_d) > e
        if e_prev is not None:
            assert e > e_prev
        e_prev = e
    # potential agrees too
    a_q = O.tree_force(ps, 0.5, 8, 64, quad=True)
    assert np.sqrt(np.mean(((a_q[:, 3] - a_d[:, 3]) / a_d[:, 3]) ** 2)) < 1e-3


def test_mean_list_length_near_paper_model():
    # equation nlist_long is a fit for a disk galaxy at theta = 0.4; a loose factor-of-two pin
    ps = I.plummer(1 << 16, seed=15, eps=1e-3)
    t = O.build_tree(ps, moments=False)
    for ng in (64, 256):
        g = O.make_groups(t, ng)
        lists = O.walk(t, g, 0.5)
        # the model is per i-group of n_grp particles; weight groups by their size
        mean = np.sum((lists.n_epj + lists.n_spj) * g.count) / ps.n
        model = O.nlist_model(ng, 0.5, ps.n)
        assert 0.5 < mean / model < 2.0


def _cell_by_halving(p, o, Lr, level):
    """Lower corner and side of the level-`level` cube holding point p, by halving the root
    cube geometrically (no keys, no bit arithmetic)."""
    lo = np.array(o, float)
    size = Lr
    for _ in range(level):
        size /= 2
        lo = lo + size * (p >= lo + size)
    return lo, size


def test_group_centre_is_its_cell_centre_by_geometric_halving():
    ps = I.concat([I.plummer(3000, seed=8, eps=0.01), I.uniform_cube(900, 9, 0.01, side=0.3)])
    tr = O.build_tree(ps, n_leaf=8, moments=False)
    g = O.make_groups(tr, 32)
    for k in range(0, g.n, 7):
        c = int(g.cell[k])
        s = int(tr.csys[c])
        o, Lr = tr.cube[s, :3], tr.cube[s, 3]
        b = int(g.begin[k])
        p = np.array([tr.sx[b], tr.sy[b], tr.sz[b]])
        lo, side = _cell_by_halving(p, o, Lr, int(tr.level[c]))
        assert np.allclose(g.centre[k], lo + side / 2, rtol=0, atol=4e-16 * (abs(o).max() + Lr))
        # every member lies in the cube of half-width side / 2 about the centre
        mem = slice(b, b + int(g.count[k]))
        for a, arr in enumerate((tr.sx, tr.sy, tr.sz)):
            assert np.all(np.abs(arr[mem] - g.centre[k, a]) <= side / 2 * (1 + 1e-12))


def test_group_features_from_geometry():
    # the network's eight inputs, recomputed from positions alone: cubes by geometric halving
    # of the root cube, counts and masses by membership, the integer box by quantising the
    # members' coordinates to the 2^21 grid of the root side
    ps = I.concat([I.plummer(2500, seed=10, eps=0.01), I.plummer(700, seed=11, eps=0.01)])
    tr = O.build_tree(ps, n_leaf=8)
    g = O.make_groups(tr, 40)
    X = O.group_features(tr, g)
    off = ps.offsets()
    pos = np.stack([ps.x, ps.y, ps.z], axis=1)
    checked = 0
    for k in range(0, g.n, 11):
        c = int(g.cell[k])
        s = int(tr.csys[c])
        o, Lr = tr.cube[s, :3], tr.cube[s, 3]
        sl = slice(int(off[s]), int(off[s + 1]))
        b = int(g.begin[k])
        p0 = np.array([tr.sx[b], tr.sy[b], tr.sz[b]])
        lc = int(tr.level[c])
        lp = max(lc - 1, 0)
        lo_p, side_p = _cell_by_halving(p0, o, Lr, lp)
        inside = np.all((pos[sl] >= lo_p) & (pos[sl] < lo_p + side_p), axis=1)
        mem = slice(b, b + int(g.count[k]))
        q = np.floor((np.stack([tr.sx[mem], tr.sy[mem], tr.sz[mem]], 1) - o) * (2.0 ** 21 / Lr))
        q = np.minimum(q, 2.0 ** 21 - 1)
        ctr = 0.5 * (q.min(0) + q.max(0) + 1.0) - 2.0 ** 20
        want = [math.log(int(g.count[k])),
                math.log(1.0 + float(np.max(q.max(0) - q.min(0)))),
                math.log(1.0 + float(np.linalg.norm(ctr))),
                math.log(ps.m[sl][inside].sum() / ps.m[sl].sum()),
                math.log(side_p / Lr), float(lc),
                math.log(int(inside.sum()) / (side_p / Lr) ** 3),
                math.log2(int(off[s + 1] - off[s]))]
        assert np.allclose(X[k], want, rtol=1e-12, atol=1e-12), (k, X[k], want)
        checked += 1
    assert checked > 20
