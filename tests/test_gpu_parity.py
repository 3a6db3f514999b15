"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded
inputs.  Keys, order, cells, groups and lists bit-exact; moments and forces to tolerances
derived in parity_util."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

from parity_util import (BAR_RMS_VS_DIRECT, F32_RMS_REL_VS_TREE, F64_MAX_REL, F64_RMS_REL,
                         check_groups, check_lists, check_moments, check_tree, pot_rel_err,
                         rel_err, tree_ref)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fdx():
    from paper_1601_03138_amd import fdx as F
    return F


@pytest.fixture(scope="module")
def ctx(fdx):
    c = fdx.Context(0)
    yield c
    c.close()


CASES = {
    # name: (particle set factory, n_leaf, n_group, theta, quad)
    "plummer4k_mono": (lambda: I.workload("plummer4k"), 8, 64, 0.5, False),
    "plummer20k_quad": (lambda: I.plummer(20000, seed=21, eps=1 / 256), 8, 256, 0.5, True),
    "clustered_quad": (lambda: I.clustered(n_background=16384, n_clusters=8, n_per_cluster=2048,
                                           seed=5), 8, 128, 0.5, True),
    "ensemble_ragged": (lambda: I.concat([I.plummer(n, seed=30 + k, eps=0.02) for k, n in
                                          enumerate([1, 2, 3, 64, 65, 1000, 4097, 257])]),
                        8, 64, 0.6, True),
    "leaf1_group5": (lambda: I.plummer(3000, seed=22, eps=0.01), 1, 5, 0.4, True),
    "group512": (lambda: I.plummer(12000, seed=23, eps=0.01), 16, 512, 0.7, True),
    # the ends of the opening-angle range: theta = 1 with 64-particle leaves, and theta = 0.1
    # (lists close to the whole system)
    "theta1_leaf64": (lambda: I.plummer(8000, seed=24, eps=0.01), 64, 256, 1.0, True),
    "theta01": (lambda: I.plummer(3000, seed=25, eps=0.01), 8, 64, 0.1, True),
}


def _coincident():
    ps = I.uniform_cube(700, 41, 0.05)
    ps.x[100:400] = ps.x[100]      # 300 coincident particles -> level-21 leaf, chunked groups
    ps.y[100:400] = ps.y[100]
    ps.z[100:400] = ps.z[100]
    return ps


CASES["coincident"] = (_coincident, 8, 64, 0.5, True)


def _deep_pairs():
    # 400 pairs about two grid units apart: with n_leaf = 1 every pair is a chain of
    # single-child cells down to level ~20, so the tree needs ~8 cells per particle, more
    # than the first allocation (n + 1024): the build is truncated, flagged and retried larger
    ps = I.uniform_cube(800, 43, 0.05)
    ps.x[1::2] = ps.x[0::2] + 1e-6
    ps.y[1::2] = ps.y[0::2]
    ps.z[1::2] = ps.z[0::2]
    return ps


CASES["deep_pairs"] = (_deep_pairs, 1, 8, 0.5, True)


@pytest.mark.parametrize("name", list(CASES))
def test_structure_and_fp64_forces(ctx, name):
    make, n_leaf, n_group, theta, quad = CASES[name]
    ps = make()
    _say(f"[parity] {name}: n={ps.n} sys={ps.n_sys} leaf={n_leaf} group={n_group} theta={theta}")
    t, g, lists = tree_ref(ps, n_leaf, n_group, theta)
    ctx.set_particles(ps)
    ctx.calc_force(theta, n_leaf, n_group, 0.0, quad=quad, fp32=False)
    st = ctx.stats()
    assert st["n_cells"] == t.n_cells and st["n_groups"] == g.n
    check_tree(ctx.tree(), t)
    check_moments(ctx.tree()["mom"], t)
    check_groups(ctx.groups(), g)
    check_lists(ctx.lists(), lists)
    ref_sorted = lists.force(quad)
    ref = np.empty_like(ref_sorted)
    ref[t.perm.astype(np.int64)] = ref_sorted
    a = ctx.forces()
    ok = np.linalg.norm(ref[:, :3], axis=1) > 0
    e = rel_err(a[ok], ref[ok])
    _say(f"  fp64 vs tree: max {e.max():.3e} rms {np.sqrt(np.mean(e**2)):.3e}")
    assert e.max() <= F64_MAX_REL and np.sqrt(np.mean(e ** 2)) <= F64_RMS_REL
    okp = ref[:, 3] != 0
    assert pot_rel_err(a[okp], ref[okp]).max() <= F64_MAX_REL
    # counts reported by the library
    assert st["n_epj"] == lists.n_epj.sum() and st["n_spj"] == lists.n_spj.sum()
    assert st["n_interactions_pp"] == int(np.sum(lists.n_epj * g.count.astype(np.int64)))


@pytest.mark.parametrize("name", ["plummer4k_mono", "plummer20k_quad", "clustered_quad",
                                  "ensemble_ragged", "coincident"])
def test_fp32_relative_forces(ctx, name):
    make, n_leaf, n_group, theta, quad = CASES[name]
    ps = make()
    _say(f"[parity-fp32] {name}: n={ps.n}")
    t, g, lists = tree_ref(ps, n_leaf, n_group, theta)
    ref_sorted = lists.force(quad)
    ref = np.empty_like(ref_sorted)
    ref[t.perm.astype(np.int64)] = ref_sorted
    ctx.set_particles(ps)
    ctx.calc_force(theta, n_leaf, n_group, 0.0, quad=quad, fp32=True)
    a = ctx.forces()
    ok = np.linalg.norm(ref[:, :3], axis=1) > 0
    e = rel_err(a[ok], ref[ok])
    rms = float(np.sqrt(np.mean(e ** 2)))
    _say(f"  fp32 vs tree: rms {rms:.3e} max {e.max():.3e}")
    assert rms <= F32_RMS_REL_VS_TREE
    # lists of the FP32 run are the same lists
    check_lists(ctx.lists(), lists)


@pytest.mark.parametrize("fp32", [False, True])
def test_accuracy_bar_against_direct_sum(ctx, fp32):
    ps = I.plummer(30000, seed=24, eps=1 / 256)
    sub = I.subset(ps.n, 2048, seed=102)
    d = O.direct(ps, sub)
    ctx.set_particles(ps)
    ctx.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=fp32)
    a = ctx.forces()[sub]
    e = O.rms_rel_error(a, d)
    _say(f"[bar] fp32={fp32}: rms vs direct {e:.3e}")
    assert e <= BAR_RMS_VS_DIRECT


def test_determinism(ctx):
    ps = I.clustered(n_background=20000, n_clusters=4, n_per_cluster=3000, seed=8)
    ctx.set_particles(ps)
    outs = []
    for _ in range(2):
        ctx.calc_force(0.5, 8, 128, 0.0, quad=True, fp32=True)
        outs.append((ctx.forces(), ctx.lists()))
    assert np.array_equal(outs[0][0], outs[1][0])
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b)


def test_two_body_and_single_particle(ctx):
    d, eps, m1, m2 = 0.7, 0.1, 0.3, 1.9
    ps = I._pack(np.array([[0.0, 0, 0], [d, 0, 0]]), np.zeros((2, 3)), np.array([m1, m2]),
                 np.full(2, eps))
    ctx.set_particles(ps)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True)
    a = ctx.forces()
    den = (d * d + eps * eps) ** 1.5
    assert a[0, 0] == pytest.approx(m2 * d / den, rel=1e-14)
    assert a[1, 0] == pytest.approx(-m1 * d / den, rel=1e-14)
    one = I._pack(np.array([[0.3, 0.2, 0.1]]), np.zeros((1, 3)), np.array([1.0]), np.array([0.1]))
    ctx.set_particles(one)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True)
    assert np.array_equal(ctx.forces(), np.zeros((1, 4)))


def test_empty_input_and_empty_system(ctx, fdx):
    empty = I._pack(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    ctx.set_particles(empty)
    ctx.calc_force(0.5, 8, 64, 0.0)
    assert ctx.forces().shape == (0, 4)
    a = I.plummer(500, seed=3, eps=0.02)
    b = I.plummer(300, seed=4, eps=0.02)
    both = I.concat([a, b])
    both.sys_off = np.array([0, 500, 500, 800], dtype=np.int64)   # empty middle system
    t, g, lists = tree_ref(both, 8, 64, 0.5)
    ctx.set_particles(both)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True)
    check_tree(ctx.tree(), t)
    check_lists(ctx.lists(), lists)


def test_steps_on_empty_input_and_an_empty_system(ctx, fdx):
    _say("[empty steps] n = 0, eager and graph steps")
    empty = I._pack(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    ctx.set_particles(empty)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True, fp32=True, persistent=True)
    ctx.integrate(1.0 / 256.0, 2)
    ctx.integrate(1.0 / 256.0, 2, graph=True)
    assert ctx.forces().shape == (0, 4)
    assert all(a.shape == (0,) for a in ctx.particles())
    _say("[empty steps] empty middle system, eager against graph steps")
    a = I.plummer(500, seed=3, eps=0.02)
    b = I.plummer(300, seed=4, eps=0.02)
    both = I.concat([a, b])
    both.sys_off = np.array([0, 500, 500, 800], dtype=np.int64)
    runs = []
    for graph in (False, True):
        ctx.set_particles(both)
        ctx.calc_force(0.5, 8, 64, 0.0, quad=True, fp32=True, persistent=True)
        ctx.integrate(1.0 / 256.0, 3, graph=graph)
        runs.append((ctx.particles(), ctx.forces()))
    for u, v in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(u, v)
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.all(np.isfinite(runs[1][1]))


def test_invalid_arguments_return_codes(ctx, fdx):
    ps = I.plummer(100, seed=1, eps=0.01)
    ctx.set_particles(ps)
    for theta, nl, ng in [(0.0, 8, 64), (1.5, 8, 64), (0.5, 0, 64), (0.5, 8, 0), (0.5, 8, 513)]:
        with pytest.raises(fdx.FdxError) as ei:
            ctx.calc_force(theta, nl, ng, 0.0)
        assert ei.value.code == fdx.EINVAL
    bad = I.plummer(100, seed=1, eps=0.01)
    bad.x[5] = np.nan
    with pytest.raises(fdx.FdxError) as ei:
        ctx.set_particles(bad)
    assert ei.value.code == fdx.EINVAL
    bad = I.plummer(100, seed=1, eps=0.01)
    bad.eps[3] = 0.0
    with pytest.raises(fdx.FdxError):
        ctx.set_particles(bad)
    # global eps must be > 0 when no per-particle eps is given
    ctx.set_particles(ps, per_particle_eps=False)
    with pytest.raises(fdx.FdxError):
        ctx.calc_force(0.5, 8, 64, 0.0)
    ctx.calc_force(0.5, 8, 64, 0.01)


def test_device_borrowed_input_and_device_check(ctx, fdx):
    import torch
    ps = I.plummer(5000, seed=25, eps=0.01)
    dev = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
           for k in ("x", "y", "z", "vx", "vy", "vz", "m", "eps")}
    ctx.set_particles_device(dev)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True)
    a_dev = ctx.forces()
    ctx.set_particles(ps)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True)
    assert np.array_equal(a_dev, ctx.forces())
    dev["x"][7] = float("nan")
    ctx.set_particles_device(dev)
    with pytest.raises(fdx.FdxError) as ei:
        ctx.calc_force(0.5, 8, 64, 0.0, quad=True)
    assert ei.value.code == fdx.EINVAL


def test_uniform_eps_array_takes_the_global_softening_path(ctx, fdx):
    # an eps array whose values are all equal is gathered as one value: forces equal those of
    # the global eps, from host and from device input; one differing value switches the
    # per-particle gather back on (its forces then match the oracle tree)
    import torch
    ps = I.plummer(5000, seed=26, eps=0.01)
    ctx.set_particles(ps, per_particle_eps=False)
    ctx.calc_force(0.5, 8, 64, 0.01, quad=True, fp32=True)
    a_global = ctx.forces()
    ctx.set_particles(ps)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True, fp32=True)
    assert np.array_equal(ctx.forces(), a_global)
    dev = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
           for k in ("x", "y", "z", "vx", "vy", "vz", "m", "eps")}
    ctx.set_particles_device(dev)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True, fp32=True)
    assert np.array_equal(ctx.forces(), a_global)
    q = I._pack(np.stack([ps.x, ps.y, ps.z], 1), np.stack([ps.vx, ps.vy, ps.vz], 1), ps.m,
                ps.eps.copy())
    q.eps[1234] = 0.02
    ref = O.tree_force(q, 0.5, 8, 64, quad=True)
    for host in (True, False):
        if host:
            ctx.set_particles(q)
        else:
            dev["eps"][1234] = 0.02
            ctx.set_particles_device(dev)
        ctx.calc_force(0.5, 8, 64, 0.0, quad=True, fp32=False)
        a = ctx.forces()
        assert not np.array_equal(a, a_global)
        assert np.allclose(a, ref, rtol=1e-9, atol=1e-12)


def test_eps_shared_within_each_system(ctx, fdx):
    # systems of one softening each (different between systems, empty systems first, in the
    # middle and last): the sorted gather takes each system's value from its first particle;
    # one differing value inside a system switches the per-particle gather back on.  Forces
    # match the oracle tree either way, from host and from device input.
    import torch
    sets = [I.plummer(700, seed=27, eps=0.01), I.plummer(1300, seed=28, eps=0.03),
            I.uniform_cube(900, seed=29, eps=0.005)]
    both = I.concat(sets)
    both.sys_off = np.array([0, 0, 700, 700, 2000, 2900, 2900], dtype=np.int64)
    _say(f"[eps per system] n={both.n} systems={len(both.sys_off) - 1}")
    for k in (None, 1500):                      # None: one eps per system; else one differs
        q = I._pack(np.stack([both.x, both.y, both.z], 1), np.zeros((both.n, 3)), both.m,
                    both.eps.copy(), both.sys_off)
        if k is not None:
            q.eps[k] *= 2.0
        ref = O.tree_force(q, 0.5, 8, 64, quad=True)
        dev = {name: torch.tensor(getattr(q, name), dtype=torch.float64, device="cuda")
               for name in ("x", "y", "z", "vx", "vy", "vz", "m", "eps")}
        for host in (True, False):
            if host:
                ctx.set_particles(q)
            else:
                ctx.set_particles_device(dev, q.sys_off)
            ctx.calc_force(0.5, 8, 64, 0.0, quad=True, fp32=False)
            assert np.allclose(ctx.forces(), ref, rtol=1e-9, atol=1e-12), (k, host)


def test_leapfrog_step_matches_oracle(ctx):
    # one force evaluation plus one KDK step of the sample program, dt = 1/128, N = 4096
    ps = I.workload("plummer4k")
    ctx.set_particles(ps)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=False, fp32=False)
    a0 = ctx.forces()
    ctx.integrate(1.0 / 128.0, 1)
    x, y, z, vx, vy, vz = ctx.particles()
    # oracle: same step with the oracle tree's forces at the same positions
    v = np.stack([ps.vx, ps.vy, ps.vz], 1).copy()
    p = np.stack([ps.x, ps.y, ps.z], 1).copy()
    aref0 = O.tree_force(ps, 0.5, 8, 64, quad=False)
    assert np.allclose(a0, aref0, rtol=1e-9, atol=1e-12)
    O.kick(v, aref0[:, :3], 1 / 128)
    O.drift(p, v, 1 / 128)
    assert np.allclose(np.stack([x, y, z], 1), p, rtol=0, atol=1e-13)
    q = I._pack(np.stack([x, y, z], 1), np.zeros_like(p), ps.m, ps.eps)
    aref1 = O.tree_force(q, 0.5, 8, 64, quad=False)   # the oracle fed the GPU's positions
    O.kick(v, aref1[:, :3], 1 / 128)
    assert np.allclose(np.stack([vx, vy, vz], 1), v, rtol=0, atol=1e-12)
    # the force accuracy of the plain (monopole) method on this input, against direct sum
    d = O.direct(ps)
    e = O.rms_rel_error(a0, d)
    _say(f"[plummer4k] monopole rms vs direct {e:.3e}")
    assert e < 2e-3


def test_direct_sum_reference_matches_the_oracle(ctx, fdx):
    """fdx_direct_forces (the bench's accuracy reference) against the oracle's direct sum:
    per-particle and global softening, several systems (sums stay inside each), argument
    errors."""
    ps = I.concat([I.plummer(n, seed=60 + k, eps=0.01 * (k + 1)) for k, n in
                   enumerate([3000, 1, 700, 20011])])
    ps.eps = ps.eps * (1.0 + 0.1 * np.sin(np.arange(ps.n)))          # per-particle values
    sub = np.concatenate([I.subset(ps.n, 400, seed=61), [3000, ps.n - 1]])
    ref = O.direct(ps, sub)
    ctx.set_particles(ps)
    d = ctx.direct_forces(sub)
    rel = np.abs(d - ref) / np.maximum(np.abs(ref), 1e-300)
    rel[sub == 3000, :3] = np.abs(d[sub == 3000, :3] - ref[sub == 3000, :3])   # alone: a = 0
    _say(f"[direct] max rel vs oracle {rel.max():.2e}")
    assert rel.max() <= 1e-12
    # one global softening
    ctx.set_particles(ps, per_particle_eps=False)
    g = I.ParticleSet(ps.x, ps.y, ps.z, ps.vx, ps.vy, ps.vz, ps.m, np.full(ps.n, 0.02),
                      ps.sys_off)
    d2 = ctx.direct_forces(sub[:50], eps=0.02)
    assert np.allclose(d2, O.direct(g, sub[:50]), rtol=1e-12, atol=0)
    with pytest.raises(fdx.FdxError):
        ctx.direct_forces([ps.n])
    with pytest.raises(fdx.FdxError):
        ctx.direct_forces([0], eps=0.0)


def _wide_groups_reference(t, g):
    """Groups the FP32 path must hand to the FP64 kernel: 9 u min(S / eps_min, 2^d) > 1e-4."""
    leaf = t.nchild == 0
    plev = np.zeros(t.sx.shape[0], np.int64)
    for b, c, l in zip(t.begin[leaf], t.count[leaf], t.level[leaf]):
        plev[int(b):int(b) + int(c)] = int(l)
    b = g.begin.astype(np.int64)
    deep = np.maximum.reduceat(plev, b)
    emin = np.minimum.reduceat(t.seps, b)
    lvl = t.level[g.cell].astype(np.int64)
    side = np.ldexp(t.cube.reshape(-1, 4)[t.csys[g.cell], 3], -lvl)
    m = np.minimum(side / emin, np.ldexp(1.0, deep - lvl))
    return (9.0 * 2.0 ** -24) * m > 1e-4


def test_fp32_path_hands_wide_groups_to_fp64(ctx):
    """A small system of two tight clumps 10^4 apart is one group: group-relative FP32 would
    lose ~1e-3 of its close-pair forces, so that group is evaluated in FP64 (its rows equal the
    FP64 evaluation bit for bit); compact groups stay FP32."""
    a = I.plummer(200, seed=81, eps=0.01)
    a.x[100:] += 1.0e4
    b = I.plummer(3000, seed=82, eps=0.01)
    ps = I.concat([a, b])
    t, g, lists = tree_ref(ps, 1, 200, 0.76)
    wide = _wide_groups_reference(t, g)
    assert wide.sum() >= 1 and not wide.all()
    ctx.set_particles(ps)
    ctx.calc_force(0.76, 1, 200, 0.0, quad=True, fp32=False)
    a64 = ctx.forces()
    ctx.calc_force(0.76, 1, 200, 0.0, quad=True, fp32=True)
    a32 = ctx.forces()
    assert ctx.stats()["fp64_groups"] == int(wide.sum())
    rows = np.concatenate([np.arange(g.begin[k], g.begin[k] + g.count[k]) for k in np.nonzero(wide)[0]])
    user = t.perm[rows].astype(np.int64)
    assert np.array_equal(a32[user], a64[user])
    other = np.setdiff1d(np.arange(ps.n), user)
    assert not np.array_equal(a32[other], a64[other])
    ref_sorted = lists.force(True)
    ref = np.empty_like(ref_sorted)
    ref[t.perm.astype(np.int64)] = ref_sorted
    ok = np.linalg.norm(ref[:, :3], axis=1) > 0
    e = rel_err(a32[ok], ref[ok])
    _say(f"[wide] fp64 groups {int(wide.sum())} of {g.n}; fp32-path rms vs tree {np.sqrt(np.mean(e ** 2)):.2e}")
    assert np.sqrt(np.mean(e ** 2)) <= F32_RMS_REL_VS_TREE


def test_wide_groups_in_graph_steps(ctx):
    """The same input through eager and graph-captured leapfrog steps with the persistent FP32
    launch: the group too wide for FP32 goes to the FP64 kernel inside the captured step too."""
    a = I.plummer(200, seed=81, eps=0.01)
    a.x[100:] += 1.0e4
    ps = I.concat([a, I.plummer(3000, seed=82, eps=0.01)])
    runs = []
    for graph in (False, True):
        ctx.set_particles(ps)
        ctx.calc_force(0.76, 1, 200, 0.0, quad=True, fp32=True, persistent=True)
        assert ctx.stats()["fp64_groups"] >= 1
        ctx.integrate(1.0 / 1024.0, 3, graph=graph)
        runs.append((ctx.particles(), ctx.forces(), ctx.stats()["fp64_groups"]))
    _say(f"[wide graph] fp64 groups after the steps: eager {runs[0][2]}, graph {runs[1][2]}")
    for u, v in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(u, v)
    assert np.array_equal(runs[0][1], runs[1][1])
