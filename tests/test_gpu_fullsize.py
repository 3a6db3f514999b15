"""GPU parity at the benchmark configurations' full sizes, in the launch configuration bench.py
times: keys, order, every cell and every group bit-exact against the oracle's full serial
build; lists and forces on sampled groups; accuracy against FP64 direct summation on seeded
subsets; the ensemble with graph-captured steps; the predictor path at full size; the
exchange lists of the benchmark input cut into 64 and 512 domains; its multisection domain
decomposition; the whole path at 4x the benchmark size; the ensemble in the one-launch walk +
force kernel."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

from parity_util import (BAR_RMS_VS_DIRECT, F32_RMS_REL_VS_TREE, check_groups, check_moments,
                         rel_err)

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(os.path.dirname(HERE), "paper_1601_03138_amd",
                       "predictor_clustered16m_ng256.bin")


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


def _compare_full(ctx, ps, n_leaf, n_group, theta, quad, n_sample_groups, seed):
    """Everything the oracle can afford at this size; returns (tree, groups, sampled lists)."""
    t = O.build_tree(ps, n_leaf)
    g = O.make_groups(t, n_group)
    tree = ctx.tree()
    assert np.array_equal(tree["cube"], t.cube)
    assert np.array_equal(tree["key"], t.skey)
    assert np.array_equal(tree["perm"], t.perm)
    for k in ("level", "prefix", "begin", "count", "first_child", "nchild", "parent"):
        assert np.array_equal(tree[k], getattr(t, k).astype(tree[k].dtype)), k
    check_moments(tree["mom"], t)
    check_groups(ctx.groups(), g)
    # lists of sampled groups
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(g.n, min(n_sample_groups, g.n), replace=False))
    lists = O.walk(t, g, theta, sel)
    ne, ns = ctx.list_counts()
    assert np.array_equal(ne[sel].astype(np.int64), lists.n_epj)
    assert np.array_equal(ns[sel].astype(np.int64), lists.n_spj)
    return t, g, sel, lists


def _sampled_force_check(ctx, t, g, sel, lists, quad):
    ref = lists.force(quad)                       # sorted order, rows of sampled groups
    a = ctx.forces()
    rows = np.concatenate([np.arange(g.begin[k], g.begin[k] + g.count[k]) for k in sel])
    user = t.perm[rows].astype(np.int64)
    e = rel_err(a[user], ref[rows])
    return float(np.sqrt(np.mean(e ** 2)))


def _check_sampled_entry_sets(gpu_lists, lists, sel):
    """The GPU's entry sets of the sampled groups equal the oracle's (as sets: the order of
    entries within a list is not part of the result)."""
    ne, ns, epj, spj = gpu_lists
    oe = np.concatenate([[0], np.cumsum(ne.astype(np.int64))])
    os_ = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    for q, k in enumerate(sel):
        e_ref, s_ref = lists.group_lists(q)
        assert np.array_equal(np.sort(epj[oe[k]:oe[k + 1]]), np.sort(e_ref)), k
        assert np.array_equal(np.sort(spj[os_[k]:os_[k + 1]]), np.sort(s_ref)), k


def test_clustered16m_bench_configuration(ctx, fdx):
    """The benchmark input: tree, groups and the entry sets of 256 sampled groups against the
    oracle for the exact walk; then the timed configuration (persistent force kernel over
    per-XCD queues, predicted walk) in the FP32 shapes the benchmark chooses between, each
    bit-identical to the direct launch of the same shape after the exact walk, with the same
    entry sets, within the FP32 tolerance of the oracle tree on the sampled groups."""
    ps = I.workload("clustered16m")
    _say(f"[fullsize] clustered16m n={ps.n}")
    ctx.set_particles(ps)
    ctx.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=True)
    t, g, sel, lists = _compare_full(ctx, ps, 8, 256, 0.5, True, 256, seed=5)
    gl = ctx.lists()
    _check_sampled_entry_sets(gl, lists, sel)
    del gl
    e_tree = _sampled_force_check(ctx, t, g, sel, lists, True)
    sub = I.subset(ps.n, 256, seed=102)
    e_direct = O.rms_rel_error(ctx.forces()[sub], O.direct(ps, sub))
    _say(f"  cells {t.n_cells} groups {g.n}; fp32 vs tree (256 sampled groups) {e_tree:.2e}; "
         f"vs direct {e_direct:.2e}")
    assert e_tree <= F32_RMS_REL_VS_TREE
    assert e_direct <= BAR_RMS_VS_DIRECT
    if not os.path.exists(WEIGHTS):
        pytest.skip("trained predictor weights not present")
    ctx.predictor_load(WEIGHTS)
    names = [ctx.shape_name(v) for v in range(ctx.lib.fdx_autotune_shapes())]
    for name in ("nt512_ipl1_pf_w8", "nt512_ipl1_w8", "nt512_ipl2"):
        ctx.set_shape(names.index(name))
        ctx.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=True)
        a_direct = ctx.forces()
        ctx.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=True, persistent=True, predictor=True)
        st = ctx.stats()
        assert st["shape"] == names.index(name)
        a = ctx.forces()
        assert np.array_equal(a, a_direct), name
        gl = ctx.lists()
        _check_sampled_entry_sets(gl, lists, sel)
        del gl
        e = _sampled_force_check(ctx, t, g, sel, lists, True)
        _say(f"  {name}: persistent + predicted walk == direct + exact walk; overflow groups "
             f"{st['overflow_groups']}; fp32 vs tree {e:.2e}")
        assert e <= F32_RMS_REL_VS_TREE
    ctx.set_shape(-1)


def test_plummer1m_fp64_fp32_and_ten_steps(ctx, fdx):
    ps = I.workload("plummer1m")
    _say(f"[fullsize] plummer1m n={ps.n}")
    sub = I.subset(ps.n, 4096, seed=102)
    d = O.direct(ps, sub)
    ctx.set_particles(ps)
    ctx.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=False)
    t, g, sel, lists = _compare_full(ctx, ps, 8, 256, 0.5, True, 64, seed=6)
    a64 = ctx.forces()
    ref = lists.force(True)
    rows = np.concatenate([np.arange(g.begin[k], g.begin[k] + g.count[k]) for k in sel])
    e64_tree = rel_err(a64[t.perm[rows].astype(np.int64)], ref[rows])
    assert e64_tree.max() <= 1e-9
    ctx.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=True)
    a32 = ctx.forces()
    e32 = O.rms_rel_error(a32[sub], d)
    e64 = O.rms_rel_error(a64[sub], d)
    _say(f"  rms vs direct (4096 subset): fp32 {e32:.3e} fp64 {e64:.3e}")
    assert e32 <= BAR_RMS_VS_DIRECT and e64 <= BAR_RMS_VS_DIRECT
    # ten leapfrog steps of dt = 1/256; energy from the tree potential
    def energy():
        x, y, z, vx, vy, vz = ctx.particles()
        return (0.5 * np.sum(ps.m * (vx ** 2 + vy ** 2 + vz ** 2))
                + 0.5 * np.sum(ps.m * ctx.forces()[:, 3]))
    E0 = energy()
    ctx.integrate(1.0 / 256.0, 10)
    E1 = energy()
    _say(f"  energy drift after 10 steps: {abs((E1 - E0) / E0):.2e}")
    assert abs((E1 - E0) / E0) < 1e-4


def test_ensemble512_graph_configuration(ctx, fdx):
    ens = I.workload("ensemble512")
    _say(f"[fullsize] ensemble512 n={ens.n} systems={ens.n_sys}")
    ctx.set_particles(ens)
    ctx.calc_force(0.6, 8, 128, 0.0, quad=True, fp32=True, persistent=True)
    t, g, sel, lists = _compare_full(ctx, ens, 8, 128, 0.6, True, 64, seed=7)
    assert _sampled_force_check(ctx, t, g, sel, lists, True) <= F32_RMS_REL_VS_TREE
    # a subset of systems against direct summation, all their particles
    off = ens.offsets()
    errs = []
    for s in (0, 100, 511):
        sl = np.arange(off[s], off[s + 1])
        errs.append(O.rms_rel_error(ctx.forces()[sl], O.direct(ens, sl)))
    _say(f"  rms da/a (theta 0.6) of systems 0, 100, 511: {np.round(errs, 5)}")
    assert max(errs) < 5e-3
    # graph-captured steps equal eager steps
    x0 = ctx.particles()
    ctx.integrate(1.0 / 256.0, 3, graph=True)
    g_state = (ctx.particles(), ctx.forces())
    ctx.set_particles(ens)
    ctx.calc_force(0.6, 8, 128, 0.0, quad=True, fp32=True, persistent=True)
    assert all(np.array_equal(a, b) for a, b in zip(ctx.particles(), x0))
    ctx.integrate(1.0 / 256.0, 3)
    for a, b in zip(ctx.particles(), g_state[0]):
        assert np.array_equal(a, b)
    assert np.array_equal(ctx.forces(), g_state[1])


def test_ensemble512_fused_walk_and_force(ctx, fdx):
    """The ensemble in the one-launch walk + force kernel, as the benchmark's ensemble line
    runs it: entry sets of 256 sampled groups against the oracle (lists captured), the
    separate walk's counts for every group, FP32 forces within the tolerance of the oracle
    tree, and graph-captured steps equal to eager steps."""
    ens = I.workload("ensemble512")
    _say(f"[fullsize] ensemble512 fused n={ens.n}")
    ctx.set_particles(ens)
    ctx.calc_force(0.6, 8, 128, 0.0, quad=True, fp32=True, persistent=True)
    counts = ctx.list_counts()
    flags = fdx.Context.flags(quad=True, fp32=True, persistent=True, fused=True)
    ctx.set_list_capture(True)
    ctx.calc_force_flags(0.6, 8, 128, 0.0, flags)
    ctx.set_list_capture(False)
    t, g, sel, lists = _compare_full(ctx, ens, 8, 128, 0.6, True, 256, seed=17)
    _check_sampled_entry_sets(ctx.lists(), lists, sel)
    for x, y in zip(ctx.list_counts(), counts):
        assert np.array_equal(x, y)
    e = _sampled_force_check(ctx, t, g, sel, lists, True)
    _say(f"  fused fp32 vs tree (256 sampled groups) {e:.2e}")
    assert e <= F32_RMS_REL_VS_TREE
    x0 = ctx.particles()
    ctx.integrate(1.0 / 256.0, 3, graph=True)
    g_state = (ctx.particles(), ctx.forces())
    ctx.set_particles(ens)
    ctx.calc_force_flags(0.6, 8, 128, 0.0, flags)
    assert all(np.array_equal(a, b) for a, b in zip(ctx.particles(), x0))
    ctx.integrate(1.0 / 256.0, 3)
    for a, b in zip(ctx.particles(), g_state[0]):
        assert np.array_equal(a, b)
    assert np.array_equal(ctx.forces(), g_state[1])


def test_clustered16m_exchange_lists_64_domains(fdx):
    """The benchmark input cut into 4 x 4 x 4 equal-count domains: local trees and the
    counts of all 4032 pairs bit-exact, entry sets of sampled pairs."""
    ps = I.workload("clustered16m")
    dom, _ = I.multisection(ps, 4, 4, 4)
    _say(f"[fullsize] exchange lists, n={dom.n} domains={dom.n_sys}")
    t = O.build_tree(dom, 8)
    L = O.exchange(t, 0.5)
    c = fdx.Context(0)
    try:
        c.set_particles(dom)
        c.build_exchange_lists(0.5, 8)
        tree = c.tree()
        assert np.array_equal(tree["key"], t.skey) and np.array_equal(tree["perm"], t.perm)
        for k in ("level", "begin", "count", "first_child", "nchild", "parent"):
            assert np.array_equal(tree[k], getattr(t, k).astype(tree[k].dtype)), k
        pairs, ne, ns, epj, spj = c.exchange_lists()
        assert np.array_equal(ne, L.n_epj) and np.array_equal(ns, L.n_spj)
        oe = np.concatenate([[0], np.cumsum(ne)])
        os_ = np.concatenate([[0], np.cumsum(ns)])
        rng = np.random.default_rng(8)
        for k in rng.choice(len(pairs), 64, replace=False):
            e_ref, s_ref = L.epj[L.epj_off[k]:L.epj_off[k + 1]], L.spj[L.spj_off[k]:L.spj_off[k + 1]]
            assert np.array_equal(np.sort(epj[oe[k]:oe[k + 1]]), np.sort(t.perm[e_ref]))
            assert np.array_equal(np.sort(spj[os_[k]:os_[k + 1]]), np.sort(s_ref))
        st = c.exchange_stats()
        _say(f"  entries {int(ne.sum() + ns.sum())}; device ms: trees {st['ms_tree']:.3f}, "
             f"lists {st['ms_lists']:.3f}")
    finally:
        c.close()


def test_clustered16m_domain_decomposition_64_domains(fdx):
    """The benchmark input in 4 x 4 x 4 current domains decomposed again into 4 x 4 x 4 from
    2^20 samples drawn in proportion to a cost per domain: samples, faces, destinations,
    exchange order and send counts bit-exact; the exchange of particles applied."""
    ps = I.workload("clustered16m")
    dom, _ = I.multisection(ps, 4, 4, 4)
    n_p = np.diff(dom.offsets())
    cost = n_p * (1.0 + np.arange(dom.n_sys) % 5)
    _say(f"[fullsize] domain decomposition, n={dom.n} current domains={dom.n_sys}")
    ref = O.decompose(dom, 4, 4, 4, 1 << 20, cost=cost, seed=1)
    c = fdx.Context(0)
    try:
        c.set_particles(dom)
        c.decompose(4, 4, 4, 1 << 20, cost=cost, seed=1)
        k, idx, cell = c.dd_samples()
        assert np.array_equal(k, ref.k) and np.array_equal(idx, ref.idx)
        assert np.array_equal(cell, ref.cell)
        d = c.decomposition()
        for f in ("bx", "by", "bz"):
            assert np.array_equal(d[f], getattr(ref, f)), f
        dest, order = c.dd_destinations()
        assert np.array_equal(dest, ref.dest) and np.array_equal(order, ref.order)
        assert np.array_equal(d["counts"], ref.counts)
        assert np.array_equal(d["dom_off"], ref.dom_off)
        c.exchange_particles()
        x, y, z, vx, vy, vz = c.particles()
        o = ref.order.astype(np.int64)
        assert np.array_equal(x, dom.x[o]) and np.array_equal(vz, dom.vz[o])
        st = c.dd_stats()
        _say(f"  samples {st['n_samples']}, moved {st['n_moved']}; device ms: sample "
             f"{st['ms_sample']:.3f}, divide {st['ms_divide']:.3f}, assign "
             f"{st['ms_assign']:.3f}, exchange {st['ms_exchange']:.3f}")
    finally:
        c.close()


def test_clustered16m_exchange_lists_512_domains_two_pass(fdx):
    """8 x 8 x 8 domains: the per-sender bound (511 n entries) exceeds the one-pass budget, so
    a count walk sizes every segment before the fill walk; counts of all 261,632 pairs and
    the entry sets of sampled pairs bit-exact, capacity = the exact total."""
    ps = I.workload("clustered16m")
    dom, _ = I.multisection(ps, 8, 8, 8)
    _say(f"[fullsize] exchange lists, n={dom.n} domains={dom.n_sys}")
    t = O.build_tree(dom, 8)
    L = O.exchange(t, 0.5)
    c = fdx.Context(0)
    try:
        c.set_particles(dom)
        c.build_exchange_lists(0.5, 8)
        pairs, ne, ns, epj, spj = c.exchange_lists()
        assert np.array_equal(ne, L.n_epj) and np.array_equal(ns, L.n_spj)
        oe = np.concatenate([[0], np.cumsum(ne)])
        os_ = np.concatenate([[0], np.cumsum(ns)])
        rng = np.random.default_rng(9)
        for k in rng.choice(len(pairs), 256, replace=False):
            e_ref, s_ref = L.epj[L.epj_off[k]:L.epj_off[k + 1]], L.spj[L.spj_off[k]:L.spj_off[k + 1]]
            assert np.array_equal(np.sort(epj[oe[k]:oe[k + 1]]), np.sort(t.perm[e_ref]))
            assert np.array_equal(np.sort(spj[os_[k]:os_[k + 1]]), np.sort(s_ref))
        st = c.exchange_stats()
        assert st["list_capacity"] == int(ne.sum() + ns.sum())     # sized by the count walk
        _say(f"  entries {int(ne.sum() + ns.sum())}; device ms: trees {st['ms_tree']:.3f}, "
             f"lists {st['ms_lists']:.3f}")
    finally:
        c.close()


def test_clustered64m_beyond_the_benchmark_size(fdx):
    """N = 2^26 clustered (4x the benchmark): 3.5e9 list entries, past signed 32-bit offsets.  Keys,
    order, every cell and group bit-exact; sampled lists exact; FP32 forces against the tree
    and against direct summation on the GPU."""
    ps = I.clustered(n_background=1 << 25, n_clusters=64, n_per_cluster=1 << 19, seed=26)
    _say(f"[fullsize] clustered n={ps.n}")
    c = fdx.Context(0)
    try:
        c.set_particles(ps)
        c.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=True)
        st = c.stats()
        assert st["n_epj"] + st["n_spj"] > (1 << 31)          # past signed 32-bit offsets
        t = O.build_tree(ps, 8)
        g = O.make_groups(t, 256)
        tree = c.tree()
        assert np.array_equal(tree["key"], t.skey) and np.array_equal(tree["perm"], t.perm)
        for k in ("level", "prefix", "begin", "count", "first_child", "nchild", "parent"):
            assert np.array_equal(tree[k], getattr(t, k).astype(tree[k].dtype)), k
        check_moments(tree["mom"], t)
        check_groups(c.groups(), g)
        rng = np.random.default_rng(3)
        sel = np.sort(rng.choice(g.n, 32, replace=False))
        lists = O.walk(t, g, 0.5, sel)
        ne, ns = c.list_counts()
        assert np.array_equal(ne[sel].astype(np.int64), lists.n_epj)
        assert np.array_equal(ns[sel].astype(np.int64), lists.n_spj)
        e_tree = _sampled_force_check(c, t, g, sel, lists, True)
        sub = I.subset(ps.n, 256, seed=102)
        e_direct = O.rms_rel_error(c.forces()[sub], c.direct_forces(sub))
        _say(f"  entries {st['n_epj'] + st['n_spj']}; fp32 vs tree {e_tree:.2e}, vs direct "
             f"{e_direct:.2e}")
        assert e_tree <= F32_RMS_REL_VS_TREE and e_direct <= BAR_RMS_VS_DIRECT
    finally:
        c.close()
