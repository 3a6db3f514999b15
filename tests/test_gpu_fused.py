"""GPU: the one-launch walk + force kernel (FDX_FUSED, the multiwalk of the batched ensemble).

The lists it evaluates (stored only with list capture on) equal the oracle's as sets and its
per-group counts equal the separate walk's; FP64 forces within the FP64 tolerance of the
oracle tree, FP32 forces within the per-particle FP32 bound; graph-captured fused steps
bit-identical to eager fused steps, whatever the queue order (members or predicted cost);
leaves of more than 2^16 coincident particles; groups too wide for FP32 handed to FP64."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

from parity_util import (F32_RMS_REL_VS_TREE, F64_MAX_REL, F64_RMS_REL, check_lists,
                         fp32_error_bound, random_case, rel_err, tree_ref)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    from paper_1601_03138_amd import fdx
    return fdx


@pytest.fixture(scope="module")
def ctx(F):
    c = F.Context(0)
    yield c
    c.close()


def _flags(F, quad, fp32, **kw):
    return F.Context.flags(quad=quad, fp32=fp32, fused=True, **kw)


@pytest.mark.parametrize("seed", range(16))
def test_fused_random_configuration(ctx, F, seed):
    ps, n_leaf, n_group, theta, quad = random_case(seed)
    n_group = min(n_group, 256)
    _say(f"[fused {seed}] n={ps.n} sys={ps.n_sys} leaf={n_leaf} group={n_group} "
         f"theta={theta:.3f} quad={quad}")
    t, g, lists = tree_ref(ps, n_leaf, n_group, theta)
    ref_sorted = lists.force(quad)
    ref = np.empty_like(ref_sorted)
    ref[t.perm.astype(np.int64)] = ref_sorted
    ok = np.linalg.norm(ref[:, :3], axis=1) > 0
    ctx.set_particles(ps)
    # the separate walk's counts
    ctx.calc_force(theta, n_leaf, n_group, 0.0, quad=quad, fp32=False)
    ne0, ns0 = ctx.list_counts()
    # FP64 fused, lists captured
    ctx.set_list_capture(True)
    ctx.calc_force_flags(theta, n_leaf, n_group, 0.0, _flags(F, quad, False))
    ctx.set_list_capture(False)
    check_lists(ctx.lists(), lists)
    ne, ns = ctx.list_counts()
    assert np.array_equal(ne, ne0) and np.array_equal(ns, ns0)
    a64 = ctx.forces()
    if ok.any():
        e = rel_err(a64[ok], ref[ok])
        assert e.max() <= F64_MAX_REL and np.sqrt(np.mean(e ** 2)) <= F64_RMS_REL
    # FP64 fused without capture: the same forces bit for bit, counts only
    ctx.calc_force_flags(theta, n_leaf, n_group, 0.0, _flags(F, quad, False))
    assert np.array_equal(ctx.forces(), a64)
    ne, ns = ctx.list_counts()
    assert np.array_equal(ne, ne0) and np.array_equal(ns, ns0)
    with pytest.raises(F.FdxError) as e:
        ctx.lists()
    assert e.value.code == F.ESTATE
    # FP32 fused
    ctx.calc_force_flags(theta, n_leaf, n_group, 0.0, _flags(F, quad, True))
    st = ctx.stats()
    assert st["n_interactions_pp"] == int(np.sum(g.count.astype(np.int64) * lists.n_epj))
    assert st["n_interactions_pc"] == int(np.sum(g.count.astype(np.int64) * lists.n_spj))
    if ok.any():
        e32 = rel_err(ctx.forces()[ok], ref[ok])
        bound = np.empty(ps.n)
        bound[t.perm.astype(np.int64)] = fp32_error_bound(t, g, lists, ref_sorted)
        bound = bound[ok]
        rms = np.sqrt(np.mean(e32 ** 2))
        _say(f"  fp32 rms {rms:.2e}, max ratio to bound {np.max(e32 / bound):.2e}, "
             f"fp64 groups {st['fp64_groups']}")
        assert np.all(e32 <= 1.5 * bound + 1e-6)
        assert rms <= F32_RMS_REL_VS_TREE


def test_fused_leaf_of_more_than_2_16_coincident_particles(ctx, F):
    # 70 000 particles at one point (one level-21 leaf, cut into consecutive groups) in a
    # Plummer background: the walk's branch for leaves of 2^16 particles or more, and the
    # fused kernel's ranges spanning many tiles
    bg = I.plummer(6000, seed=71, eps=0.01)
    k = 70000
    pos = np.zeros((k, 3)) + np.array([0.3, -0.2, 0.1])
    blob = I._pack(pos, np.zeros((k, 3)), np.full(k, 1.0 / k), np.full(k, 0.01))
    ps = I.concat([bg, blob])
    ps = I._pack(np.stack([ps.x, ps.y, ps.z], 1), np.stack([ps.vx, ps.vy, ps.vz], 1), ps.m, ps.eps)
    theta, n_leaf, n_group = 0.5, 8, 256
    t = O.build_tree(ps, n_leaf)
    g = O.make_groups(t, n_group)
    big = int(np.max(t.count[t.nchild == 0]))
    _say(f"[big leaf] largest leaf {big} particles, {g.n} groups")
    assert big >= 1 << 16
    # groups to check: a sample of the leaf's chunks and of the background
    rng = np.random.default_rng(72)
    sel = np.unique(np.concatenate([rng.choice(g.n, 24, replace=False), [0, g.n - 1]]))
    lists = O.walk(t, g, theta, sel)
    ctx.set_particles(ps)
    for flags in (F.Context.flags(quad=True), _flags(F, True, False)):
        ctx.set_list_capture(True)
        ctx.calc_force_flags(theta, n_leaf, n_group, 0.0, flags)
        ctx.set_list_capture(False)
        ne, ns, epj, spj = ctx.lists()
        oe = np.concatenate([[0], np.cumsum(ne.astype(np.int64))])
        os_ = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
        for q, gi in enumerate(sel):
            e_ref, s_ref = lists.group_lists(q)
            assert np.array_equal(np.sort(epj[oe[gi]:oe[gi + 1]]), np.sort(e_ref)), gi
            assert np.array_equal(np.sort(spj[os_[gi]:os_[gi + 1]]), np.sort(s_ref)), gi
        assert int(ne.max()) >= 1 << 16
        a = ctx.forces()
        ref_sorted = lists.force(True)
        rows = np.concatenate([np.arange(g.begin[gi], g.begin[gi] + g.count[gi]) for gi in sel])
        got = a[t.perm.astype(np.int64)[rows]]
        want = ref_sorted[rows]
        # the blob's particles feel only the background (pairs at zero separation add 0)
        scale = np.linalg.norm(want[:, :3], axis=1) + 1e-300
        assert np.all(np.linalg.norm(got[:, :3] - want[:, :3], axis=1) <= 1e-9 * scale)
        assert np.allclose(got[:, 3], want[:, 3], rtol=1e-9, atol=0)


def _ensemble():
    return I.ensemble(n_sys=10, seed=81, nmin=700, nmax=12000)


def test_fused_graph_steps_equal_eager_steps(F):
    ps = _ensemble()
    theta, n_group, dt = 0.6, 128, 1.0 / 256.0
    flags = _flags(F, True, True)
    out = []
    for graph in (False, True):
        with F.Context(0) as c:
            c.set_particles(ps)
            c.calc_force_flags(theta, 8, n_group, 0.0, flags)
            c.integrate(dt, 4, graph=graph)
            out.append((np.array(c.particles()), c.forces(), c.list_counts()))
            if graph:
                assert c.stats()["graph_recoveries"] == 0
    (p0, f0, (e0, s0)), (p1, f1, (e1, s1)) = out
    assert np.array_equal(p0, p1)
    assert np.array_equal(f0, f1)
    assert np.array_equal(e0, e1) and np.array_equal(s0, s1)


def test_fused_queue_order_does_not_change_results(F):
    # the predictor's cost only moves the per-XCD run boundaries: forces are bit-identical with
    # and without it, eager and graph-captured
    ps = _ensemble()
    theta, n_group, dt = 0.6, 128, 1.0 / 256.0
    with F.Context(0) as c:
        c.set_particles(ps)
        # a small predictor trained on this input's exact walk
        c.build_tree(8, n_group)
        X = c.predictor_features()
        c.calc_force(theta, 8, n_group, 0.0, quad=True, fp32=True)
        ne, ns = c.list_counts()
        c.predictor_train(X, np.log((ne + ns).astype(np.float64)).astype(np.float32), epochs=4,
                          batch=256, lr=3e-3, seed=5)
        base = _flags(F, True, True)
        c.calc_force_flags(theta, 8, n_group, 0.0, base)
        f_plain = c.forces()
        c.calc_force_flags(theta, 8, n_group, 0.0, base | F.PREDICTOR | F.TIMING)
        assert np.array_equal(c.forces(), f_plain)
        st = c.stats()
        assert st["t_walk"] == 0.0 and st["t_force"] > 0 and st["t_predict"] > 0
        c.integrate(dt, 3)
        p_eager, f_eager = np.array(c.particles()), c.forces()
    with F.Context(0) as c:
        c.set_particles(ps)
        c.build_tree(8, n_group)
        c.calc_force(theta, 8, n_group, 0.0, quad=True, fp32=True)
        c.predictor_train(X, np.log((ne + ns).astype(np.float64)).astype(np.float32), epochs=4,
                          batch=256, lr=3e-3, seed=5)
        c.calc_force_flags(theta, 8, n_group, 0.0, _flags(F, True, True) | F.PREDICTOR)
        c.integrate(dt, 3, graph=True)
        assert np.array_equal(np.array(c.particles()), p_eager)
        assert np.array_equal(c.forces(), f_eager)


def test_fused_wide_groups_are_evaluated_in_fp64(F):
    # a small system of two tight clumps 10^4 apart forms one group too wide for group-relative
    # FP32: its rows equal the FP64 fused evaluation bit for bit
    a = I.plummer(150, seed=91, eps=0.01)
    a.x[75:] += 1.0e4
    ps = I.concat([a, I.plummer(3000, seed=92, eps=0.01)])
    with F.Context(0) as c:
        c.set_particles(ps)
        c.calc_force_flags(0.5, 8, 256, 0.0, _flags(F, True, True))
        st = c.stats()
        f32 = c.forces()
        c.calc_force_flags(0.5, 8, 256, 0.0, _flags(F, True, False))
        f64 = c.forces()
    _say(f"[wide] fp64 groups {st['fp64_groups']}")
    assert st["fp64_groups"] >= 1
    assert np.array_equal(f32[:150], f64[:150])


def test_fused_errors(ctx, F):
    ps = I.plummer(2000, seed=95, eps=0.01)
    ctx.set_particles(ps)
    with pytest.raises(F.FdxError) as e:
        ctx.calc_force_flags(0.5, 8, 300, 0.0, _flags(F, True, True))
    assert e.value.code == F.EINVAL
    with pytest.raises(F.FdxError) as e:
        ctx._check(ctx.lib.fdx_calc_force_cutoff(ctx.h, 0.5, 8, 64, 0.0, 0.05, F.FUSED), "cutoff")
    assert e.value.code == F.EINVAL
