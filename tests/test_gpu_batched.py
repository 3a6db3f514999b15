"""GPU: kernel shapes, persistent per-XCD queues, autotuner, and batched ensembles with
HIP-graph-captured leapfrog steps, against the oracle and the eager path."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

from parity_util import F32_RMS_REL_VS_TREE, F64_MAX_REL, rel_err, tree_ref

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


def _ref_forces(ps, n_leaf, n_group, theta, quad):
    t, g, lists = tree_ref(ps, n_leaf, n_group, theta)
    ref_sorted = lists.force(quad)
    ref = np.empty_like(ref_sorted)
    ref[t.perm.astype(np.int64)] = ref_sorted
    return ref


def test_every_shape_and_the_persistent_queue(ctx, fdx):
    ps = I.clustered(n_background=12000, n_clusters=6, n_per_cluster=1500, seed=12)
    _say(f"[shapes] n={ps.n}")
    ref = _ref_forces(ps, 8, 200, 0.5, True)
    ctx.set_particles(ps)
    for shape in range(ctx.lib.fdx_autotune_shapes()):
        ctx.set_shape(shape)
        for fp32 in (False, True):
            ctx.calc_force(0.5, 8, 200, 0.0, quad=True, fp32=fp32)
            a = ctx.forces()
            ctx.calc_force(0.5, 8, 200, 0.0, quad=True, fp32=fp32, persistent=True)
            ap = ctx.forces()
            # the same per-group code runs whichever workgroup picks the group up
            assert np.array_equal(a, ap)
            e = rel_err(a, ref)
            if fp32:
                assert np.sqrt(np.mean(e ** 2)) <= F32_RMS_REL_VS_TREE
            else:
                assert e.max() <= F64_MAX_REL
    ctx.set_shape(-1)


def test_every_shape_with_a_page_exact_particle_array(fdx):
    # 2^16 particles: the sorted particle records (32 B each) fill exactly 2 MiB, so nothing
    # lies behind the last one; the last group holds 3 particles, so a shape with two
    # i-particles per lane has slots past the group's end in it.  Every shape, direct and
    # persistent, FP32 and FP64, agrees with the oracle tree; a kernel that read a slot past
    # the group would read past the array here.
    ps = I.clustered(n_background=(1 << 16) - 8 * 2000, n_clusters=8, n_per_cluster=2000,
                     seed=44, eps=0.01)
    t = O.build_tree(ps, 8)
    g = O.make_groups(t, 200)
    assert ps.n == 1 << 16 and int(g.count[-1]) % 2 == 1
    ref = _ref_forces(ps, 8, 200, 0.5, True)
    with fdx.Context(0) as c:                   # a fresh context: buffers sized exactly
        c.set_particles(ps)
        for shape in range(c.lib.fdx_autotune_shapes()):
            c.set_shape(shape)
            _say(f"[page-exact] shape {c.shape_name(shape)}")
            for fp32 in (False, True):
                c.calc_force(0.5, 8, 200, 0.0, quad=True, fp32=fp32)
                a = c.forces()
                c.calc_force(0.5, 8, 200, 0.0, quad=True, fp32=fp32, persistent=True)
                assert np.array_equal(a, c.forces())
                e = rel_err(a, ref)
                if fp32:
                    assert np.sqrt(np.mean(e ** 2)) <= F32_RMS_REL_VS_TREE
                else:
                    assert e.max() <= F64_MAX_REL
                assert np.allclose(a[:, 3], ref[:, 3], rtol=1e-4 if fp32 else 1e-9, atol=0)


def test_autotuner_picks_a_measured_candidate(ctx, fdx):
    ps = I.plummer(60000, seed=13, eps=1 / 256)
    ctx.set_particles(ps)
    flags = fdx.Context.flags(quad=True, fp32=True)
    cand = [64, 128, 256, 512]
    bg, bv, times = ctx.autotune(0.5, 8, 0.0, flags, cand, reps=2)
    _say("[autotune] times (ms) per n_group x shape:\n", np.round(times, 3), "best", bg, bv)
    assert bg in cand and 0 <= bv < times.shape[1]
    assert np.nanmin(times) == times[cand.index(bg), bv]
    assert np.isnan(times[cand.index(512), 0])           # shape 0 holds at most 256
    ctx.calc_force(0.5, 8, bg, 0.0, quad=True, fp32=True)
    assert ctx.stats()["shape"] == bv                     # the FP32 choice is in use
    # tuning the FP32 kernel leaves the FP64 kernel's shape at its default
    ctx.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=False)
    s64 = ctx.stats()["shape"]
    ctx.set_shape(-1)
    ctx.calc_force(0.5, 8, 256, 0.0, quad=True, fp32=False)
    assert ctx.stats()["shape"] == s64
    ctx.set_shape(-1)


def test_autotuner_times_graph_steps_without_moving_particles(ctx, fdx):
    ens = I.ensemble(n_sys=8, seed=42, nmin=256, nmax=2048)
    ctx.set_particles(ens)
    flags = fdx.Context.flags(quad=True, fp32=True, persistent=True) | fdx.GRAPH
    cand = [64, 128]
    bg, bv, times = ctx.autotune(0.6, 8, 0.0, flags, cand, reps=2)
    _say("[autotune graph] times (ms):\n", np.round(times, 3), "best", bg, bv)
    assert bg in cand and np.nanmin(times) == times[cand.index(bg), bv]
    # the timed steps had dt = 0: positions and velocities are the input's, bit for bit
    x = ctx.particles()
    for a, b in zip(x, (ens.x, ens.y, ens.z, ens.vx, ens.vy, ens.vz)):
        assert np.array_equal(a, b)
    ctx.set_shape(-1)


def test_autotuner_records_and_reuses_its_choice(ctx, fdx, tmp_path):
    ps = I.plummer(20000, seed=14, eps=1 / 256)
    ctx.set_particles(ps)
    flags = fdx.Context.flags(quad=True, fp32=True)
    path = tmp_path / "autotune.jsonl"
    path.write_text("not a record\n")                  # unparsable lines are ignored
    bg, bv, hit = ctx.autotune_cached(path, 0.5, 8, 0.0, flags, [64, 256], reps=1)
    assert not hit and bg in (64, 256)
    lines = path.read_text().splitlines()
    assert len(lines) == 2 and f'"n_group": {bg}, "shape": {bv}}}' in lines[1]
    ctx.set_shape(-1)
    bg2, bv2, hit2 = ctx.autotune_cached(path, 0.5, 8, 0.0, flags, [64, 256], reps=1)
    assert hit2 and (bg2, bv2) == (bg, bv)
    ctx.calc_force(0.5, 8, bg2, 0.0, quad=True, fp32=True)
    assert ctx.stats()["shape"] == bv2                   # the recorded shape is in use
    # another opening angle is another key: measured and appended
    _, _, hit3 = ctx.autotune_cached(path, 0.7, 8, 0.0, flags, [64, 256], reps=1)
    assert not hit3 and len(path.read_text().splitlines()) == 3
    with pytest.raises(fdx.FdxError):
        ctx.autotune_cached(tmp_path / "missing_dir" / "x.jsonl", 0.4, 8, 0.0, flags, [64])
    ctx.set_shape(-1)


def _list_sets(lists):
    ne, ns, epj, spj = lists
    oe = np.concatenate([[0], np.cumsum(ne.astype(np.int64))])
    os_ = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    return ne, ns, [np.sort(epj[oe[k]:oe[k + 1]]) for k in range(len(ne))], \
        [np.sort(spj[os_[k]:os_[k + 1]]) for k in range(len(ns))]


def test_graph_steps_match_eager_steps_on_an_ensemble(ctx, fdx):
    """Several systems: the captured step sizes list segments by the system-size bound and
    fills them in one walk; particles, forces and every list equal the eager steps' (count
    walk, then fill)."""
    ens = I.ensemble(n_sys=24, seed=40, nmin=256, nmax=4096)
    _say(f"[graph] ensemble n={ens.n} systems={ens.n_sys}")
    dt, steps = 1.0 / 256.0, 6
    runs = {}
    for graph in (False, True):
        ctx.set_particles(ens)
        ctx.calc_force(0.6, 8, 128, 0.0, quad=True, fp32=True, persistent=True)
        ctx.integrate(dt, steps, graph=graph)
        runs[graph] = (ctx.particles(), ctx.forces(), _list_sets(ctx.lists()))
    for a, b in zip(runs[False][0], runs[True][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(runs[False][1], runs[True][1])
    (ne0, ns0, e0, s0), (ne1, ns1, e1, s1) = runs[False][2], runs[True][2]
    assert np.array_equal(ne0, ne1) and np.array_equal(ns0, ns1)
    assert all(np.array_equal(a, b) for a, b in zip(e0, e1))
    assert all(np.array_equal(a, b) for a, b in zip(s0, s1))


@pytest.mark.parametrize("shape", ["nt256_ipl2", "nt512_ipl2"])
def test_graph_steps_match_eager_steps_in_two_per_lane_shapes(ctx, fdx, shape):
    """The shapes the autotuner picks for the ensemble and the N = 2^24 benchmark (two
    i-particles per lane) in captured steps: particles and forces equal the eager steps'."""
    ens = I.ensemble(n_sys=24, seed=41, nmin=256, nmax=4096)
    names = [ctx.shape_name(v) for v in range(ctx.lib.fdx_autotune_shapes())]
    _say(f"[graph] shape {shape}, ensemble n={ens.n} systems={ens.n_sys}")
    dt, steps = 1.0 / 256.0, 5
    runs = {}
    try:
        ctx.set_shape(names.index(shape))
        for graph in (False, True):
            ctx.set_particles(ens)
            ctx.calc_force(0.6, 8, 128, 0.0, quad=True, fp32=True, persistent=True)
            assert ctx.stats()["shape"] == names.index(shape)
            ctx.integrate(dt, steps, graph=graph)
            runs[graph] = (ctx.particles(), ctx.forces())
    finally:
        ctx.set_shape(-1)
    for a, b in zip(runs[False][0], runs[True][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(runs[False][1], runs[True][1])


@pytest.mark.parametrize("percent", [0, 50])
def test_graph_list_sizing_and_recovery(ctx, fdx, percent):
    """percent 0: a count walk sizes the lists in every captured step; 50: the first capture's
    segments are too short for the longest lists, which move to the list buffer's spare space
    inside the walk (or, where that runs out, the step is redone eagerly and captured again
    with a doubled percentage).  Either way the steps equal the eager ones."""
    ens = I.ensemble(n_sys=12, seed=41, nmin=256, nmax=2048)
    dt, steps = 1.0 / 256.0, 4
    runs = {}
    for graph in (False, True):
        ctx.set_particles(ens)
        ctx.set_graph_list_margin(percent if graph else 200)
        ctx.calc_force(0.6, 8, 64, 0.0, quad=True, fp32=True, persistent=True)
        ctx.integrate(dt, steps, graph=graph)
        st = ctx.stats()
        runs[graph] = (ctx.particles(), ctx.forces(), st["graph_recoveries"], st["list_spills"])
    for a, b in zip(runs[False][0], runs[True][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(runs[False][1], runs[True][1])
    _say(f"[graph] percent {percent}: recoveries {runs[True][2]}, spilled lists {runs[True][3]}")
    if percent == 50:
        # short segments: lists moved to the spare space inside the walk, or steps redone
        assert runs[True][2] + runs[True][3] > runs[False][2] + runs[False][3]
    ctx.set_graph_list_margin(200)
    with pytest.raises(fdx.FdxError):
        ctx.set_graph_list_margin(-1)


def test_graph_steps_with_many_lists_moved_to_spare_space(fdx):
    """A fresh context runs the 50 % case twice.  In the second run the list buffer, grown by
    the first run's eager redo, has room for every list that outgrows its segment, so hundreds
    of groups per step are walked again in the spare space inside graph replays (for runs of
    groups that share the upper tree, the run's first walk is repeated into the new space).
    Every step equals the eager one bit for bit."""
    ens = I.ensemble(n_sys=12, seed=41, nmin=256, nmax=2048)
    dt, steps = 1.0 / 256.0, 4
    with fdx.Context(0) as c:
        for rep in range(2):
            runs = {}
            for graph in (False, True):
                c.set_particles(ens)
                c.set_graph_list_margin(50 if graph else 200)
                c.calc_force(0.6, 8, 64, 0.0, quad=True, fp32=True, persistent=True)
                s0 = c.stats()["list_spills"]
                c.integrate(dt, steps, graph=graph)
                st = c.stats()
                runs[graph] = ([a.copy() for a in c.particles()], c.forces(),
                               st["list_spills"] - s0)
            _say(f"[graph spare space] run {rep}: lists walked again in spare space "
                 f"{runs[True][2]}")
            for a, b in zip(runs[False][0], runs[True][0]):
                assert np.array_equal(a, b), rep
            assert np.array_equal(runs[False][1], runs[True][1]), rep
        assert runs[True][2] > 100 * steps // 2         # the second run moved many lists


def test_ensemble_energy_and_force_error(ctx, fdx):
    ens = I.ensemble(n_sys=16, seed=50, nmin=512, nmax=4096)
    off = ens.offsets()
    ctx.set_particles(ens)
    ctx.calc_force(0.6, 8, 128, 0.0, quad=True, fp32=True, persistent=True)
    a = ctx.forces()
    # parity: against the oracle tree at the same theta = 0.6 (FP32 rounding only)
    ref = _ref_forces(ens, 8, 128, 0.6, True)
    assert np.sqrt(np.mean(rel_err(a, ref) ** 2)) <= F32_RMS_REL_VS_TREE
    # accuracy of the method at theta = 0.6 against FP64 direct sum, per system (the 1e-3 bar
    # is stated at theta = 0.5; at 0.6 the quadrupole tree error is a few 1e-3)
    d = O.direct(ens)
    errs = [O.rms_rel_error(a[off[s]:off[s + 1]], d[off[s]:off[s + 1]]) for s in range(ens.n_sys)]
    _say("[ensemble] per-system rms da/a:", np.round(errs, 6))
    assert max(errs) < 5e-3
    # per-system energy over 40 graph-captured steps of dt = 1/256
    def energies(pot, xs):
        x, y, z, vx, vy, vz = xs
        out = []
        for s in range(ens.n_sys):
            sl = slice(off[s], off[s + 1])
            K = 0.5 * np.sum(ens.m[sl] * (vx[sl] ** 2 + vy[sl] ** 2 + vz[sl] ** 2))
            W = 0.5 * np.sum(ens.m[sl] * pot[sl])
            out.append(K + W)
        return np.array(out)
    E0 = energies(a[:, 3], ctx.particles())
    ctx.integrate(1.0 / 256.0, 40, graph=True)
    E1 = energies(ctx.forces()[:, 3], ctx.particles())
    drift = np.abs((E1 - E0) / E0)
    _say("[ensemble] per-system |dE/E| after 40 steps:", np.round(drift, 7))
    assert drift.max() < 1e-3


def test_integrate_requires_a_force_first(ctx, fdx):
    c = fdx.Context(0)
    c.set_particles(I.plummer(100, seed=3, eps=0.02))
    with pytest.raises(fdx.FdxError) as ei:
        c.integrate(0.01, 1)
    assert ei.value.code == fdx.ESTATE
    c.close()
