"""GPU tree part of TreePM (monopole tree with the S2 cutoff) through the C ABI against the
oracle: lists bit-exact, FP64 forces to round-off, FP32 group-relative forces to the FP32
tolerance, accuracy against the cutoff direct sum, persistent == direct, no potential,
integration, argument errors."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

from parity_util import F32_RMS_REL_VS_TREE

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


def _glob(a, ref):
    return float(np.sqrt(np.mean(np.sum((a - ref) ** 2, axis=1)) / np.mean(np.sum(ref ** 2, axis=1))))


CASES = {
    "uniform": (lambda: I.uniform_cube(8192, 71, 1e-3), 3 / 32),
    "clustered": (lambda: I.clustered(n_background=6000, n_clusters=4, n_per_cluster=500,
                                      seed=72), 3 / 16),
}


@pytest.mark.parametrize("name", list(CASES))
def test_cutoff_lists_and_forces_match_the_oracle(ctx, name):
    make, r_cut = CASES[name]
    ps = make()
    t = O.build_tree(ps, 8)
    g = O.make_groups(t, 64)
    L = O.cutoff_lists(t, g, 0.5, r_cut)
    ref = np.empty((ps.n, 3))
    ref[t.perm.astype(np.int64)] = L.force()
    d = O.direct_cutoff(ps, r_cut)
    ctx.set_particles(ps)
    ctx.calc_force_cutoff(0.5, 8, 64, 0.0, r_cut)
    ne, ns, epj, spj = ctx.lists()
    assert np.array_equal(ne.astype(np.int64), L.n_epj) and np.array_equal(ns.astype(np.int64), L.n_spj)
    oe = np.concatenate([[0], np.cumsum(ne.astype(np.int64))])
    os_ = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    for k in range(g.n):
        e_ref, s_ref = L.group_lists(k)
        assert np.array_equal(np.sort(epj[oe[k]:oe[k + 1]]), np.sort(e_ref))
        assert np.array_equal(np.sort(spj[os_[k]:os_[k + 1]]), np.sort(s_ref))
    a64 = ctx.forces()
    assert np.all(a64[:, 3] == 0.0)
    e64 = _glob(a64[:, :3], ref)
    ctx.calc_force_cutoff(0.5, 8, 64, 0.0, r_cut, fp32=True)
    a32 = ctx.forces()
    e32 = _glob(a32[:, :3], ref)
    ctx.calc_force_cutoff(0.5, 8, 64, 0.0, r_cut, fp32=True, persistent=True)
    assert np.array_equal(ctx.forces(), a32)
    ed = _glob(a64[:, :3], d)
    _say(f"[treepm] {name}: fp64 vs tree {e64:.2e}, fp32 vs tree {e32:.2e}, vs direct {ed:.2e}")
    assert e64 <= 1e-12 and e32 <= F32_RMS_REL_VS_TREE and ed <= 3e-3


def test_cutoff_integration_and_errors(ctx, fdx):
    ps = I.uniform_cube(4096, 77, 1e-3)
    ctx.set_particles(ps)
    ctx.calc_force_cutoff(0.5, 8, 64, 0.0, 0.1, fp32=True)
    a0 = ctx.forces()
    ctx.integrate(1e-3, 2)
    x, y, z, vx, vy, vz = ctx.particles()
    assert np.all(np.isfinite(vx)) and np.any(vx != 0.0)
    assert not np.array_equal(ctx.forces(), a0)
    for kw in (dict(r_cut=0.0), dict(r_cut=float("inf"))):
        with pytest.raises(fdx.FdxError) as ei:
            ctx.calc_force_cutoff(0.5, 8, 64, 0.0, **kw)
        assert ei.value.code == fdx.EINVAL
    for fl in (fdx.QUAD, fdx.PREDICTOR, fdx.GRAPH):
        rc = ctx.lib.fdx_calc_force_cutoff(ctx.h, 0.5, 8, 64, 0.0, 0.1, fl)
        assert rc == fdx.EINVAL
    ctx.calc_force_cutoff(0.5, 8, 64, 0.0, 0.1)
    with pytest.raises(fdx.FdxError) as ei:
        ctx.integrate(1e-3, 1, graph=True)
    assert ei.value.code == fdx.EINVAL
