"""Comparison helpers for GPU-vs-oracle parity tests (test infrastructure)."""
import numpy as np

import oracle as O

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
