"""GPU exchange lists between domains (section "Exchange of particles and superparticles",
long-range mode) through the C ABI, against the oracle: the local trees bit-exact, every
pair's counts and entry sets bit-exact, the limiting cases, and the error codes."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

from parity_util import check_tree

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


def _compare(ctx, dom, theta, n_leaf=8):
    t = O.build_tree(dom, n_leaf)
    L = O.exchange(t, theta)
    ctx.set_particles(dom)
    ctx.build_exchange_lists(theta, n_leaf)
    check_tree(ctx.tree(), t)
    pairs, ne, ns, epj, spj = ctx.exchange_lists()
    assert pairs == L.pairs
    assert np.array_equal(ne, L.n_epj) and np.array_equal(ns, L.n_spj)
    oe = np.concatenate([[0], np.cumsum(ne)])
    os_ = np.concatenate([[0], np.cumsum(ns)])
    for k in range(len(pairs)):
        e_ref, s_ref = L.epj[L.epj_off[k]:L.epj_off[k + 1]], L.spj[L.spj_off[k]:L.spj_off[k + 1]]
        assert np.array_equal(np.sort(epj[oe[k]:oe[k + 1]]), np.sort(t.perm[e_ref]))
        assert np.array_equal(np.sort(spj[os_[k]:os_[k + 1]]), np.sort(s_ref))
    st = ctx.exchange_stats()
    assert st["n_domains"] == dom.n_sys and st["n_pairs"] == len(pairs)
    assert st["n_epj"] == L.n_epj.sum() and st["n_spj"] == L.n_spj.sum()
    return t, L, st


@pytest.mark.parametrize("shape,theta", [((2, 2, 2), 0.5), ((3, 2, 2), 0.7), ((4, 1, 1), 0.3)])
def test_lists_match_the_oracle(ctx, shape, theta):
    ps = I.clustered(n_background=12000, n_clusters=6, n_per_cluster=1500, seed=31)
    dom, _ = I.multisection(ps, *shape)
    _say(f"[exchange] n={ps.n} domains={dom.n_sys} theta={theta}")
    _, L, st = _compare(ctx, dom, theta)
    _say(f"  entries {int((L.n_epj + L.n_spj).sum())}, ms tree {st['ms_tree']:.3f} "
         f"lists {st['ms_lists']:.3f}")


def test_ragged_domains_and_small_leaves(ctx):
    sets = [I.plummer(n, seed=40 + k, eps=0.02) for k, n in enumerate([1, 2, 5, 300, 2049])]
    for k, s in enumerate(sets):
        s.x += 3.0 * k                                  # side by side, some overlap in y, z
    _compare(ctx, I.concat(sets), 0.6, n_leaf=1)


def test_limiting_cases(ctx):
    a = I.plummer(3000, seed=5, eps=0.01)
    b = I.plummer(2000, seed=6, eps=0.01)
    b.x += 1000.0
    t, L, _ = _compare(ctx, I.concat([a, b]), 0.5)
    _, ne, ns, epj, spj = ctx.exchange_lists()
    assert ne.tolist() == [0, 0] and spj.tolist() == [0, 1]        # the roots
    c = I.uniform_cube(1500, 8, 0.01)
    d = I.uniform_cube(1200, 9, 0.01)
    d.x[:2], d.y[:2], d.z[:2] = [-0.6, 0.6], [-0.6, 0.6], [-0.6, 0.6]
    _compare(ctx, I.concat([c, d]), 1.0)
    _, ne, ns, epj, spj = ctx.exchange_lists()
    assert ns[0] == 0 and np.array_equal(np.sort(epj[:ne[0]]), np.arange(1500))


def test_exchange_errors(ctx, fdx):
    c = fdx.Context(0)
    with pytest.raises(fdx.FdxError) as ei:
        c.build_exchange_lists(0.5)
    assert ei.value.code == fdx.ESTATE
    c.set_particles(I.plummer(1000, seed=1, eps=0.01))          # one domain
    with pytest.raises(fdx.FdxError) as ei:
        c.build_exchange_lists(0.5)
    assert ei.value.code == fdx.EINVAL
    two = I.concat([I.plummer(500, seed=2, eps=0.01), I.plummer(400, seed=3, eps=0.01)])
    c.set_particles(two)
    for bad in (0.0, 1.5, float("nan")):
        with pytest.raises(fdx.FdxError) as ei:
            c.build_exchange_lists(bad)
        assert ei.value.code == fdx.EINVAL
    with pytest.raises(fdx.FdxError) as ei:
        c.exchange_counts()
    assert ei.value.code == fdx.ESTATE
    c.build_exchange_lists(0.5)
    ne, ns = c.exchange_counts()
    assert ne[0, 0] == 0 and ne[1, 1] == 0 and (ne + ns)[0, 1] > 0
    c.set_particles(two)                                        # lists are now stale
    with pytest.raises(fdx.FdxError) as ei:
        c.exchange_lists()
    assert ei.value.code == fdx.ESTATE
    c.close()
