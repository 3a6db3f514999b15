"""Seeded random configurations of the domain-level parts against the oracle: exchange lists
between random multisection cuts of random particle sets (counts and entry sets of every pair
bit-exact), and the multisection decomposition with random current domains (some empty),
random n_x n_y n_z, sample counts and costs (everything exact)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

from test_gpu_dd import _check as _check_dd

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


def _one(rng, n, seed):
    kind = int(rng.integers(0, 3))
    if kind == 0:
        return I.plummer(n, seed=seed, eps=0.01)
    if kind == 1:
        return I.uniform_cube(n, seed, 0.01)
    return I.clustered(n_background=n // 2, n_clusters=4, n_per_cluster=n // 8, seed=seed)


@pytest.mark.parametrize("seed", range(8))
def test_random_exchange_lists(ctx, seed):
    rng = np.random.default_rng(4000 + seed)
    dims = tuple(int(v) for v in rng.integers(1, 4, size=3))
    if np.prod(dims) < 2:
        dims = (2, 1, 1)
    ps = _one(rng, int(rng.integers(400, 6000)), 40 + seed)
    theta = float(rng.uniform(0.3, 1.0))
    n_leaf = int(rng.choice([1, 4, 8, 16]))
    dom, _ = I.multisection(ps, *dims)
    _say(f"[random exchange {seed}] n={ps.n} domains={dims} theta={theta:.3f} leaf={n_leaf}")
    t = O.build_tree(dom, n_leaf)
    L = O.exchange(t, theta)
    ctx.set_particles(dom)
    ctx.build_exchange_lists(theta, n_leaf)
    pairs, ne, ns, epj, spj = ctx.exchange_lists()
    assert pairs == L.pairs
    assert np.array_equal(ne, L.n_epj) and np.array_equal(ns, L.n_spj)
    oe = np.concatenate([[0], np.cumsum(ne)])
    os_ = np.concatenate([[0], np.cumsum(ns)])
    for k in range(len(pairs)):
        e_ref, s_ref = L.epj[L.epj_off[k]:L.epj_off[k + 1]], L.spj[L.spj_off[k]:L.spj_off[k + 1]]
        assert np.array_equal(np.sort(epj[oe[k]:oe[k + 1]]), np.sort(t.perm[e_ref]))
        assert np.array_equal(np.sort(spj[os_[k]:os_[k + 1]]), np.sort(s_ref))


@pytest.mark.parametrize("seed", range(8))
def test_random_decomposition(ctx, seed):
    rng = np.random.default_rng(5000 + seed)
    ps = _one(rng, int(rng.integers(200, 8000)), 50 + seed)
    # random current domains, possibly empty ones
    n_cur = int(rng.integers(1, 7))
    cuts = np.sort(rng.integers(0, ps.n + 1, size=n_cur - 1))
    ps.sys_off = np.concatenate([[0], cuts, [ps.n]]).astype(np.int64)
    dims = tuple(int(v) for v in rng.integers(1, 5, size=3))
    D = int(np.prod(dims))
    n_sample = int(rng.integers(D * (n_cur + 1), 20 * D * (n_cur + 1) + 1))
    cost = None if rng.integers(0, 2) else rng.uniform(0.1, 5.0, n_cur)
    k = O.dd_sample_counts(np.diff(ps.sys_off), cost, n_sample)
    if k.sum() < D:                            # too few samples: the call must refuse
        n_sample = 40 * D * (n_cur + 1)
    _say(f"[random dd {seed}] n={ps.n} current={n_cur} dims={dims} samples={n_sample} "
         f"cost={'given' if cost is not None else 'counts'}")
    ctx.set_particles(ps)
    _check_dd(ctx, ps, dims, n_sample, cost=cost, seed=seed)
