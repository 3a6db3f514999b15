"""GPU multisection domain decomposition with cost-weighted sampling (section "Domain
decomposition") through the C ABI, against the oracle: sample counts, sampled particles,
the faces of every division (FP64, bitwise), the domain of every sample, every particle's
destination, the exchange order, send counts and offsets -- all exact; costs from the last
walk; the particle exchange itself; ties, signed zeros, oversampling, the limiting cases and
the error codes."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

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


def _check(ctx, ps, dims, n_sample, cost=None, seed=0, cost_lists=False, oracle_cost=None):
    """Decompose on the GPU and compare everything with the oracle; returns the oracle's
    decomposition."""
    nx, ny, nz = dims
    ref = O.decompose(ps, nx, ny, nz, n_sample, cost=oracle_cost if cost_lists else cost,
                      seed=seed)
    ctx.decompose(nx, ny, nz, n_sample, cost=cost, seed=seed, cost_lists=cost_lists)
    k, idx, cell = ctx.dd_samples()
    assert np.array_equal(k, ref.k)
    assert np.array_equal(idx, ref.idx)
    assert np.array_equal(cell, ref.cell)
    d = ctx.decomposition()
    for f in ("bx", "by", "bz"):
        assert np.array_equal(d[f], getattr(ref, f)), f
        assert np.array_equal(np.signbit(d[f]), np.signbit(getattr(ref, f))), f
    dest, order = ctx.dd_destinations()
    assert np.array_equal(dest, ref.dest)
    assert np.array_equal(order, ref.order)
    assert np.array_equal(d["counts"], ref.counts)
    assert np.array_equal(d["dom_off"], ref.dom_off)
    st = ctx.dd_stats()
    assert st["n_samples"] == ref.k.sum() and st["n_domains"] == nx * ny * nz
    assert st["n_src"] == ps.n_sys
    return ref


@pytest.mark.parametrize("dims,n_sample,seed", [((3, 2, 2), 5000, 7), ((4, 4, 4), 9973, 1),
                                                 ((5, 1, 3), 40000, 2)])
def test_one_domain_uniform_sampling(ctx, dims, n_sample, seed):
    ps = I.plummer(50001, seed=21, eps=0.01)          # ragged against tiles and blocks
    _say(f"[dd] n={ps.n} dims={dims} samples={n_sample} seed={seed}")
    ctx.set_particles(ps)
    ref = _check(ctx, ps, dims, n_sample, seed=seed)
    n_d = np.diff(ref.dom_off)
    assert n_d.min() > 0


def test_many_sources_with_given_costs_and_an_empty_domain(ctx):
    ps = I.clustered(n_background=20000, n_clusters=8, n_per_cluster=2000, seed=22)
    dom, _ = I.multisection(ps, 2, 2, 2)
    # insert an empty current domain in the middle
    off = dom.offsets()
    dom.sys_off = np.concatenate([off[:4], off[3:]]).astype(np.int64)
    rng = np.random.default_rng(3)
    cost = rng.uniform(0.5, 4.0, dom.n_sys)
    _say(f"[dd] sources={dom.n_sys} (one empty), costs given")
    ctx.set_particles(dom)
    ref = _check(ctx, dom, (4, 3, 2), 20000, cost=cost, seed=11)
    assert ref.k[3] == 0
    st = ctx.dd_stats()
    diag = sum(ref.counts[p, p] for p in range(dom.n_sys))
    assert st["n_moved"] == dom.n - diag


def test_costs_from_the_last_walk(ctx):
    ps = I.clustered(n_background=16000, n_clusters=6, n_per_cluster=2000, seed=23)
    dom, _ = I.multisection(ps, 2, 2, 1)
    _say(f"[dd] cost from lists, sources={dom.n_sys}")
    t = O.build_tree(dom, 8)
    g = O.make_groups(t, 64)
    L = O.walk(t, g, 0.5)
    cost = np.zeros(dom.n_sys)
    per = g.count.astype(np.float64) * (L.n_epj + L.n_spj)
    np.add.at(cost, g.root.astype(np.int64), per)
    ctx.set_particles(dom)
    ctx.calc_force(0.5, 8, 64, 0.0, quad=True, fp32=True)
    ref = _check(ctx, dom, (2, 2, 2), 30000, seed=5, cost_lists=True, oracle_cost=cost)
    assert ref.k.sum() <= 30000 and not np.array_equal(
        ref.k, O.dd_sample_counts(np.diff(dom.offsets()), None, 30000))


def test_exchange_particles_and_a_second_decomposition(ctx, fdx):
    ps = I.plummer(30000, seed=24, eps=0.01)
    ps.vx[:] = np.arange(ps.n)                        # a tracer through the exchange
    ctx.set_particles(ps)
    ref = _check(ctx, ps, (2, 3, 2), 6000, seed=3)
    ctx.exchange_particles()
    x, y, z, vx, vy, vz = ctx.particles()
    o = ref.order.astype(np.int64)
    assert np.array_equal(x, ps.x[o]) and np.array_equal(vx, ps.vx[o])
    assert np.array_equal(vz, ps.vz[o])
    assert ctx.dd_stats()["ms_exchange"] > 0.0
    with pytest.raises(fdx.FdxError):
        ctx.exchange_particles()                      # already applied
    # the domains are now the systems: the next decomposition starts from them
    take = lambda a: np.ascontiguousarray(a[o])
    moved = I.ParticleSet(take(ps.x), take(ps.y), take(ps.z), take(ps.vx), take(ps.vy),
                          take(ps.vz), take(ps.m), take(ps.eps), ref.dom_off.copy())
    ref2 = _check(ctx, moved, (3, 2, 2), 6000, seed=4)
    assert ref2.counts.shape == (12, 12)
    # and the exchange lists run on them
    ctx.build_exchange_lists(0.5, 8)
    assert ctx.exchange_stats()["n_domains"] == 12


def test_ties_signed_zeros_and_oversampling(ctx):
    # coordinates on a coarse lattice (many equal values, both signs of zero) and more
    # samples than particles (every particle sampled several times)
    rng = np.random.default_rng(25)
    n = 3000
    x = rng.integers(-3, 4, n).astype(np.float64) * 0.5
    y = rng.integers(-2, 3, n).astype(np.float64)
    z = rng.integers(-1, 2, n).astype(np.float64)
    x[x == 0] = np.where(rng.uniform(size=int((x == 0).sum())) < 0.5, -0.0, 0.0)
    z[z == 0] = -0.0
    ps = I.ParticleSet(x, y, z, 0 * x, 0 * x, 0 * x, np.full(n, 1.0 / n), np.full(n, 0.1))
    ctx.set_particles(ps)
    _say("[dd] lattice with ties, K = 3n")
    _check(ctx, ps, (3, 3, 2), 3 * n, seed=9)


def test_limiting_cases(ctx):
    ps = I.plummer(4099, seed=26, eps=0.01)
    ctx.set_particles(ps)
    ref = _check(ctx, ps, (1, 1, 1), 100, seed=1)           # one domain: no cut
    assert np.all(ref.dest == 0) and np.array_equal(ref.order, np.arange(ps.n))
    _check(ctx, ps, (2, 3, 4), 24, seed=2)                  # exactly one sample per domain
    _check(ctx, ps, (7, 1, 1), 7000, seed=3)                # one axis only


def test_errors(ctx, fdx):
    ps = I.plummer(2000, seed=27, eps=0.01)
    ctx.set_particles(ps)
    with pytest.raises(fdx.FdxError):
        ctx.dd_stats()                                      # nothing decomposed yet
    with pytest.raises(fdx.FdxError):
        ctx.decompose(2, 2, 2, 7)                           # fewer samples than domains
    with pytest.raises(fdx.FdxError):
        ctx.decompose(0, 2, 2, 100)
    with pytest.raises(fdx.FdxError):
        ctx.decompose(2, 2, 2, 100, cost=[-1.0])
    with pytest.raises(fdx.FdxError):
        ctx.decompose(2, 2, 2, 100, cost=[0.0])             # zero total cost
    with pytest.raises(fdx.FdxError):
        ctx.decompose(2, 2, 2, 100, cost=[1.0], cost_lists=True)
    with pytest.raises(fdx.FdxError):
        ctx.decompose(4096, 4096, 2, 100000)                # too many pairs
    ctx.set_particles(ps)
    with pytest.raises(fdx.FdxError):
        ctx.decompose(2, 2, 2, 100, cost_lists=True)        # no walk on these particles
    ctx.decompose(2, 2, 2, 100)
    ctx.set_particles(ps)
    with pytest.raises(fdx.FdxError):
        ctx.decomposition()                                 # dropped by set_particles
