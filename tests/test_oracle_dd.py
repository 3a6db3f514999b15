"""Pins of the oracle's multisection domain decomposition with cost-weighted sampling
(section "Domain decomposition"): the generator against its published outputs, the sample
mapping against closed forms, the division against library order statistics and brute-force
box counts, the assignment against brute-force box membership, the exchange against a plain
loop, and the load balance the method is for (uniform and cost-weighted)."""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden_splitmix():
    rows = []
    for line in open(os.path.join(HERE, "golden", "splitmix64.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 0) for t in line.split()]
        rows.append((v[0], v[1:]))
    return rows


def test_splitmix64_published_outputs():
    rows = _golden_splitmix()
    assert len(rows) == 2
    for seed, outs in rows:
        assert [O.splitmix64(seed, k) for k in range(len(outs))] == outs


def test_sample_mapping_closed_forms():
    # one particle: every sample is it; 2^k particles: the top k bits of the generator output
    off = np.array([0, 1, 1 + 1024], np.int64)
    k = np.array([50, 300], np.int64)
    idx = O.dd_sample(off, k, seed=99)
    assert np.all(idx[:50] == 0)
    for s in range(50, 350):
        assert idx[s] == 1 + (O.splitmix64(99, s) >> 54)


def test_sample_range_and_uniformity():
    off = np.array([0, 10, 10, 25], np.int64)          # an empty domain in the middle
    k = np.array([100000, 0, 30000], np.int64)
    idx = O.dd_sample(off, k, seed=5).astype(np.int64)
    a, b = idx[:100000], idx[100000:]
    assert a.min() >= 0 and a.max() < 10 and b.min() >= 10 and b.max() < 25
    h = np.bincount(a, minlength=10)
    chi2 = float(np.sum((h - 10000.0) ** 2 / 10000.0))
    assert chi2 < 40.0                                   # 9 dof, p < 1e-5
    assert not np.array_equal(idx, O.dd_sample(off, k, seed=6))


def test_sample_counts_follow_cost():
    assert list(O.dd_sample_counts([10, 10, 10], None, 100)) == [33, 33, 33]
    assert list(O.dd_sample_counts([10, 10, 10], [1.0, 2.0, 1.0], 100)) == [25, 50, 25]
    assert list(O.dd_sample_counts([5, 0, 5], [3.0, 7.0, 1.0], 1100)) == [300, 0, 100]
    assert list(O.dd_sample_counts([30, 10], None, 1000)) == [750, 250]


def test_division_median_and_quantiles():
    rng = np.random.default_rng(1)
    x = rng.normal(size=1000)
    bx, by, bz, cell = O.dd_multisection(x, rng.normal(size=1000), rng.normal(size=1000), 2, 1, 1)
    assert bx[0] == -np.inf and bx[2] == np.inf
    assert bx[1] == np.median(x)                         # midpoint of the middle pair
    assert np.all(by[:, 0] == -np.inf) and np.all(bz[..., -1] == np.inf)
    # nx = 5, 1000 samples: the cuts are the midpoint quantiles; y cuts per slab likewise
    y = rng.uniform(size=1000)
    bx, by, _, _ = O.dd_multisection(x, y, np.zeros(1000), 5, 4, 1)
    for i in range(1, 5):
        q = np.quantile(x, i / 5, method="midpoint")
        assert abs(bx[i] - q) <= 2 * np.spacing(abs(q))
    for a in range(5):
        ys = y[(x >= bx[a]) & (x < bx[a + 1])]
        assert len(ys) == 200
        for j in range(1, 4):
            q = np.quantile(ys, j / 4, method="midpoint")
            assert abs(by[a, j] - q) <= 2 * np.spacing(abs(q))


@pytest.mark.parametrize("K,dims", [(1000, (3, 4, 2)), (97, (2, 3, 5)), (24, (2, 3, 4))])
def test_division_equal_counts_by_brute_force(K, dims):
    nx, ny, nz = dims
    rng = np.random.default_rng(K)
    sx, sy, sz = rng.uniform(-1, 1, K), rng.uniform(-1, 1, K), rng.uniform(-1, 1, K)
    bx, by, bz, cell = O.dd_multisection(sx, sy, sz, nx, ny, nz)
    split = lambda m, n, i: (i * m) // n
    for a in range(nx):
        in_a = [s for s in range(K) if bx[a] <= sx[s] < bx[a + 1]]
        assert len(in_a) == split(K, nx, a + 1) - split(K, nx, a)
        for c in range(ny):
            in_c = [s for s in in_a if by[a, c] <= sy[s] < by[a, c + 1]]
            assert len(in_c) == split(len(in_a), ny, c + 1) - split(len(in_a), ny, c)
            for e in range(nz):
                in_e = [s for s in in_c if bz[a, c, e] <= sz[s] < bz[a, c, e + 1]]
                assert len(in_e) == split(len(in_c), nz, e + 1) - split(len(in_c), nz, e)
                assert len(in_e) >= 1
                assert all(cell[s] == (a * ny + c) * nz + e for s in in_e)
    # the result does not depend on the order the samples come in (positions permuted)
    p = rng.permutation(K)
    bx2, by2, bz2, cell2 = O.dd_multisection(sx[p], sy[p], sz[p], nx, ny, nz)
    assert np.array_equal(bx, bx2) and np.array_equal(by, by2) and np.array_equal(bz, bz2)
    assert np.array_equal(cell[p], cell2)


def test_division_too_few_samples_and_single_domain():
    rng = np.random.default_rng(3)
    s = rng.uniform(size=(3, 11))
    with pytest.raises(ValueError):
        O.dd_multisection(s[0], s[1], s[2], 2, 3, 2)
    bx, by, bz, cell = O.dd_multisection(s[0][:1], s[1][:1], s[2][:1], 1, 1, 1)
    assert list(bx) == [-np.inf, np.inf] and np.all(cell == 0)


def test_assignment_by_brute_force_with_particles_on_faces():
    rng = np.random.default_rng(4)
    nx, ny, nz = 3, 2, 4
    s = rng.uniform(-1, 1, size=(3, 500))
    bx, by, bz, _ = O.dd_multisection(s[0], s[1], s[2], nx, ny, nz)
    x, y, z = rng.uniform(-1.5, 1.5, size=(3, 3000))
    x[:3] = bx[1]                   # on an x face: the upper slab
    y[3:6] = by[0, 1]
    z[6:9] = bz[1, 1, 2]
    dest = O.dd_assign(x, y, z, nx, ny, nz, bx, by, bz)
    for i in range(len(x)):
        hits = [(a * ny + c) * nz + e for a in range(nx) for c in range(ny) for e in range(nz)
                if bx[a] <= x[i] < bx[a + 1] and by[a, c] <= y[i] < by[a, c + 1]
                and bz[a, c, e] <= z[i] < bz[a, c, e + 1]]
        assert hits == [dest[i]]
    assert all(dest[i] // (ny * nz) == 1 for i in range(3))


def test_exchange_against_a_plain_loop():
    rng = np.random.default_rng(5)
    n_src, n_dom = 3, 5
    src = np.sort(rng.integers(0, n_src, 400))
    dest = rng.integers(0, n_dom, 400)
    order, counts, dom_off = O.dd_exchange(dest, src, n_dom, n_src)
    ref = [i for d in range(n_dom) for i in range(400) if dest[i] == d]
    assert list(order) == ref
    for p in range(n_src):
        for d in range(n_dom):
            assert counts[p, d] == sum(1 for i in range(400) if src[i] == p and dest[i] == d)
    assert list(dom_off) == [0] + list(np.cumsum([sum(dest == d) for d in range(n_dom)]))


def test_every_particle_sampled_once_reproduces_the_exact_multisection():
    # sampling each particle exactly once (counts divisible at every level) makes the division
    # the exact equal-count multisection of the particles themselves
    ps = I.plummer(64 * 50, seed=11, eps=0.01)
    bx, by, bz, cell = O.dd_multisection(ps.x, ps.y, ps.z, 4, 4, 4)
    dest = O.dd_assign(ps.x, ps.y, ps.z, 4, 4, 4, bx, by, bz)
    assert np.array_equal(dest, cell)
    dom, order = I.multisection(ps, 4, 4, 4)
    ref = np.empty(ps.n, np.int64)
    ref[order] = np.repeat(np.arange(64), np.diff(dom.offsets()))
    assert np.array_equal(dest.astype(np.int64), ref)


def test_uniform_cost_balances_particle_counts():
    ps = I.clustered(n_background=1 << 15, n_clusters=64, n_per_cluster=1 << 9, seed=12)
    D = O.decompose(ps, 3, 3, 3, 1 << 14, seed=1)
    n_d = np.diff(D.dom_off)
    assert n_d.sum() == ps.n and D.k.sum() == 1 << 14
    dev = n_d / (ps.n / 27.0) - 1.0
    assert np.max(np.abs(dev)) < 0.25 and np.mean(np.abs(dev)) < 0.06


def test_cost_weighted_sampling_balances_cost():
    # two current domains: x < 0 costs 3 per particle, x >= 0 costs 1; four slabs in x put
    # three of them in the costly half
    rng = np.random.default_rng(13)
    n = 1 << 16
    x = np.concatenate([rng.uniform(-1, 0, n // 2), rng.uniform(0, 1, n // 2)])
    y, z = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    ps = I.ParticleSet(x, y, z, 0 * x, 0 * x, 0 * x, np.full(n, 1.0 / n), np.full(n, 0.01),
                       np.array([0, n // 2, n], np.int64))
    D = O.decompose(ps, 4, 1, 1, 1 << 14, cost=[3.0 * (n // 2), 1.0 * (n // 2)], seed=2)
    assert list(D.k) == [3 << 12, 1 << 12]
    assert np.allclose(D.bx[1:4], [-2 / 3, -1 / 3, 0.0], atol=0.03)
    w = np.where(x < 0, 3.0, 1.0)
    cost = np.array([w[D.dest == d].sum() for d in range(4)])
    assert np.max(np.abs(cost / cost.mean() - 1.0)) < 0.1
    # without the cost the slabs hold equal particle counts instead
    U = O.decompose(ps, 4, 1, 1, 1 << 14, seed=2)
    assert np.allclose(U.bx[1:4], [-0.5, 0.0, 0.5], atol=0.03)


def test_factorisation_close_to_cube_root():
    for n, ref in ((1, (1, 1, 1)), (8, (2, 2, 2)), (27, (3, 3, 3)), (64, (4, 4, 4)),
                   (7, (7, 1, 1)), (12, (3, 2, 2)), (42, (7, 3, 2))):
        assert O.dd_factor(n) == ref
    for n in range(1, 200):
        nx, ny, nz = O.dd_factor(n)
        assert nx * ny * nz == n and nx >= ny >= nz >= 1
        c = round(n ** (1 / 3))
        if c ** 3 == n:
            assert (nx, ny, nz) == (c, c, c)
