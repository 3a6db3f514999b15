"""Seeded random configurations of the predicted single-pass walk against the exact two-pass
walk: Plummer, clustered or multi-system inputs, random n_group and theta, and a margin that
scales every predicted capacity by 0.2 to 2 around a network trained here on inputs of the
same kinds (capacities never exceed the system size, which bounds every list), so that lists
outgrow their segments in various proportions.  A fresh context (small list buffer: outgrown
lists mostly take the host's exact re-walk) or one that already holds the exact walk's buffer
(spare space takes them inside the walk).  Forces and every list must be bit-identical to
the exact walk."""
import math
import sys

import numpy as np
import pytest

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
def weights(fdx, tmp_path_factory):
    """A network trained on exact list lengths of inputs like the cases below."""
    c = fdx.Context(0)
    try:
        Xs, ts = [], []
        rng = np.random.default_rng(7500)
        for k in range(6):
            ps = _input(rng, 750 + k)
            c.set_particles(ps)
            c.calc_force(0.55, 8, int(rng.choice([64, 128, 256])), 0.0, quad=True, fp32=True)
            ne, ns, _, _ = c.lists()
            Xs.append(c.predictor_features())
            ts.append(np.log(ne.astype(np.float64) + ns).astype(np.float32))
        c.predictor_train(np.concatenate(Xs), np.concatenate(ts), epochs=30, batch=512, lr=3e-3,
                          seed=5)
        path = str(tmp_path_factory.mktemp("pred") / "w.bin")
        c.predictor_save(path)
    finally:
        c.close()
    return path


def _input(rng, seed):
    kind = int(rng.integers(0, 3))
    if kind == 0:
        return I.plummer(int(rng.integers(2000, 30001)), seed=seed, eps=1 / 256)
    if kind == 1:
        return I.clustered(n_background=int(rng.integers(4000, 20001)), n_clusters=4,
                           n_per_cluster=int(rng.integers(500, 3001)), seed=seed)
    return I.concat([I.plummer(int(rng.integers(200, 4001)), seed=seed * 10 + s, eps=0.02)
                     for s in range(int(rng.integers(2, 6)))])


@pytest.mark.parametrize("seed", range(8))
def test_random_predicted_walk_equals_exact(fdx, weights, seed):
    rng = np.random.default_rng(7000 + seed)
    ps = _input(rng, 70 + seed)
    n_group = int(rng.choice([64, 128, 256]))
    theta = float(rng.uniform(0.35, 0.8))
    scale = float(rng.choice([0.2, 0.5, 1.0, 2.0]))
    fresh = bool(rng.integers(0, 2))
    _say(f"[random predictor {seed}] n={ps.n} systems={ps.n_sys} group={n_group} "
         f"theta={theta:.3f} capacity scale={scale} fresh={fresh}")
    c = fdx.Context(0)
    try:
        c.set_particles(ps)
        c.calc_force(theta, 8, n_group, 0.0, quad=True, fp32=True)
        a_exact, l_exact = c.forces(), c.lists()
        p = fdx.Context(0) if fresh else c
        try:
            p.predictor_load(weights)
            p.predictor_margin(p.predictor_margin() + math.log(scale))
            p.set_particles(ps)
            p.calc_force(theta, 8, n_group, 0.0, quad=True, fp32=True, predictor=True)
            st = p.stats()
            a_pred, l_pred = p.forces(), p.lists()
        finally:
            if fresh:
                p.close()
    finally:
        c.close()
    _say(f"  overflow groups {st['overflow_groups']} of {st['n_groups']}, "
         f"walked again in spare space {st['list_spills']}")
    if scale <= 0.2:
        assert st["overflow_groups"] > 0
    assert np.array_equal(a_pred, a_exact)
    for u, v in zip(l_pred, l_exact):
        assert np.array_equal(u, v)
