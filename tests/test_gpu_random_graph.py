"""Seeded random ensembles through graph-captured leapfrog steps against the same steps taken
eagerly: 2 to 12 systems of ragged sizes (Plummer spheres and clumps), random opening angle,
group size, moment order and list sizing of the captured step (count walk, or per-system
segments at 25 %, 100 % or 200 % of each system's longest list, with lists that outgrow them
walked again in spare space or the step redone).  Positions, velocities, forces and every
list must be bit-identical."""
import sys

import numpy as np
import pytest

from paper_1601_03138_amd import inputs as I

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


def _ensemble(rng, seed):
    sets = []
    for s in range(int(rng.integers(2, 13))):
        n = int(rng.integers(64, 4097))
        if rng.integers(0, 2):
            p = I.plummer(n, seed=seed * 100 + s, eps=float(4.0 / n ** (1 / 3)))
        else:
            p = I.plummer(n, seed=seed * 100 + s, eps=0.02)
            p.x[n // 2:] += 3.0                        # two clumps
        sets.append(p)
    return I.concat(sets)


def _lists(ctx):
    ne, ns, epj, spj = ctx.lists()
    oe = np.concatenate([[0], np.cumsum(ne.astype(np.int64))])
    os_ = np.concatenate([[0], np.cumsum(ns.astype(np.int64))])
    return (ne, ns, [np.sort(epj[oe[k]:oe[k + 1]]) for k in range(len(ne))],
            [np.sort(spj[os_[k]:os_[k + 1]]) for k in range(len(ns))])


@pytest.mark.parametrize("seed", range(8))
def test_random_graph_steps_equal_eager_steps(ctx, seed):
    rng = np.random.default_rng(6000 + seed)
    ps = _ensemble(rng, seed)
    theta = float(rng.uniform(0.4, 0.8))
    n_group = int(rng.choice([16, 64, 128]))
    quad = bool(rng.integers(0, 2))
    percent = int(rng.choice([0, 25, 100, 200]))
    steps = int(rng.integers(2, 5))
    _say(f"[random graph {seed}] n={ps.n} systems={ps.n_sys} theta={theta:.3f} "
         f"group={n_group} quad={quad} percent={percent} steps={steps}")
    runs = []
    for graph in (False, True):
        ctx.set_particles(ps)
        ctx.set_graph_list_margin(percent)
        ctx.calc_force(theta, 8, n_group, 0.0, quad=quad, fp32=True, persistent=True)
        ctx.integrate(1.0 / 256.0, steps, graph=graph)
        runs.append((ctx.particles(), ctx.forces(), _lists(ctx)))
    ctx.set_graph_list_margin(200)
    (x0, a0, l0), (x1, a1, l1) = runs
    for u, v in zip(x0, x1):
        assert np.array_equal(u, v)
    assert np.array_equal(a0, a1)
    assert np.array_equal(l0[0], l1[0]) and np.array_equal(l0[1], l1[1])
    assert all(np.array_equal(u, v) for u, v in zip(l0[2], l1[2]))
    assert all(np.array_equal(u, v) for u, v in zip(l0[3], l1[3]))
