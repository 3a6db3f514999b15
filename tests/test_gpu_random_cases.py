"""Seeded random configurations of the whole path against the oracle: particle
distributions (Plummer, uniform cube, clustered, coarse lattice with coincident particles, two
far-apart clumps), one to three systems of ragged sizes, and random n_leaf, n_group, theta
and moment order.  Keys, order, cells, groups and every list bit-exact; FP64 forces within
the FP64 tolerance of the oracle's forces on the same lists; FP32 group-relative forces within
the per-particle bound that FP32 rounding of group-relative coordinates allows (it grows with
a group's extent over its pair separations: a small system of two far-apart clumps forms one
wide group) and within the FP32 tolerance (groups too wide for FP32 are handed to the FP64
kernel)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

from parity_util import (F32_RMS_REL_VS_TREE, F64_MAX_REL, F64_RMS_REL, check_groups,
                         check_lists, check_moments, check_tree, fp32_error_bound, random_case,
                         rel_err, tree_ref)

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


@pytest.mark.parametrize("seed", range(24))
def test_random_configuration(ctx, seed):
    ps, n_leaf, n_group, theta, quad = random_case(seed)
    _say(f"[random {seed}] n={ps.n} sys={ps.n_sys} leaf={n_leaf} group={n_group} "
         f"theta={theta:.3f} quad={quad}")
    t, g, lists = tree_ref(ps, n_leaf, n_group, theta)
    ref_sorted = lists.force(quad)
    ref = np.empty_like(ref_sorted)
    ref[t.perm.astype(np.int64)] = ref_sorted
    ok = np.linalg.norm(ref[:, :3], axis=1) > 0
    ctx.set_particles(ps)
    ctx.calc_force(theta, n_leaf, n_group, 0.0, quad=quad, fp32=False)
    check_tree(ctx.tree(), t)
    check_moments(ctx.tree()["mom"], t)
    check_groups(ctx.groups(), g)
    check_lists(ctx.lists(), lists)
    if ok.any():
        e = rel_err(ctx.forces()[ok], ref[ok])
        assert e.max() <= F64_MAX_REL and np.sqrt(np.mean(e ** 2)) <= F64_RMS_REL
    ctx.calc_force(theta, n_leaf, n_group, 0.0, quad=quad, fp32=True)
    if ok.any():
        e32 = rel_err(ctx.forces()[ok], ref[ok])
        bound = np.empty(ps.n)
        bound[t.perm.astype(np.int64)] = fp32_error_bound(t, g, lists, ref_sorted)
        bound = bound[ok]
        rms, brms = np.sqrt(np.mean(e32 ** 2)), np.sqrt(np.mean(bound ** 2))
        _say(f"  fp32 rms {rms:.2e} (bound rms {brms:.2e}), max ratio to bound "
             f"{np.max(e32 / bound):.2e}")
        assert np.all(e32 <= 1.5 * bound + 1e-6)
        assert rms <= F32_RMS_REL_VS_TREE      # groups too wide for FP32 run in FP64
