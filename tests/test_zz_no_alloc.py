"""GPU: fdx_calc_force_noalloc, the evaluation that allocates nothing (every buffer carved from
one static device array), against fdx_calc_force with the same parameters: forces bit-identical
on two calls in a row, the second with a smaller input (the array keeps the first call's
contents), both precisions and launches; the FP64 result also against the oracle tree; limits
and errors."""
import sys

import numpy as np
import pytest

from paper_1601_03138_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(ps):
    import torch
    return {k: torch.tensor(np.ascontiguousarray(getattr(ps, k)), dtype=torch.float64,
                            device="cuda") for k in ("x", "y", "z", "m", "eps")}


def _noalloc(F, ps, theta, n_leaf, n_group, flags, eps_arr=True):
    import torch
    t = _dev(ps)
    out = [torch.full((ps.n,), float("nan"), dtype=torch.float64, device="cuda")
           for _ in range(4)]
    F.calc_force_noalloc(0, torch.cuda.current_stream(), t["x"], t["y"], t["z"], t["m"],
                         t["eps"] if eps_arr else None, float(ps.eps[0]), theta, n_leaf, n_group,
                         flags, *out)
    torch.cuda.synchronize()
    return np.stack([o.cpu().numpy() for o in out], axis=1)


def _context(F, ps, theta, n_leaf, n_group, flags, eps_arr=True):
    with F.Context(0) as ctx:
        ctx.set_particles(ps, per_particle_eps=eps_arr)
        ctx.calc_force_flags(theta, n_leaf, n_group, float(ps.eps[0]), flags)
        return ctx.forces()


def test_noalloc_equals_calc_force_on_two_calls_in_a_row():
    from paper_1601_03138_amd import fdx as F
    cases = [
        # (particles, theta, n_leaf, n_group, flags, per-particle eps)
        (I.plummer(120000, seed=61, eps=1.0 / 256.0), 0.5, 8, 256,
         F.QUAD | F.FP32REL | F.PERSISTENT, True),
        (I.clustered(n_background=20000, n_clusters=6, n_per_cluster=3001, seed=62, eps=1e-3),
         0.6, 8, 64, F.QUAD, False),
        (I.plummer(5003, seed=63, eps=1.0 / 64.0), 0.4, 4, 128, F.FP32REL, True),
    ]
    for k, (ps, theta, n_leaf, n_group, flags, ea) in enumerate(cases):
        _say(f"[noalloc] case {k}: n={ps.n} theta={theta} n_leaf={n_leaf} n_group={n_group} "
             f"flags={flags}")
        a = _noalloc(F, ps, theta, n_leaf, n_group, flags, ea)
        b = _context(F, ps, theta, n_leaf, n_group, flags, ea)
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), np.max(np.abs(a - b))


def test_noalloc_fp64_matches_oracle_tree(oracle_mod):
    from paper_1601_03138_amd import fdx as F
    O = oracle_mod
    ps = I.plummer(4096, seed=64, eps=1.0 / 64.0)
    a = _noalloc(F, ps, 0.5, 8, 64, F.QUAD)
    ref = O.tree_force(ps, 0.5, 8, 64, quad=True)
    rel = np.linalg.norm(a[:, :3] - ref[:, :3], axis=1) / np.linalg.norm(ref[:, :3], axis=1)
    _say(f"[noalloc] vs oracle tree: max rel {rel.max():.2e}")
    assert rel.max() < 1e-9
    assert np.allclose(a[:, 3], ref[:, 3], rtol=1e-9, atol=0)


def test_noalloc_limits_and_errors():
    import torch
    from paper_1601_03138_amd import fdx as F
    # beyond the particle limit
    big = I.plummer((1 << 17) + 1, seed=65, eps=0.01)
    with pytest.raises(F.FdxError) as e:
        _noalloc(F, big, 0.5, 8, 64, F.QUAD)
    assert e.value.code == F.EINVAL and "131072" in str(e.value)
    # flags it does not take
    small = I.plummer(1000, seed=66, eps=0.01)
    for fl in (F.PREDICTOR, F.TIMING, F.GRAPH):
        with pytest.raises(F.FdxError) as e:
            _noalloc(F, small, 0.5, 8, 64, F.QUAD | fl)
        assert e.value.code == F.EINVAL
    # lists that cannot fit the array: refused after the counting walk, nothing allocated
    at = I.plummer(1 << 17, seed=67, eps=0.01)
    with pytest.raises(F.FdxError) as e:
        _noalloc(F, at, 0.05, 8, 64, F.QUAD)
    assert e.value.code == F.ENOMEM and "entries" in str(e.value)
    # and a following call is unaffected
    a = _noalloc(F, small, 0.5, 8, 64, F.QUAD)
    b = _context(F, small, 0.5, 8, 64, F.QUAD)
    assert np.array_equal(a, b)
    # no particles: nothing to do
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    F.calc_force_noalloc(0, None, z, z, z, z, None, 0.01, 0.5, 8, 64, F.QUAD, z, z, z, z)
