"""Time the SPH density (short-range neighbour lists + Wendland C6 density, FP64) on one GPU:
a uniform cube of N particles with a support radius of `k` mean interparticle distances
(about (4/3) pi k^3 neighbours; the paper's SPH run uses k = 4.2, about 300), in the given
cutoff mode (fixed, or per-particle radii drawn uniformly within +-10 % for the others).

  python -m paper_1601_03138_amd.sph_timing [--log2n 24] [--k 4.2] [--mode 0] [--reps 5]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import fdx, inputs


def workload(log2n: int, k: float, mode: int, seed: int = 61):
    n = 1 << log2n
    ps = inputs.uniform_cube(n, seed, 1e-3)
    spacing = n ** (-1.0 / 3.0)
    r_cut = k * spacing
    h = None
    if mode != fdx.CUT_FIXED:
        h = r_cut * np.random.default_rng(seed + 1).uniform(0.9, 1.1, n)
    return ps, r_cut, h


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--k", type=float, default=4.2)
    ap.add_argument("--mode", type=int, default=0)
    ap.add_argument("--n-group", type=int, default=64)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    ps, r_cut, h = workload(args.log2n, args.k, args.mode)
    ctx = fdx.Context(0)
    ctx.set_particles(ps)
    rows = []
    for r in range(args.reps + 1):
        ctx.calc_density(args.mode, r_cut, h, n_group=args.n_group, timing=True)
        st = ctx.stats()
        print(f"[sph] call {r}: walk {st['t_walk']:.3f} ms, density {st['t_force']:.3f} ms, "
              f"total {st['t_total']:.3f} ms", flush=True)
        if r:
            rows.append((st["t_walk"], st["t_force"], st["t_total"]))
    rho, n = ctx.density()
    med = np.median(np.array(rows), axis=0)
    print(json.dumps({"n": ps.n, "mode": args.mode, "k": args.k, "n_group": args.n_group,
                      "ms_walk": round(med[0], 3), "ms_density": round(med[1], 3),
                      "ms_total": round(med[2], 3), "mean_neighbours": round(float(n.mean()), 1),
                      "candidates": int(st["n_epj"]), "pair_tests": int(st["n_interactions_pp"])}),
          flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
