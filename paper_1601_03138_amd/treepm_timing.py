"""Time the tree part of TreePM on one GPU: particles placed uniformly in the unit cube at rest
(the start of the paper's cosmological run), a cutoff of three widths of a mesh with N^(1/3)
cells per side, theta 0.5, monopole kernel with the S2 cutoff, FP32 group-relative.

  python -m paper_1601_03138_amd.treepm_timing [--log2n 24] [--n-group 256] [--reps 5]
                                                [--persistent] [--fp64]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import fdx, inputs


def workload(log2n: int, seed: int = 81):
    n = 1 << log2n
    ps = inputs.uniform_cube(n, seed, 0.5 / round(n ** (1.0 / 3.0)) / 20.0)
    mesh = round(n ** (1.0 / 3.0))
    return ps, 3.0 / mesh


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--n-group", type=int, default=256)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--persistent", action="store_true",
                    help="persistent force kernel over per-XCD queues (default: one workgroup "
                         "per group)")
    args = ap.parse_args()
    ps, r_cut = workload(args.log2n)
    ctx = fdx.Context(0)
    ctx.set_particles(ps)
    rows = []
    for r in range(args.reps + 1):
        ctx.calc_force_cutoff(args.theta, 8, args.n_group, 0.0, r_cut, fp32=not args.fp64,
                              persistent=args.persistent, timing=True)
        st = ctx.stats()
        print(f"[treepm] call {r}: walk {st['t_walk']:.3f} ms, force {st['t_force']:.3f} ms, "
              f"total {st['t_total']:.3f} ms", flush=True)
        if r:
            rows.append((st["t_walk"], st["t_force"], st["t_total"]))
    med = np.median(np.array(rows), axis=0)
    inter = int(st["n_interactions_pp"] + st["n_interactions_pc"])
    print(json.dumps({"n": ps.n, "r_cut": r_cut, "theta": args.theta, "n_group": args.n_group,
                      "fp32": not args.fp64, "persistent": args.persistent, "ms_walk": round(med[0], 3),
                      "ms_force": round(med[1], 3), "ms_total": round(med[2], 3),
                      "interactions": inter, "epj": int(st["n_epj"]), "spj": int(st["n_spj"]),
                      "particles_per_s": round(ps.n / (med[2] / 1e3), -5)}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
