"""Time the exchange lists between domains on one GPU: a workload cut into k x k x k
equal-count domains (virtual processes), the local trees and every pair's list built by
fdx_build_exchange_lists, repeated; prints the device times of each call and one summary
line.

  python -m paper_1601_03138_amd.exchange_timing [--workload clustered16m] [--k 4]
         [--theta 0.5] [--reps 5]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import fdx, inputs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="clustered16m")
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--n-leaf", type=int, default=8)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    ps = inputs.workload(args.workload)
    dom, _ = inputs.multisection(ps, args.k, args.k, args.k)
    ctx = fdx.Context(0)
    ctx.set_particles(dom)
    rows = []
    for r in range(args.reps + 1):
        ctx.build_exchange_lists(args.theta, args.n_leaf)
        st = ctx.exchange_stats()
        print(f"[exchange] call {r}: trees {st['ms_tree']:.3f} ms, lists {st['ms_lists']:.3f} ms",
              flush=True)
        if r:
            rows.append((st["ms_tree"], st["ms_lists"]))
    med = np.median(np.array(rows), axis=0)
    print(json.dumps({"workload": args.workload, "domains": args.k ** 3, "theta": args.theta,
                      "entries": int(st["n_epj"] + st["n_spj"]),
                      "list_capacity": int(st["list_capacity"]),
                      "ms_trees": round(float(med[0]), 3), "ms_lists": round(float(med[1]), 3),
                      "entries_per_s": float(round((st["n_epj"] + st["n_spj"])
                                                   / (med[1] / 1e3), -6))}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
