"""Time the multisection domain decomposition with cost-weighted sampling and the exchange of
particles on one GPU: the N = 2^24 clustered workload cut into k x k x k equal-count domains
(the current domains, one per virtual process), each costed by its interaction count in a
force evaluation of its own local tree, then decomposed into k x k x k new domains from
n_sample samples and exchanged.

  python -m paper_1601_03138_amd.dd_timing [--log2n 24] [--k 4] [--samples 1048576] [--reps 3]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import fdx, inputs

# algorithmic HBM bytes per particle: destinations (read x, y, z, write destination, grouping
# key and index) 40 + grouping sort, one 8-bit pass per byte of the destination (histogram
# reads the key, scatter reads and writes key and index) 32 each + run bounds (read key, order
# and the source domain) 16; exchange: read the order and 8 FP64 arrays (x, y, z, vx, vy, vz,
# m, eps), write the 8 arrays
def bytes_assign(domains: int) -> int:
    passes = max(1, ((domains - 1).bit_length() + 7) // 8) if domains > 1 else 0
    return 40 + 32 * passes + 16


BYTES_EXCHANGE = 4 + 64 + 64


def workload(log2n: int, k: int):
    ps = inputs.workload("clustered16m") if log2n == 24 else inputs.clustered(
        n_background=1 << (log2n - 1), n_clusters=64, n_per_cluster=1 << (log2n - 7), seed=3)
    dom, _ = inputs.multisection(ps, k, k, k)
    return dom


def run(dom, k: int, n_sample: int, reps: int, theta: float = 0.5, log=print) -> dict:
    ctx = fdx.Context(0)
    rows = []
    try:
        for r in range(reps + 1):
            ctx.set_particles(dom)
            ctx.calc_force(theta, 8, 256, 0.0, quad=True, fp32=True)
            t0 = time.perf_counter()
            ctx.decompose(k, k, k, n_sample, seed=r, cost_lists=True)
            ctx.exchange_particles()
            st = ctx.dd_stats()
            wall = (time.perf_counter() - t0) * 1e3
            log(f"[dd] call {r}: sample {st['ms_sample']:.3f} ms, divide {st['ms_divide']:.3f} "
                f"ms, assign {st['ms_assign']:.3f} ms, exchange {st['ms_exchange']:.3f} ms, "
                f"wall {wall:.3f} ms, moved {st['n_moved']}")
            if r:
                rows.append((st["ms_sample"], st["ms_divide"], st["ms_assign"],
                             st["ms_exchange"], wall))
        d = ctx.decomposition()
    finally:
        ctx.close()
    med = np.median(np.array(rows), axis=0)
    n = dom.n
    dev = float(med[0] + med[1] + med[2] + med[3])
    n_d = np.diff(d["dom_off"])
    gbs = lambda b, ms: round(float(b / (ms / 1e3) / 1e9), 1)
    return {"n": n, "current_domains": dom.n_sys, "domains": int(k ** 3),
            "n_sample": n_sample, "samples": int(st["n_samples"]),
            "cost": "interaction count of each current domain's last walk",
            "ms_sample": round(float(med[0]), 3), "ms_divide": round(float(med[1]), 3),
            "ms_assign": round(float(med[2]), 3), "ms_exchange": round(float(med[3]), 3),
            "ms_device_total": round(dev, 3), "ms_wall": round(float(med[4]), 3),
            "particles_per_s": float(round(n / (dev / 1e3), -5)),
            "assign_gbs": gbs(bytes_assign(k ** 3) * n, med[2]),
            "exchange_gbs": gbs(BYTES_EXCHANGE * n, med[3]),
            "moved": int(st["n_moved"]),
            "particles_per_domain_min_max": [int(n_d.min()), int(n_d.max())]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--samples", type=int, default=1 << 20)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    dom = workload(args.log2n, args.k)
    print(json.dumps(run(dom, args.k, args.samples, args.reps,
                         log=lambda m: print(m, flush=True))), flush=True)


if __name__ == "__main__":
    main()
