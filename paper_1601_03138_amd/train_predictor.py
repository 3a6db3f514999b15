"""Train the learned list-length predictor on groups harvested from exact walks.

Harvest: for each training input (Plummer N = 2^20 and clustered N = 2^24 systems drawn
with seeds other than the evaluation seed), one exact force evaluation at the given theta and
n_group; per group the 8 raw features and ln(|EPJ| + |SPJ|).  Training runs on the GPU with
the library's own forward/backward/Adam kernels (fdx_predictor_train) and the weights are
saved with fdx_predictor_save.

  python -m paper_1601_03138_amd.train_predictor --out predictor.bin [--n-group 256]
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

from . import fdx, inputs


def harvest(ctx, sets, theta, n_group, log=print):
    Xs, ts = [], []
    for name, make in sets:
        t0 = time.perf_counter()
        ps = make()
        ctx.set_particles(ps)
        ctx.calc_force(theta, 8, n_group, 0.0, quad=True, fp32=True)
        X = ctx.predictor_features()
        ne, ns = ctx.list_counts()
        Xs.append(X)
        ts.append(np.log(ne.astype(np.float64) + ns).astype(np.float32))
        log(f"[harvest] {name}: {X.shape[0]} groups ({time.perf_counter() - t0:.1f} s)")
    return np.concatenate(Xs), np.concatenate(ts)


def default_sets(n_plummer=8, n_clustered=4):
    sets = [(f"plummer1m seed {1001 + k}",
             (lambda k=k: inputs.plummer(1 << 20, seed=1001 + k, eps=1.0 / 256.0)))
            for k in range(n_plummer)]
    sets += [(f"clustered16m seed {1001 + n_plummer + k}",
              (lambda k=k: inputs.clustered(seed=1001 + n_plummer + k)))
             for k in range(n_clustered)]
    return sets


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--n-group", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--plummer", type=int, default=8)
    ap.add_argument("--clustered", type=int, default=4)
    args = ap.parse_args()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    ctx = fdx.Context(0)
    X, t = harvest(ctx, default_sets(args.plummer, args.clustered), args.theta, args.n_group, log)
    log(f"[train] {X.shape[0]} samples")
    t0 = time.perf_counter()
    losses = ctx.predictor_train(X, t, epochs=args.epochs, batch=args.batch, lr=args.lr,
                                 seed=args.seed)
    log(f"[train] {time.perf_counter() - t0:.1f} s; loss {losses[0]:.4f} -> {losses[-1]:.4f}; "
        f"var(t) {np.var(t):.4f}; margin {ctx.predictor_margin():.4f}")
    ctx.predictor_save(args.out)
    print(f"{{\"samples\": {X.shape[0]}, \"loss_first\": {losses[0]:.6f}, "
          f"\"loss_last\": {losses[-1]:.6f}, \"var_target\": {float(np.var(t)):.6f}, "
          f"\"margin\": {ctx.predictor_margin():.6f}}}")
    ctx.close()


if __name__ == "__main__":
    main()
