"""Benchmark: particles per second per force evaluation of the Barnes-Hut hot path on one GPU.

One step = one leapfrog step of the sample program (kick + drift, one full force evaluation:
keys, sort, tree, moments, groups, walk, force, unsort; kick) on the N = 2^24 clustered
workload, theta = 0.5, quadrupole superparticles, FP32 group-relative force kernels.
Inputs are resident in device memory before the timed region.  Prints one JSON line.

n_group and the force kernel's workgroup shape are chosen first by the library's autotuner
(n_group in {64, 128, 256, 512} x every shape, full evaluations timed; --no-autotune keeps the
workload default), for the headline workload and for the batched ensemble.

Also reported: the FP64 force path on the same input, the force-kernel roofline (measured with
HIP events on the library's stream), accuracy against FP64 direct summation on a seeded
subset, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
# Algorithmic flops per interaction of the force kernels (FMA = 2, rsqrt = 1), counted from
# the formulas they evaluate: particle 20; superparticle monopole 20, quadrupole 54.
FLOPS_PP = 20
FLOPS_PC_MONO = 20
FLOPS_PC_QUAD = 54

WORKLOADS = {
    # name: (n_group, theta, quad, dt); the clustered and ensemble workloads are defined with
    # an autotuned n_group (the value here is the default without the autotuner), the two
    # Plummer spheres with a fixed one
    "clustered16m": (256, 0.5, True, 1.0 / 1024.0),
    "ensemble512": (128, 0.6, True, 1.0 / 256.0),
    "plummer1m": (256, 0.5, True, 1.0 / 256.0),
    "plummer4k": (64, 0.5, False, 1.0 / 128.0),
}
AUTOTUNED = {"clustered16m", "ensemble512"}


# list-length predictor weights shipped with the package: (workload, n_group, theta) they were
# trained for (on inputs of other seeds)
PREDICTOR_WEIGHTS = {("clustered16m", 256, 0.5):
                     os.path.join(ROOT, "paper_1601_03138_amd", "predictor_clustered16m_ng256.bin")}


def exchange_list_model(n: float, theta: float, n_p: float) -> float:
    """Equation n_list_long: total exchange-list length of one of n_p cubic domains of n
    particles (section "Exchange of particles and superparticles")."""
    return (14.0 * n ** (2.0 / 3.0) / theta + 21.0 * math.pi * n ** (1.0 / 3.0) / theta ** 2
            + 28.0 * math.pi / (3.0 * theta ** 3)
            * math.log2(theta / 2.8 * ((n * n_p) ** (1.0 / 3.0) - n ** (1.0 / 3.0))))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_flops(st, quad):
    return st["n_interactions_pp"] * FLOPS_PP + st["n_interactions_pc"] * (
        FLOPS_PC_QUAD if quad else FLOPS_PC_MONO)


def force_source_sha():
    """sha256 over the force kernel's sources (k_force.hip, then interact.h, byte for byte):
    a traffic summary counts only for the code it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_force.hip", "interact.h"):
        try:
            h.update(open(os.path.join(ROOT, "paper_1601_03138_amd", "csrc", f), "rb").read())
        except OSError:
            return None
    return h.hexdigest()


def read_traffic(kernel_tag: str, shape: str, launch: str):
    """HBM bytes per launch of the force kernel measured by rocprofv3 counters, if a summary
    for the current kernel source, this shape and this launch is committed under profiles/
    (files <kernel_tag>_<shape>_traffic.txt; else None)."""
    import glob
    sha = force_source_sha()
    if sha is None:
        return None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{kernel_tag}_*traffic.txt"))):
        vals = {}
        for line in open(path):
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
        if (vals.get("force kernel sources sha256") != sha or vals.get("shape") != shape
                or vals.get("launch") != launch):
            continue
        try:
            return float(vals["hbm bytes per launch"])
        except (KeyError, ValueError):
            return None
    return None


def rms_rel_error(a, a_ref) -> float:
    """sqrt(mean_i |a_i - a_ref_i|^2 / |a_ref_i|^2) over the rows given (3 components)."""
    d = np.sum((a[:, :3] - a_ref[:, :3]) ** 2, axis=1)
    r = np.sum(a_ref[:, :3] ** 2, axis=1)
    return float(math.sqrt(np.mean(d / r)))


def autotune(ctx, theta, quad, persistent, graph=False, fused=False):
    """n_group in {64, 128, 256, 512} x every force-kernel shape (the fused launch: n_group up to
    256, one timing each), full evaluations (graph: graph-captured steps of dt = 0) timed by the
    library's autotuner (the median of 3 after one untimed; shapes that spill registers are not
    timed); its choice stays set in ctx."""
    from paper_1601_03138_amd import fdx
    cand = [64, 128, 256] if fused else [64, 128, 256, 512]
    flags = fdx.Context.flags(quad=quad, fp32=True, persistent=persistent, fused=fused)
    if graph:
        flags |= fdx.GRAPH
    bg, bv, times = ctx.autotune(theta, 8, 0.0, flags, cand, reps=3)
    return {"n_group": bg, "shape": bv, "shape_name": ctx.shape_name(bv), "candidates": cand,
            "ms": [[None if np.isnan(v) else round(float(v), 3) for v in row] for row in times]}


def cpu_model() -> str:
    """The host CPU's model name (as lscpu prints it), from /proc/cpuinfo."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ps, n_group, theta, quad, n_sample_groups, n_sample_groups_1t=64, seed=7):
    """The oracle as it stands (FP64 serial tree, OpenMP over groups): the full tree build of
    the workload plus the walk and force of a random sample of groups, scaled to one whole
    force evaluation -- on all the threads OpenMP is given, and once more single-threaded (a
    smaller sample of groups)."""
    import oracle as O

    def one(k_groups):
        t0 = time.perf_counter()
        tr = O.build_tree(ps, 8)
        g = O.make_groups(tr, n_group)
        t1 = time.perf_counter()
        rng = np.random.default_rng(seed)
        k = min(k_groups, g.n)
        sel = np.sort(rng.choice(g.n, k, replace=False))
        lists = O.walk(tr, g, theta, sel)
        lists.force(quad)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, k, g.n

    threads = O.set_threads(0)
    tb, tw, k, G = one(n_sample_groups)
    t_eval = tb + tw * G / k
    O.set_threads(1)
    try:
        tb1, tw1, k1, _ = one(n_sample_groups_1t)
    finally:
        O.set_threads(threads)
    t_eval1 = tb1 + tw1 * G / k1
    return {"value": ps.n / t_eval, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"FP64 oracle tree on {threads} threads: full build of all {ps.n} "
                      f"particles ({tb:.1f} s) + walk and force of {k} random groups of {G} "
                      f"({tw:.2f} s), scaled to all groups; est. {t_eval:.0f} s per force "
                      f"evaluation",
            "single_thread": {"value": ps.n / t_eval1, "unit": "particles/s", "cores": 1,
                              "sample": f"full build ({tb1:.1f} s) + walk and force of {k1} "
                                        f"random groups ({tw1:.2f} s), scaled to all "
                                        f"groups; est. {t_eval1:.0f} s per force "
                                        f"evaluation"}}


def system_energies(ps, ctx):
    """Kinetic + potential energy of every system at the context's current state."""
    a = ctx.forces()
    x, y, z, vx, vy, vz = ctx.particles()
    off = ps.offsets()
    e = np.empty(ps.n_sys)
    for s in range(ps.n_sys):
        sl = slice(off[s], off[s + 1])
        e[s] = (0.5 * np.sum(ps.m[sl] * (vx[sl] ** 2 + vy[sl] ** 2 + vz[sl] ** 2))
                + 0.5 * np.sum(ps.m[sl] * a[sl, 3]))
    return e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered16m", choices=sorted(WORKLOADS))
    ap.add_argument("--n-group", type=int, default=0, help="0: workload default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--accuracy-subset", type=int, default=4096,
                    help="particles whose forces are checked against FP64 direct summation")
    ap.add_argument("--fp64-evals", type=int, default=3)
    ap.add_argument("--cpu-sample-groups", type=int, default=512)
    ap.add_argument("--graph", action="store_true",
                    help="replay each leapfrog step as a captured HIP graph (persistent force)")
    ap.add_argument("--direct", action="store_true",
                    help="one workgroup per group in group order (XCD-aware) instead of the "
                         "default persistent force kernel over per-XCD queues of groups")
    ap.add_argument("--fused", action="store_true",
                    help="walk and force in one persistent launch (FDX_FUSED; n_group <= 256)")
    ap.add_argument("--walk", default="auto", choices=["auto", "exact", "predicted"],
                    help="exact: count pass + fill pass; predicted: the learned list-length "
                         "predictor sizes the lists for a single fill pass (groups that do not "
                         "fit are re-walked exactly; results are identical); auto: predicted "
                         "when weights for the workload exist")
    ap.add_argument("--predictor", default="",
                    help="predictor weights (default: the shipped ones for the workload)")
    ap.add_argument("--shape", default="",
                    help="force-kernel shape by name (e.g. nt512_ipl1_w8); skips the autotuner")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (n_group x kernel shape) and use the workload's "
                         "default n_group and shape")
    ap.add_argument("--exchange-domains", type=int, default=4,
                    help="also time the exchange lists of the input cut into k x k x k "
                         "equal-count domains (0: skip)")
    ap.add_argument("--sph-log2n", type=int, default=24,
                    help="also time the SPH density (fixed cutoff of 4.2 mean spacings, uniform "
                         "cube of 2^k particles; 0: skip)")
    ap.add_argument("--dd-k", type=int, default=4,
                    help="domain decomposition of the clustered workload from k^3 current "
                         "domains into k^3 new ones (0: skip)")
    ap.add_argument("--dd-samples", type=int, default=1 << 20)
    ap.add_argument("--treepm-log2n", type=int, default=24,
                    help="also time the tree part of TreePM (uniform cube of 2^k particles, cutoff "
                         "of three mesh widths; 0: skip)")
    ap.add_argument("--ensemble-steps", type=int, default=100,
                    help="also time the batched ensemble (512 Plummer systems, graph-captured "
                         "steps; one walk + force launch, and walk then force) for this many "
                         "steps (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1601_03138_amd import fdx, inputs

    n_group, theta, quad, dt = WORKLOADS[args.workload]
    if args.n_group:
        n_group = args.n_group
    if args.copy_calibration:
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)      # one plain streaming kernel: 256 MiB in, 256 MiB out
        torch.cuda.synchronize()
        log("[bench] copy calibration: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    log(f"[bench] generating {args.workload}")
    ps = inputs.workload(args.workload)
    ctx = fdx.Context(0)
    ctx.set_particles(ps)
    persistent = not args.direct or args.graph or args.fused
    flags = fdx.Context.flags(quad=quad, fp32=True, timing=True, persistent=persistent,
                              fused=args.fused)
    tuned = None
    if args.shape:
        names = [ctx.shape_name(v) for v in range(ctx.lib.fdx_autotune_shapes())]
        if args.shape not in names:
            print(f"bench.py: unknown shape {args.shape}; shapes: {names}", file=sys.stderr)
            sys.exit(2)
        ctx.set_shape(names.index(args.shape))
    elif not args.no_autotune and not args.n_group and args.workload in AUTOTUNED:
        tuned = autotune(ctx, theta, quad, persistent, graph=args.graph, fused=args.fused)
        n_group = tuned["n_group"]
        log(f"[bench] autotune: n_group={n_group} shape={tuned['shape_name']} times={tuned['ms']}")

    weights = args.predictor or PREDICTOR_WEIGHTS.get((args.workload, n_group, theta), "")
    if weights and not os.path.exists(weights):
        weights = ""
    walk = args.walk
    if walk == "auto":
        walk = "predicted" if weights and not args.graph else "exact"
    if walk == "predicted" and (not weights or args.graph):
        print("bench.py: --walk predicted needs predictor weights and no --graph", file=sys.stderr)
        sys.exit(2)
    if weights:
        ctx.predictor_load(weights)

    # initial force (its flags, walk included, are those of every step), then warm-up steps
    step_flags = flags | (fdx.PREDICTOR if walk == "predicted" else 0)
    ctx.calc_force_flags(theta, 8, n_group, 0.0, step_flags)
    energy0 = system_energies(ps, ctx)
    for _ in range(args.warmup):
        ctx.integrate(dt, 1, graph=args.graph)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t_force, flops, phases = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.integrate(dt, 1, graph=args.graph)
        if not args.graph:
            st = ctx.stats()
            t_force.append(st["t_force"])
            flops.append(force_flops(st, quad))
            phases.append({k: st[k] for k in st if k.startswith("t_")})
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = ps.n / (ms_step / 1e3)
    drift = None
    if energy0 is not None:
        e1 = system_energies(ps, ctx)
        d = np.abs((e1 - energy0) / energy0)
        drift = {"max": float(d.max()), "median": float(np.median(d)),
                 "steps": args.warmup + args.steps}
    if args.graph:
        # kernel timing of the same evaluation, eager, on the current particles
        for _ in range(2):
            ctx.calc_force_flags(theta, 8, n_group, 0.0, flags)
            st = ctx.stats()
            t_force.append(st["t_force"])
            flops.append(force_flops(st, quad))
            phases.append({k: st[k] for k in st if k.startswith("t_")})
    st = ctx.stats()
    mean_force_ms = float(np.mean(t_force))
    achieved = float(np.mean(flops)) / (mean_force_ms / 1e3) / 1e12
    phase_ms = {k[2:]: round(float(np.mean([p[k] for p in phases])), 4) for k in phases[0]}
    shape = ctx.shape_name(st["shape"])
    # algorithmic bytes of the HBM-bound phases (per particle unless stated): keys = bbox read
    # 24 + key kernel read 32 (x, y, z, m) / write 12 (key, index) + 32 ((x, y, z, m) record
    # for the sorted gather); sort = 32 per radix pass (8 B
    # histogram read, 12 B pair read and written) + sorted gather (4 perm + 32 record + 32 out
    # + 8 eps + 4 inverse); walk = the 4-byte list entries written by the fill pass
    passes = 8 + (0 if ps.n_sys <= 1 else (int(np.ceil(np.log2(ps.n_sys))) + 7) // 8)
    gbs = lambda b, ms: round(b / (ms / 1e3) / 1e9, 1) if ms > 0 else None
    # tree = 30 B per particle (keys read by the level, count and emit passes) + 60 B per
    # cell written; moments = 80 B per cell written + 80 B per child read; groups = 16 B per
    # particle + 1 B leaf level written and read
    ncell = int(st["n_cells"])
    phase_gbs = {"keys": gbs(100 * ps.n, phase_ms["keys"]),
                 "sort": gbs((32 * passes + 80) * ps.n, phase_ms["sort"]),
                 "tree": gbs(30 * ps.n + 60 * ncell, phase_ms["tree"]),
                 "moments": gbs(160 * ncell, phase_ms["moments"]),
                 "groups": gbs(18 * ps.n, phase_ms["groups"]),
                 "walk_list_write": gbs(4 * (int(st["n_epj"]) + int(st["n_spj"])),
                                        phase_ms["walk"])}
    traffic = None if args.fused else read_traffic(
        f"force_fp32_quad_{args.workload}" if quad else f"force_fp32_mono_{args.workload}",
        shape, "persistent" if persistent else "direct")

    # the same evaluation with the exact and the predicted walk
    pred = None
    if weights:
        pflags = flags | fdx.PREDICTOR
        ctx.calc_force_flags(theta, 8, n_group, 0.0, flags)
        exact_total = int(sum(int(a.sum()) for a in ctx.list_counts()))
        a_exact = ctx.forces()
        ctx.calc_force_flags(theta, 8, n_group, 0.0, pflags)
        identical = bool(np.array_equal(ctx.forces(), a_exact))
        rows = {"exact": [], "predicted": []}
        for _ in range(max(3, args.steps // 2)):
            for key, fl in (("exact", flags), ("predicted", pflags)):
                torch.cuda.synchronize()
                ta = time.perf_counter()
                ctx.calc_force_flags(theta, 8, n_group, 0.0, fl)
                torch.cuda.synchronize()
                sp = ctx.stats()
                rows[key].append(((time.perf_counter() - ta) * 1e3, sp["t_walk"],
                                  sp["overflow_groups"], sp["list_capacity"], sp["n_groups"]))
        med = {k: np.median(np.array(v), axis=0) for k, v in rows.items()}
        pred = {"ms_per_eval_exact": round(float(med["exact"][0]), 3),
                "ms_per_eval_predicted": round(float(med["predicted"][0]), 3),
                "walk_ms_exact": round(float(med["exact"][1]), 3),
                "walk_ms_predicted": round(float(med["predicted"][1]), 3),
                "overflow_groups": int(med["predicted"][2]), "groups": int(med["predicted"][4]),
                "list_entries_exact": exact_total,
                "list_capacity_predicted": int(med["predicted"][3]),
                "margin": ctx.predictor_margin(),
                "forces_bit_identical": identical}
        log(f"[bench] predictor: {pred}")

    # FP64 force path on the same (current) particles
    fp64 = None
    if args.fp64_evals > 0:
        f64flags = fdx.Context.flags(quad=quad, fp32=False, timing=True, persistent=persistent)
        ctx.calc_force_flags(theta, 8, n_group, 0.0, f64flags)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        tf = []
        for _ in range(args.fp64_evals):
            ctx.calc_force_flags(theta, 8, n_group, 0.0, f64flags)
            s64 = ctx.stats()
            tf.append(s64["t_force"])
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ms64 = (tb - ta) * 1e3 / args.fp64_evals
        fp64 = {"ms_per_eval": round(ms64, 3), "particles_per_s": ps.n / (ms64 / 1e3),
                "force_kernel_ms": round(float(np.mean(tf)), 3),
                "force_tflops": round(force_flops(s64, quad) / (np.mean(tf) / 1e3) / 1e12, 2),
                "frac_of_fp64_peak": round(force_flops(s64, quad) / (np.mean(tf) / 1e3) / 1e12
                                           / PEAK_FP64_TFLOPS, 4)}

    # accuracy of both paths against FP64 direct summation at the current positions
    accuracy = None
    if not args.no_accuracy:
        sub = inputs.subset(ps.n, min(args.accuracy_subset, ps.n), seed=102)
        d = ctx.direct_forces(sub)                  # FP64 direct sum on the GPU
        ctx.calc_force_flags(theta, 8, n_group, 0.0, fdx.Context.flags(quad=quad, fp32=False))
        e64 = rms_rel_error(ctx.forces()[sub], d)
        ctx.calc_force_flags(theta, 8, n_group, 0.0, fdx.Context.flags(quad=quad, fp32=True))
        e32 = rms_rel_error(ctx.forces()[sub], d)
        accuracy = {"rms_da_over_a_fp32": e32, "rms_da_over_a_fp64": e64,
                    "subset": f"{len(sub)} particles, seed 102, FP64 direct sum (fdx_direct_forces)"}

    # exchange lists between domains (the same particles as k x k x k virtual processes)
    exch = None
    if args.exchange_domains > 0 and ps.n_sys == 1:
        kd = args.exchange_domains
        dom, _ = inputs.multisection(ps, kd, kd, kd)
        cx = fdx.Context(0)
        cx.set_particles(dom)
        cx.build_exchange_lists(theta, 8)
        ts, tl = [], []
        for _ in range(5):
            cx.build_exchange_lists(theta, 8)
            xs = cx.exchange_stats()
            ts.append(xs["ms_tree"])
            tl.append(xs["ms_lists"])
        entries = int(xs["n_epj"] + xs["n_spj"])
        ms_lists = float(np.median(tl))
        exch = {"domains": kd ** 3, "theta": theta, "n_leaf": 8,
                "ms_local_trees": round(float(np.median(ts)), 3), "ms_lists": round(ms_lists, 3),
                "entries": entries, "epj": int(xs["n_epj"]), "spj": int(xs["n_spj"]),
                "entries_per_s": round(entries / (ms_lists / 1e3), -6),
                "mean_entries_per_domain": round(entries / kd ** 3, 1),
                "model_eq_n_list_long": round(exchange_list_model(ps.n / kd ** 3, theta,
                                                                  kd ** 3), 1),
                "paper_s_per_entry_one_cpu_process": 1.12e-7}
        cx.close()
        log(f"[bench] exchange lists: {exch}")

    # multisection domain decomposition with cost-weighted sampling + exchange of particles
    dd = None
    if args.dd_k > 0 and ps.n_sys == 1:
        from paper_1601_03138_amd import dd_timing
        kd = args.dd_k
        ddom = dom if exch is not None and kd == args.exchange_domains else \
            inputs.multisection(ps, kd, kd, kd)[0]
        dd = dd_timing.run(ddom, kd, args.dd_samples, 3, theta, log=log)
        log(f"[bench] domain decomposition: {dd}")

    # SPH density: short-range neighbour lists (fixed cutoff) + Wendland C6 density, FP64
    sph = None
    if args.sph_log2n > 0:
        from paper_1601_03138_amd import sph_timing
        sps, r_cut, _ = sph_timing.workload(args.sph_log2n, 4.2, fdx.CUT_FIXED)
        cs = fdx.Context(0)
        cs.set_particles(sps)
        cs.calc_density(fdx.CUT_FIXED, r_cut, n_group=64, timing=True)
        rows = []
        for _ in range(3):
            cs.calc_density(fdx.CUT_FIXED, r_cut, n_group=64, timing=True)
            ss = cs.stats()
            rows.append((ss["t_walk"], ss["t_force"], ss["t_total"]))
        _, nngb = cs.density()
        med = np.median(np.array(rows), axis=0)
        spacing = sps.n ** (-1.0 / 3.0)
        n_grp = sps.n / max(1, int(ss["n_groups"]))
        sph = {"n": sps.n, "cutoff": "fixed, 4.2 mean spacings", "n_group": 64,
               "ms_walk": round(float(med[0]), 3), "ms_density": round(float(med[1]), 3),
               "ms_total": round(float(med[2]), 3),
               "particles_per_s": float(round(sps.n / (med[2] / 1e3), -5)),
               "pair_tests_per_s": float(round(int(ss["n_interactions_pp"]) / (med[1] / 1e3), -8)),
               "mean_neighbours": round(float(nngb.mean()), 1),
               "mean_candidates_per_group": round(int(ss["n_epj"]) / int(ss["n_groups"]), 1),
               "model_eq_nlist_short": round((n_grp ** (1 / 3) - 1 + 2 * r_cut / spacing) ** 3, 1)}
        cs.close()
        del sps
        log(f"[bench] sph: {sph}")

    # batched ensemble: 512 independent Plummer systems, steps captured as a HIP graph; the walk
    # and force of all systems in one persistent launch (FDX_FUSED), and beside it the walk
    # launch followed by the persistent force launch; FP32 group-relative and FP64 against
    # direct summation; per-system energy drift over the graph-replayed steps
    ens = None
    if args.ensemble_steps > 0 and args.workload != "ensemble512":
        eg0, eth, equad, edt = WORKLOADS["ensemble512"]
        eps_ = inputs.workload("ensemble512")
        ce = fdx.Context(0)
        ce.set_particles(eps_)
        sub = inputs.subset(eps_.n, min(args.accuracy_subset, eps_.n), seed=103)
        d = ce.direct_forces(sub)
        ens = {"n": eps_.n, "systems": eps_.n_sys, "theta": eth, "steps_graph": args.ensemble_steps,
               "accuracy_subset": f"{len(sub)} particles, seed 103, FP64 direct sum within each "
                                  "system"}
        for mode in ("fused", "separate"):
            fused = mode == "fused"
            eg, etuned = eg0, None
            if not args.no_autotune:
                etuned = autotune(ce, eth, equad, True, graph=True, fused=fused)
                eg = etuned["n_group"]
                log(f"[bench] ensemble ({mode}) autotune: n_group={eg} shape={etuned['shape_name']}")
            f32 = fdx.Context.flags(quad=equad, fp32=True, persistent=True, fused=fused)
            ce.set_particles(eps_)
            ce.calc_force_flags(eth, 8, eg, 0.0, f32)
            for _ in range(2):
                ce.integrate(edt, 1, graph=True)
            e_start = system_energies(eps_, ce)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            ce.integrate(edt, args.ensemble_steps, graph=True)
            torch.cuda.synchronize()
            ms_graph = (time.perf_counter() - ta) * 1e3 / args.ensemble_steps
            e_end = system_energies(eps_, ce)
            sys_drift = np.abs((e_end - e_start) / e_start)
            recoveries = int(ce.stats()["graph_recoveries"])
            # kernel timing, accuracy and the FP64 path on the initial particles
            ce.set_particles(eps_)
            tf, fl32 = [], []
            for _ in range(3):
                ce.calc_force_flags(eth, 8, eg, 0.0, f32 | fdx.TIMING)
                st_ = ce.stats()
                tf.append(st_["t_force"] + st_["t_walk"])
                fl32.append(force_flops(st_, equad))
            t32 = ce.stats()["t_total"]
            e32 = rms_rel_error(ce.forces()[sub], d)
            f64 = fdx.Context.flags(quad=equad, fp32=False, persistent=True, timing=True,
                                    fused=fused)
            ce.calc_force_flags(eth, 8, eg, 0.0, f64)
            ce.calc_force_flags(eth, 8, eg, 0.0, f64)
            t64 = ce.stats()["t_total"]
            e64 = rms_rel_error(ce.forces()[sub], d)
            kms = float(np.median(tf))
            ens[mode] = {
                "launch": ("one walk + force launch (FDX_FUSED)" if fused else
                           "walk launch, then persistent force launch"),
                "n_group": eg, "ms_per_step_graph": round(ms_graph, 3),
                "particles_per_s_graph": float(round(eps_.n / (ms_graph / 1e3), -5)),
                "walk_plus_force_ms": round(kms, 3),
                "walk_plus_force_tflops": round(float(np.mean(fl32)) / (kms / 1e3) / 1e12, 2),
                "ms_per_eval_fp32": round(float(t32), 3), "ms_per_eval_fp64": round(float(t64), 3),
                "particles_per_s_fp64": float(round(eps_.n / (t64 / 1e3), -5)),
                "rms_da_over_a_fp32": e32, "rms_da_over_a_fp64": e64,
                "energy_drift_per_system": {"max": float(sys_drift.max()),
                                            "median": float(np.median(sys_drift)),
                                            "steps": args.ensemble_steps},
                "graph_recoveries": recoveries,
                "autotune": etuned and {k: etuned[k] for k in ("n_group", "shape_name")}}
            log(f"[bench] ensemble ({mode}): {ens[mode]}")
        ce.close()
        del eps_

    # tree part of TreePM: monopole tree with the S2 cutoff, FP32 group-relative
    treepm = None
    if args.treepm_log2n > 0:
        from paper_1601_03138_amd import treepm_timing
        tps, r_cut = treepm_timing.workload(args.treepm_log2n)
        ct = fdx.Context(0)
        ct.set_particles(tps)
        ct.calc_force_cutoff(0.5, 8, 256, 0.0, r_cut, fp32=True, persistent=True,
                              timing=True)
        rows = []
        for _ in range(3):
            ct.calc_force_cutoff(0.5, 8, 256, 0.0, r_cut, fp32=True, persistent=True,
                              timing=True)
            ts_ = ct.stats()
            rows.append((ts_["t_walk"], ts_["t_force"], ts_["t_total"]))
        med = np.median(np.array(rows), axis=0)
        inter = int(ts_["n_interactions_pp"] + ts_["n_interactions_pc"])
        treepm = {"n": tps.n, "r_cut": r_cut, "theta": 0.5, "n_group": 256, "dtype": "f32",
                  "ms_walk": round(float(med[0]), 3), "ms_force": round(float(med[1]), 3),
                  "ms_total": round(float(med[2]), 3),
                  "particles_per_s": float(round(tps.n / (med[2] / 1e3), -5)),
                  "interactions_per_s": float(round(inter / (med[1] / 1e3), -8))}
        ct.close()
        del tps
        log(f"[bench] treepm tree part: {treepm}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(ps, n_group, theta, quad, args.cpu_sample_groups)
        # the oracle on the "next" rows' workloads, for the same comparison
        import oracle as O
        nxt = {}
        if exch is not None:
            ta = time.perf_counter()
            O.exchange(O.build_tree(dom, 8), theta)
            nxt["exchange_lists_s"] = round(time.perf_counter() - ta, 2)
        if dd is not None:
            ta = time.perf_counter()
            O.decompose(ddom, args.dd_k, args.dd_k, args.dd_k, args.dd_samples, seed=1)
            nxt["domain_decomposition_s_uniform_cost"] = round(time.perf_counter() - ta, 2)
        cpu["next_rows"] = nxt

    out = {
        "metric": "particles/s per force eval at N=2^24, theta=0.5; FP32 vs FP64 at rms da/a<=1e-3",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": ps.n, "systems": ps.n_sys, "theta": theta,
                   "n_group": n_group, "n_leaf": 8, "quadrupole": quad,
                   "eps": float(ps.eps[0]) if ps.n_sys == 1 else "4/N_s^(1/3)", "dt": dt,
                   "graph": args.graph, "persistent": persistent, "fused": args.fused,
                   "walk": ("predicted single pass, exact re-walk of groups that overflow"
                            if walk == "predicted" else "exact count + fill passes"),
                   "step": "leapfrog kick-drift, full force evaluation, kick"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": traffic,
                     "kernel": ("k_fused<float, quad> (walk + force, one launch)" if args.fused
                                else f"k_force_persistent<float, quad> {shape}" if persistent
                                else f"k_force_direct<float, quad> {shape}"),
                     "kernel_ms": round(mean_force_ms, 3),
                     "interactions_per_launch": int(st["n_interactions_pp"] + st["n_interactions_pc"]),
                     "interactions_per_s": round((st["n_interactions_pp"] + st["n_interactions_pc"])
                                                 / (mean_force_ms / 1e3), -8),
                     "flops_per_interaction": {"pp": FLOPS_PP,
                                               "pc": FLOPS_PC_QUAD if quad else FLOPS_PC_MONO}},
        "cpu_baseline": cpu,
        "fp64": fp64,
        "accuracy": accuracy,
        "phases_ms": phase_ms,
        "phase_gbs": phase_gbs,
        "exchange": exch,
        "domain_decomposition": dd,
        "ensemble": ens,
        "sph": sph,
        "treepm_tree": treepm,
        "energy_drift": drift,
        "graph_recoveries": int(ctx.stats()["graph_recoveries"]) if args.graph else None,
        "predictor": pred,
        "autotune": tuned,
        "tree": {"cells": int(st["n_cells"]), "groups": int(st["n_groups"]),
                 "depth": int(st["depth"]), "epj": int(st["n_epj"]), "spj": int(st["n_spj"])},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
