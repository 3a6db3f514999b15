"""Summarise rocprofv3 output of the library's runs as short markdown.

  python -m paper_1601_03138_amd.profile_summary stats DIR
      kernel statistics (calls, total, average) from DIR/*_results.db (kernel trace)
  python -m paper_1601_03138_amd.profile_summary pmc FETCH_DIR WRITE_DIR --kernel REGEX
      --calib REGEX --calib-read BYTES --calib-write BYTES
      FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the matching kernel, scaled by what the
      same counters read for a plain streaming kernel of known size
  python -m paper_1601_03138_amd.profile_summary sq DIR --kernel REGEX
      SQ counters per dispatch of the matching kernel
  python -m paper_1601_03138_amd.profile_summary phases TRACE_DIR FETCH_DIR WRITE_DIR
      --n N --cells C --groups G --entries E --calib REGEX --calib-read B --calib-write B
      per kernel of the force evaluation: median duration per dispatch (kernel trace), HBM bytes
      per dispatch from FETCH_SIZE and WRITE_SIZE (scaled as for pmc), the bytes the kernel's
      algorithm must move (ALGO_BYTES below) and both as GB/s; kernels launched once per tree
      level are summed over one evaluation
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import re
import sqlite3
import statistics


def _db(path):
    dbs = glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True)
    if not dbs:
        raise SystemExit(f"no *_results.db under {path}")
    return sqlite3.connect(dbs[0])


def stats(path, top=25):
    db = _db(path)
    rows = db.execute("select name, total_calls, total_duration, average, percentage "
                      "from top_kernels").fetchall()
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, total, avg, pct in rows[:top]:
        short = re.sub(r"fdx::\(anonymous namespace\)::", "", name)
        short = re.sub(r"\(.*", "", short)
        out.append(f"| `{short}` | {calls} | {total / 1e3:.3f} | {avg:.1f} | {pct:.2f} |")
    return "\n".join(out)


def _pmc(path):
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {path}")
    rows = list(csv.DictReader(open(files[0])))
    per = collections.defaultdict(list)
    for r in rows:
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        per[(r["Kernel_Name"], r["Counter_Name"])].append((float(r["Counter_Value"]), dur))
    return per


def _pick(per, regex, counter):
    vals = [v for (k, c), v in per.items() if c == counter and re.search(regex, k)]
    if not vals:
        raise SystemExit(f"no dispatch of /{regex}/ with {counter}")
    return [x for v in vals for x in v]


def pmc(fetch_dir, write_dir, kernel, calib, calib_read, calib_write):
    f, w = _pmc(fetch_dir), _pmc(write_dir)
    cf = _pick(f, calib, "FETCH_SIZE")
    cw = _pick(w, calib, "WRITE_SIZE")
    kf = _pick(f, kernel, "FETCH_SIZE")
    kw = _pick(w, kernel, "WRITE_SIZE")
    sf = calib_read / (statistics.median(v for v, _ in cf) * 1024)
    sw = calib_write / (statistics.median(v for v, _ in cw) * 1024)
    fetch = statistics.median(v for v, _ in kf) * 1024 * sf
    write = statistics.median(v for v, _ in kw) * 1024 * sw
    dur = statistics.median(d for _, d in kf)
    lines = [
        f"calibration kernel /{calib}/: FETCH_SIZE {statistics.median(v for v, _ in cf):.0f} KiB "
        f"for {calib_read} B read -> scale {sf:.4f}; WRITE_SIZE "
        f"{statistics.median(v for v, _ in cw):.0f} KiB for {calib_write} B written -> scale {sw:.4f}",
        f"kernel /{kernel}/: {len(kf)} dispatches, median {dur:.3f} ms",
        f"fetch bytes per launch (scaled): {fetch:.4e}",
        f"write bytes per launch (scaled): {write:.4e}",
        f"hbm bytes per launch: {fetch + write:.6e}",
    ]
    return "\n".join(lines)


def sq(path, kernel):
    per = _pmc(path)
    out = []
    for (k, c), v in sorted(per.items()):
        if re.search(kernel, k):
            vals = [x for x, _ in v]
            out.append(f"{c}: median per dispatch {statistics.median(vals):.4e} ({len(vals)} dispatches)")
    return "\n".join(out)


# Bytes each kernel of the path must move per dispatch (N particles, C cells, G groups,
# E interaction-list entries): the arrays it reads and writes, each counted once.  Rows in
# PER_EVALUATION are dispatched several times in one force evaluation with different sizes
# (one launch per tree level) and are given per evaluation instead.
ALGO_BYTES = [
    # (kernel regex, what, bytes per dispatch)
    (r"^k_bbox\b", "read x, y, z", lambda N, C, G, E: 24 * N),
    (r"^k_keys\b", "read x, y, z, m; write key, index, (x, y, z, m)",
     lambda N, C, G, E: 76 * N),
    (r"^void k_rs_hist", "read key (one 8-bit pass)", lambda N, C, G, E: 8 * N),
    (r"^void k_rs_scatter", "read and write key + index (one pass)", lambda N, C, G, E: 24 * N),
    (r"^k_gather_sorted\b", "read index, record, eps; write record, eps, inverse",
     lambda N, C, G, E: 88 * N),
    (r"^k_cells_prefix\b", "read keys; write two bytes per position", lambda N, C, G, E: 10 * N),
    (r"^void k_cells_count|^k_cells_count\b", "read two bytes, write one per position",
     lambda N, C, G, E: 3 * N),
    (r"^k_cells_emit\b", "read keys + three bytes per position; write 20 B per cell",
     lambda N, C, G, E: 11 * N + 20 * C),
    (r"^k_cells_finish\b", "read 20 B, write 36 B per cell", lambda N, C, G, E: 56 * C),
    (r"^k_moments\b", "all levels of one evaluation (one dispatch per level): write 80 B per "
     "cell, read 80 B per child and 32 B per particle", lambda N, C, G, E: 160 * C + 32 * N),
    (r"^k_group_flags\b", "read counts, write flags per cell", lambda N, C, G, E: 12 * C),
    (r"^k_leaf_level\b", "write a byte per particle", lambda N, C, G, E: 1 * N),
    (r"^void k_group_geom|^k_group_geom\b", "read member keys; write box and centre per group",
     lambda N, C, G, E: 8 * N + 48 * G),
    (r"^void k_walk(_runs)?<true(, 0)?>", "write 4 B per list entry", lambda N, C, G, E: 4 * E),
    (r"^k_unsort\b", "read inverse, result; write four arrays", lambda N, C, G, E: 68 * N),
    (r"^k_kick_drift\b", "read x, v, a; write x, v", lambda N, C, G, E: 120 * N),
    (r"^k_kick\b", "read v, a; write v", lambda N, C, G, E: 72 * N),
]


PER_EVALUATION = {r"^k_moments\b"}
# a kernel dispatched exactly once per force evaluation: counts the evaluations in a trace
EVALUATION_MARKER = r"^k_bbox_init\b"


def _durations(path):
    """Per-dispatch durations (ms) by kernel name from a kernel trace in CSV form
    (rocprofv3 --kernel-trace --output-format csv: *kernel_trace.csv)."""
    files = glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_trace.csv under {path}")
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(files[0])):
        out[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    return out


def stats_csv(path, top=25):
    """stats from a CSV kernel trace: calls, total and average per kernel."""
    durs = _durations(path)
    tot_all = sum(sum(v) for v in durs.values())
    rows = sorted(durs.items(), key=lambda kv: -sum(kv[1]))
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, v in rows[:top]:
        out.append(f"| `{_short(name)}` | {len(v)} | {sum(v):.3f} | {1e3 * sum(v) / len(v):.1f} | "
                   f"{100 * sum(v) / tot_all:.2f} |")
    return "\n".join(out)


def _short(name):
    n = re.sub(r"fdx::\(anonymous namespace\)::", "", name)
    return re.sub(r"\(.*", "", n)


def phases(trace_dir, fetch_dir, write_dir, N, C, G, E, calib, calib_read, calib_write):
    f, w = _pmc(fetch_dir), _pmc(write_dir)
    sf = calib_read / (statistics.median(v for v, _ in _pick(f, calib, "FETCH_SIZE")) * 1024)
    sw = calib_write / (statistics.median(v for v, _ in _pick(w, calib, "WRITE_SIZE")) * 1024)
    durs = _durations(trace_dir)

    def evaluations(per_kernel):
        return sum(len(v) if isinstance(v, list) else 1 for k, v in per_kernel
                   if re.search(EVALUATION_MARKER, _short(k)))

    n_eval = evaluations(durs.items())
    f_eval = evaluations([(k, v) for (k, c), v in f.items() if c == "FETCH_SIZE"])
    w_eval = evaluations([(k, v) for (k, c), v in w.items() if c == "WRITE_SIZE"])
    out = ["| kernel | what it must move | ms (trace) | algorithmic B | HBM B (counters) "
           "| algorithmic GB/s | HBM GB/s |", "|---|---|---|---|---|---|---|"]
    for rx, what, fn in ALGO_BYTES:
        names = [k for k in durs if re.search(rx, _short(k))]
        if not names:
            continue
        fe = [v for (k, c), vs in f.items() if c == "FETCH_SIZE" and k in names for v, _ in vs]
        wr = [v for (k, c), vs in w.items() if c == "WRITE_SIZE" and k in names for v, _ in vs]
        if rx in PER_EVALUATION:
            # sums over one evaluation's dispatches, averaged over the evaluations
            if not (n_eval and f_eval and w_eval):
                raise SystemExit(f"no dispatch of /{EVALUATION_MARKER}/ to count evaluations")
            d = sum(x for k in names for x in durs[k]) / n_eval
            hbm = ((sum(fe) / f_eval) * sf + (sum(wr) / w_eval) * sw) * 1024 if fe and wr else None
        else:
            d = statistics.median(x for k in names for x in durs[k])
            hbm = (statistics.median(fe) * sf + statistics.median(wr) * sw) * 1024 if fe and wr else None
        alg = fn(N, C, G, E)
        out.append(f"| `{_short(names[0])}` | {what} | {d:.3f} | {alg:.3e} | "
                   f"{'n/a' if hbm is None else f'{hbm:.3e}'} | {alg / (d / 1e3) / 1e9:.0f} | "
                   f"{'n/a' if hbm is None else f'{hbm / (d / 1e3) / 1e9:.0f}'} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    b = sub.add_parser("pmc")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--kernel", required=True)
    b.add_argument("--calib", required=True)
    b.add_argument("--calib-read", type=float, required=True)
    b.add_argument("--calib-write", type=float, required=True)
    c = sub.add_parser("sq")
    c.add_argument("dir")
    c.add_argument("--kernel", required=True)
    d = sub.add_parser("phases")
    d.add_argument("trace_dir")
    d.add_argument("fetch_dir")
    d.add_argument("write_dir")
    for k in ("n", "cells", "groups", "entries"):
        d.add_argument("--" + k, type=float, required=True)
    d.add_argument("--calib", required=True)
    d.add_argument("--calib-read", type=float, required=True)
    d.add_argument("--calib-write", type=float, required=True)
    args = ap.parse_args()
    if args.cmd == "phases":
        print(phases(args.trace_dir, args.fetch_dir, args.write_dir, args.n, args.cells,
                     args.groups, args.entries, args.calib, args.calib_read, args.calib_write))
        return
    if args.cmd == "stats":
        has_db = glob.glob(os.path.join(args.dir, "**", "*_results.db"), recursive=True)
        print(stats(args.dir) if has_db else stats_csv(args.dir))
    elif args.cmd == "pmc":
        print(pmc(args.fetch_dir, args.write_dir, args.kernel, args.calib, args.calib_read,
                  args.calib_write))
    else:
        print(sq(args.dir, args.kernel))


if __name__ == "__main__":
    main()
