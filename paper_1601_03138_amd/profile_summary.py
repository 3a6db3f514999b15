"""Summarise rocprofv3 output of the library's runs as short markdown.

  python -m paper_1601_03138_amd.profile_summary stats DIR
      kernel statistics (calls, total, average) from DIR/*_results.db (kernel trace)
  python -m paper_1601_03138_amd.profile_summary pmc FETCH_DIR WRITE_DIR --kernel REGEX
      --calib REGEX --calib-read BYTES --calib-write BYTES
      FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the matching kernel, scaled by what the
      same counters read for a plain streaming kernel of known size
  python -m paper_1601_03138_amd.profile_summary sq DIR --kernel REGEX
      SQ counters per dispatch of the matching kernel
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
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.dir))
    elif args.cmd == "pmc":
        print(pmc(args.fetch_dir, args.write_dir, args.kernel, args.calib, args.calib_read,
                  args.calib_write))
    else:
        print(sq(args.dir, args.kernel))


if __name__ == "__main__":
    main()
