"""The profile summary tool on synthetic rocprofv3 counter files (no GPU): per-kernel medians,
and the traffic scaling (a counter reading divided into the bytes a calibration kernel of
known size moved) applied to the kernel's median reading."""
import csv
import os

import pytest

from paper_1601_03138_amd import profile_summary as P


def _write(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for k, c, v, t0, t1 in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v,
                        "Start_Timestamp": t0, "End_Timestamp": t1})


def test_sq_medians_per_counter(tmp_path):
    rows = [("k_force<float>", "SQ_INSTS_VALU", v, 0, 1000) for v in (5.0, 1.0, 3.0)]
    rows += [("k_force<float>", "SQ_WAVES", 8192, 0, 1000), ("k_walk", "SQ_INSTS_VALU", 99, 0, 9)]
    _write(str(tmp_path / "sq"), rows)
    out = P.sq(str(tmp_path / "sq"), r"k_force<float>").splitlines()
    assert out == ["SQ_INSTS_VALU: median per dispatch 3.0000e+00 (3 dispatches)",
                   "SQ_WAVES: median per dispatch 8.1920e+03 (1 dispatches)"]


def test_pmc_scaling(tmp_path):
    # calibration: 1 MiB read and 1 MiB written; FETCH reads twice the bytes, WRITE reads them
    mib = 1 << 20
    _write(str(tmp_path / "f"), [("copy", "FETCH_SIZE", 2048, 0, 10),
                                 ("k_force", "FETCH_SIZE", 4096, 0, 3_000_000),
                                 ("k_force", "FETCH_SIZE", 8192, 0, 5_000_000),
                                 ("k_force", "FETCH_SIZE", 6144, 0, 4_000_000)])
    _write(str(tmp_path / "w"), [("copy", "WRITE_SIZE", 1024, 0, 10),
                                 ("k_force", "WRITE_SIZE", 512, 0, 4_000_000)])
    out = P.pmc(str(tmp_path / "f"), str(tmp_path / "w"), "k_force", "copy", mib, mib)
    lines = dict(l.split(": ", 1) for l in out.splitlines() if l.startswith(("fetch", "write", "hbm")))
    fetch = 6144 * 1024 * 0.5          # median reading x (1 MiB / 2048 KiB)
    write = 512 * 1024 * 1.0
    assert float(lines["fetch bytes per launch (scaled)"]) == pytest.approx(fetch, rel=1e-4)
    assert float(lines["write bytes per launch (scaled)"]) == pytest.approx(write, rel=1e-4)
    assert float(lines["hbm bytes per launch"]) == pytest.approx(fetch + write, rel=1e-6)
    assert "3 dispatches, median 4.000 ms" in out


def test_missing_kernel_is_an_error(tmp_path):
    _write(str(tmp_path / "f"), [("copy", "FETCH_SIZE", 1, 0, 1)])
    _write(str(tmp_path / "w"), [("copy", "WRITE_SIZE", 1, 0, 1)])
    with pytest.raises(SystemExit):
        P.pmc(str(tmp_path / "f"), str(tmp_path / "w"), "k_force", "copy", 1, 1)


def test_phases_table_scales_counters_and_counts_algorithmic_bytes(tmp_path):
    # one plain copy kernel of 1 MiB each way for the calibration (FETCH_SIZE reads half the
    # bytes, WRITE_SIZE all of them), and k_unsort at N = 1000 particles: 68 N algorithmic bytes
    trace = tmp_path / "trace"
    os.makedirs(trace)
    with open(trace / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for t in (2000, 1000, 3000):             # ns: median 2 us
            w.writerow({"Kernel_Name": "k_unsort(unsigned long, ...)", "Start_Timestamp": 0,
                        "End_Timestamp": t})
    _write(str(tmp_path / "f"), [("copy", "FETCH_SIZE", 512.0, 0, 1),
                                 ("k_unsort(unsigned long, ...)", "FETCH_SIZE", 40.0, 0, 1)])
    _write(str(tmp_path / "w"), [("copy", "WRITE_SIZE", 1024.0, 0, 1),
                                 ("k_unsort(unsigned long, ...)", "WRITE_SIZE", 30.0, 0, 1)])
    out = P.phases(str(trace), str(tmp_path / "f"), str(tmp_path / "w"), 1000, 0, 0, 0, "copy",
                   1048576, 1048576)
    row = [r for r in out.splitlines() if "k_unsort" in r][0].split("|")
    assert float(row[3]) == pytest.approx(0.002)                 # ms
    assert float(row[4]) == pytest.approx(68000)                 # algorithmic bytes
    assert float(row[5]) == pytest.approx((40 * 2 + 30) * 1024, rel=1e-3)   # scaled counters
    assert float(row[6]) == pytest.approx(68000 / 2e-6 / 1e9, abs=1)
    assert P.stats_csv(str(trace)).splitlines()[2].startswith("| `k_unsort` | 3 | 0.006 |")


def test_phases_table_sums_per_level_kernels_over_an_evaluation(tmp_path):
    # two evaluations (two k_bbox_init dispatches), each with three k_moments launches of 1, 2
    # and 3 us and counter readings 10, 20, 30 KiB: the row is per evaluation (6 us, 60 KiB
    # scaled), not a median over the launches
    trace = tmp_path / "trace"
    os.makedirs(trace)
    names = []
    with open(trace / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for _ in range(2):
            w.writerow({"Kernel_Name": "k_bbox_init(int, ...)", "Start_Timestamp": 0,
                        "End_Timestamp": 500})
            for t in (1000, 2000, 3000):
                w.writerow({"Kernel_Name": "k_moments(int, ...)", "Start_Timestamp": 0,
                            "End_Timestamp": t})
    f_rows = [("copy", "FETCH_SIZE", 512.0, 0, 1)]
    w_rows = [("copy", "WRITE_SIZE", 1024.0, 0, 1)]
    for _ in range(2):
        f_rows.append(("k_bbox_init(int, ...)", "FETCH_SIZE", 1.0, 0, 1))
        w_rows.append(("k_bbox_init(int, ...)", "WRITE_SIZE", 1.0, 0, 1))
        for v in (10.0, 20.0, 30.0):
            f_rows.append(("k_moments(int, ...)", "FETCH_SIZE", v, 0, 1))
            w_rows.append(("k_moments(int, ...)", "WRITE_SIZE", v, 0, 1))
    _write(str(tmp_path / "f"), f_rows)
    _write(str(tmp_path / "w"), w_rows)
    N, C = 1000, 100
    out = P.phases(str(trace), str(tmp_path / "f"), str(tmp_path / "w"), N, C, 0, 0, "copy",
                   1048576, 1048576)
    row = [r for r in out.splitlines() if "k_moments" in r][0].split("|")
    assert float(row[3]) == pytest.approx(0.006)                         # ms per evaluation
    assert float(row[4]) == pytest.approx(160 * C + 32 * N)              # algorithmic bytes
    assert float(row[5]) == pytest.approx((60 * 2 + 60) * 1024, rel=1e-3)  # scaled counters
