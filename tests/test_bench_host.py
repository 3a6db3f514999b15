"""Host-side logic of bench.py (no GPU): the one-GPU rule, the traffic lookup that ties a
committed counter summary to the kernel source, shape and launch it was taken for, the flop
accounting of the roofline and the error metric of reading R14."""
import os
import shutil
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "--gpus 1" in r.stderr


def test_traffic_lookup_matches_source_shape_and_launch(tmp_path, monkeypatch):
    tag = "force_fp32_quad_clustered16m"
    shapes = {}
    for f in os.listdir(os.path.join(ROOT, "profiles")):
        if f.startswith(tag) and f.endswith("traffic.txt"):
            vals = dict(line.split(":", 1) for line in open(os.path.join(ROOT, "profiles", f))
                        if ":" in line)
            shapes[vals["shape"].strip()] = (vals["launch"].strip(),
                                             float(vals["hbm bytes per launch"]))
    assert shapes, "no committed traffic summary"
    for shape, (launch, hbm) in shapes.items():
        assert bench.read_traffic(tag, shape, launch) == hbm
        assert bench.read_traffic(tag, shape, "direct" if launch != "direct" else "x") is None
    assert bench.read_traffic(tag, "no_such_shape", "persistent") is None
    # a kernel source that differs from the one the counters were taken on: no traffic
    fake = tmp_path / "root"
    (fake / "paper_1601_03138_amd" / "csrc").mkdir(parents=True)
    shutil.copytree(os.path.join(ROOT, "profiles"), fake / "profiles")
    src = open(os.path.join(ROOT, "paper_1601_03138_amd", "csrc", "k_force.hip")).read()
    (fake / "paper_1601_03138_amd" / "csrc" / "k_force.hip").write_text(src + "\n// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(fake))
    for shape, (launch, _) in shapes.items():
        assert bench.read_traffic(tag, shape, launch) is None


def test_flop_accounting():
    st = {"n_interactions_pp": 3, "n_interactions_pc": 5}
    assert bench.force_flops(st, True) == 3 * 20 + 5 * 54
    assert bench.force_flops(st, False) == 3 * 20 + 5 * 20


def test_rms_relative_error():
    ref = np.array([[3.0, 4.0, 0.0, 1.0], [0.0, 0.0, 2.0, 1.0]])
    a = ref.copy()
    a[0, 0] += 0.5                      # |da|/|a| = 0.1
    a[1, 2] -= 0.2                      # 0.1
    a[:, 3] += 7.0                      # the potential column is not part of the metric
    assert abs(bench.rms_rel_error(a, ref) - 0.1) < 1e-15
    assert bench.rms_rel_error(ref, ref) == 0.0
