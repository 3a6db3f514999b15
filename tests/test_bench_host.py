"""Host-side logic of bench.py (no GPU): the one-GPU rule, the traffic lookup that ties a
committed counter summary to the kernel source, shape and launch it was taken for, the flop
accounting of the roofline and the rms relative error of the accelerations."""
import os
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


def _summary(shape, launch, hbm, sha):
    return (f"HBM traffic of a force kernel\n"
            f"fetch bytes per launch (scaled): 1.0e+09\n"
            f"hbm bytes per launch: {hbm:.6e}\n"
            f"shape: {shape}\nlaunch: {launch}\nforce kernel sources sha256: {sha}\n")


def test_traffic_lookup_matches_source_shape_and_launch(tmp_path, monkeypatch):
    import hashlib
    tag = "force_fp32_quad_clustered16m"
    root = tmp_path / "root"
    (root / "paper_1601_03138_amd" / "csrc").mkdir(parents=True)
    (root / "profiles").mkdir()
    src = root / "paper_1601_03138_amd" / "csrc" / "k_force.hip"
    src.write_text("// kernel source as profiled\n")
    inc = root / "paper_1601_03138_amd" / "csrc" / "interact.h"
    inc.write_text("// interaction functions as profiled\n")
    sha = hashlib.sha256(src.read_bytes() + inc.read_bytes()).hexdigest()
    (root / "profiles" / f"{tag}_nt512_ipl1_w8_traffic.txt").write_text(
        _summary("nt512_ipl1_w8", "persistent", 8.3e9, sha))
    (root / "profiles" / f"{tag}_nt512_ipl1_pf_w8_traffic.txt").write_text(
        _summary("nt512_ipl1_pf_w8", "persistent", 1.36e10, sha))
    (root / "profiles" / f"{tag}_nt256_ipl1_traffic.txt").write_text(
        _summary("nt256_ipl1", "direct", 7.0e9, "0" * 64))          # another source
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.read_traffic(tag, "nt512_ipl1_w8", "persistent") == 8.3e9
    assert bench.read_traffic(tag, "nt512_ipl1_pf_w8", "persistent") == 1.36e10
    assert bench.read_traffic(tag, "nt512_ipl1_w8", "direct") is None       # other launch
    assert bench.read_traffic(tag, "nt256_ipl1", "direct") is None          # stale source
    assert bench.read_traffic(tag, "no_such_shape", "persistent") is None
    assert bench.read_traffic("force_fp32_quad_other", "nt512_ipl1_w8", "persistent") is None
    # a kernel source changes after the counters were taken: no traffic is reported
    inc.write_text("// interaction functions as profiled\n// changed\n")
    assert bench.read_traffic(tag, "nt512_ipl1_w8", "persistent") is None
    inc.write_text("// interaction functions as profiled\n")
    assert bench.read_traffic(tag, "nt512_ipl1_w8", "persistent") == 8.3e9
    src.write_text("// kernel source as profiled\n// changed\n")
    assert bench.read_traffic(tag, "nt512_ipl1_w8", "persistent") is None


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
