"""No C++ exception crosses the C ABI (include/fdx.h conventions): the guard maps
std::bad_alloc to FDX_ENOMEM and any other exception to FDX_EINVAL with a message in the
context's fixed-size last-error buffer (checked by compiling it into a small CPU program),
and every exported entry point whose body spans several lines runs it inside the guard
(checked on the sources)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1601_03138_amd", "csrc")
EINVAL, ENOMEM = -1, -2


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_guard_maps_exceptions_to_status_codes(tmp_path):
    exe = tmp_path / "abi_guard_check"
    src = os.path.join(ROOT, "tests", "native", "abi_guard_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, src, "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    rows = {r.split("|")[0]: r.split("|", 2)[1:] for r in out.strip().splitlines()}
    assert rows["bad_alloc"] == [str(ENOMEM), "host memory allocation failed"]
    assert rows["huge_vector"][0] in (str(ENOMEM), str(EINVAL))
    assert rows["huge_vector"][1]
    code, msg = rows["runtime_error"]
    assert code == str(EINVAL) and msg.startswith("internal error: a long message")
    assert len(msg) == 63                      # truncated to the buffer, terminated
    assert rows["int"] == [str(EINVAL), "internal error: unknown exception"]
    assert rows["ok"] == ["0", ""]
    assert rows["null"] == [str(ENOMEM), ""]


# entry points whose whole body is one expression that cannot allocate
UNGUARDED = {"fdx_autotune_shapes", "fdx_mlp_params", "fdx_shape_name", "fdx_last_error"}


def _definitions():
    for fn in sorted(os.listdir(CSRC)):
        if not fn.endswith((".cpp", ".hip")):
            continue
        lines = open(os.path.join(CSRC, fn)).read().split("\n")
        i = 0
        while i < len(lines):
            m = re.match(r"^(?:int|const char \*)\s*(fdx_\w+)\(", lines[i])
            if not m:
                i += 1
                continue
            j = i
            while not lines[j].rstrip().endswith("{") and not lines[j].rstrip().endswith("}"):
                j += 1
            if lines[j].rstrip().endswith("}"):          # one-line body
                yield fn, m.group(1), None
                i = j + 1
                continue
            k = j + 1
            while lines[k] != "}":
                k += 1
            yield fn, m.group(1), lines[j + 1:k]
            i = k + 1


def test_every_entry_point_runs_inside_the_guard():
    seen = set()
    for fn, name, body in _definitions():
        seen.add(name)
        if name in UNGUARDED:
            continue
        assert body is not None, (fn, name)
        assert body[0].strip() == "FDX_ABI_TRY", (fn, name, body[0])
        assert body[-1].strip().startswith("FDX_ABI_CATCH("), (fn, name, body[-1])
    header = open(os.path.join(ROOT, "include", "fdx.h")).read()
    declared = set(re.findall(r"^(?:int|const char \*)\s*(fdx_\w+)\(", header, re.M))
    assert declared <= seen, declared - seen
