"""The rule by which the library's gravity walk shares the upper tree between runs of four
consecutive groups, checked on the CPU against the oracle's per-group walk.

For a run whose groups' boxes lie inside the box B: a cell that passes the opening test
against B passes against every member's box; a cell that fails it even at B's far corners is
opened by every member.  One walk of B emits the cells and leaf particles every member's
list holds and keeps the undecided cells as a frontier, from which each member walks on.
The union must be the member's own list, entry for entry (as a set), for every group; runs
that straddle two systems or whose frontier exceeds the kernel's 224 cells are walked group
by group.  This is a model of the rule, in plain Python on the oracle's tree; the GPU kernel
that follows it is checked against the oracle's lists by the GPU parity tests."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_1601_03138_amd import inputs as I

RUN, FRONT = 4, 224
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _centres(t):
    """Cell centres in half-grid units (2^22 per root side) from level and key prefix."""
    lev = t.level.astype(np.int64)
    cen = np.zeros((lev.shape[0], 3), np.int64)
    for c in range(lev.shape[0]):
        l, p = int(lev[c]), int(t.prefix[c])
        x = y = z = 0
        for b in range(l):
            d = (p >> (3 * (l - 1 - b))) & 7
            x, y, z = (x << 1) | ((d >> 2) & 1), (y << 1) | ((d >> 1) & 1), (z << 1) | (d & 1)
        s = 1 << (22 - l)
        cen[c] = (x * s + s // 2, y * s + s // 2, z * s + s // 2)
    return cen


def _accepted(cen, lev, c, b, theta2, far=False):
    if far:
        e = np.maximum(cen[c] - b[:3], b[3:] - cen[c])
    else:
        e = np.maximum(0, np.maximum(b[:3] - cen[c], cen[c] - b[3:]))
    d2 = float(e @ e)                                   # an exact integer
    return 2.0 ** (2 * (22 - int(lev[c]))) < theta2 * d2


def _box(g, k):
    return np.concatenate([2 * g.qmin[k].astype(np.int64), 2 * g.qmax[k].astype(np.int64) + 2])


def _walk(t, cen, start, b, theta2, out):
    stack = list(start)
    while stack:
        c = stack.pop()
        if _accepted(cen, t.level, c, b, theta2):
            out[1].append(c)
        elif t.nchild[c] == 0:
            out[0].extend(range(int(t.begin[c]), int(t.begin[c] + t.count[c])))
        else:
            stack.extend(range(int(t.first_child[c]), int(t.first_child[c] + t.nchild[c])))


def _run_lists(t, g, theta):
    """Every group's (EPJ, SPJ) under the shared-run rule, and the number of shared runs."""
    cen = _centres(t)
    theta2 = theta * theta
    lists, shared_runs = [None] * g.n, 0
    for r0 in range(0, g.n, RUN):
        r1 = min(r0 + RUN, g.n)
        B = _box(g, r0)
        for k in range(r0 + 1, r1):
            b = _box(g, k)
            B[:3], B[3:] = np.minimum(B[:3], b[:3]), np.maximum(B[3:], b[3:])
        shared = r1 - r0 > 1 and g.root[r0] == g.root[r1 - 1]
        common, front = ([], []), []
        if shared:
            stack = [int(g.root[r0])]
            while stack:
                c = stack.pop()
                if _accepted(cen, t.level, c, B, theta2):
                    common[1].append(c)
                elif _accepted(cen, t.level, c, B, theta2, far=True):
                    front.append(c)
                elif t.nchild[c] == 0:
                    common[0].extend(range(int(t.begin[c]), int(t.begin[c] + t.count[c])))
                else:
                    stack.extend(range(int(t.first_child[c]),
                                       int(t.first_child[c] + t.nchild[c])))
            shared = len(front) <= FRONT
        shared_runs += shared
        for k in range(r0, r1):
            out = (list(common[0]), list(common[1])) if shared else ([], [])
            _walk(t, cen, front if shared else [int(g.root[k])], _box(g, k), theta2, out)
            lists[k] = out
    return lists, shared_runs


@pytest.mark.parametrize("name,make,n_leaf,n_group,theta,min_shared", [
    ("clustered", lambda: I.clustered(n_background=2048, n_clusters=4, n_per_cluster=512,
                                      seed=3, eps=1e-3), 8, 64, 0.5, 0.8),
    ("plummer_theta1", lambda: I.plummer(3000, seed=5, eps=0.01), 8, 32, 1.0, 0.8),
    # a small opening angle: frontiers outgrow the 224 kept cells, groups walked alone
    ("plummer_theta02", lambda: I.plummer(2000, seed=6, eps=0.01), 4, 16, 0.2, 0.0),
    # many small systems: runs straddle systems
    ("ensemble", lambda: I.ensemble(n_sys=9, seed=8, nmin=40, nmax=700), 8, 32, 0.6, 0.3),
])
def test_shared_runs_give_every_group_its_own_list(name, make, n_leaf, n_group, theta,
                                                   min_shared):
    ps = make()
    t = O.build_tree(ps, n_leaf, moments=False)
    g = O.make_groups(t, n_group)
    ref = O.walk(t, g, theta)
    lists, shared_runs = _run_lists(t, g, theta)
    for k in range(g.n):
        e_ref, s_ref = ref.group_lists(k)
        assert sorted(lists[k][0]) == sorted(int(v) for v in e_ref), (name, k)
        assert sorted(lists[k][1]) == sorted(int(v) for v in s_ref), (name, k)
    runs = (g.n + RUN - 1) // RUN
    assert shared_runs >= min_shared * runs, (name, shared_runs, runs)
    if name == "plummer_theta02":
        assert shared_runs < runs                       # the fallback is exercised


def test_far_corner_test_separates_opened_from_undecided_cells():
    # a cell that fails the test at the run box's far corners is accepted by no member, while
    # some cells that fail only the near test are accepted by a member: without the frontier
    # those members would lose entries
    ps = I.plummer(1500, seed=9, eps=0.01)
    t = O.build_tree(ps, 8, moments=False)
    g = O.make_groups(t, 32)
    cen = _centres(t)
    theta2 = 0.25
    lost = 0
    for r0 in range(0, g.n - RUN + 1, RUN):
        B = _box(g, r0)
        for k in range(r0 + 1, r0 + RUN):
            b = _box(g, k)
            B[:3], B[3:] = np.minimum(B[:3], b[:3]), np.maximum(B[3:], b[3:])
        for c in range(t.n_cells):
            if _accepted(cen, t.level, c, B, theta2):
                continue
            if not _accepted(cen, t.level, c, B, theta2, far=True):
                # opened by every member: no member accepts it
                assert not any(_accepted(cen, t.level, c, _box(g, k), theta2)
                               for k in range(r0, r0 + RUN))
            elif any(_accepted(cen, t.level, c, _box(g, k), theta2) for k in range(r0, r0 + RUN)):
                lost += 1                               # a frontier cell some member accepts
    assert lost > 0


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_xcd_aware_run_order_is_a_permutation(tmp_path):
    # the walk kernel's launch rule and wave -> run mapping (walk_order.h), compiled into a
    # small host program: every run is taken exactly once per grid-wide round
    exe = tmp_path / "walk_order_check"
    src = os.path.join(ROOT, "tests", "native", "walk_order_check.cpp")
    inc = os.path.join(ROOT, "paper_1601_03138_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", inc, src, "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
