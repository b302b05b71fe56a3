"""Host-side checks of the benchmark's contract (no GPU needed)."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from workloads import make  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""          # no JSON line


def test_algorithmic_bytes_of_the_deblurring_workload():
    """Per-launch bytes at the 256 x 256 deblurring workload, worked out by hand from its sizes
    (m = n = 65,536, p = 131,072, nnz(A) = 5,216,656, nnz(L) = 261,120, FP32 values, s = 400,
    zeta = 8):
      SpMV of the new column: 8 (nnz(A) + nnz(L)) = 43,822,208 for values and columns,
        4 (m + 1) + 4 (p + 1) = 786,440 for row pointers, 8 n = 524,288 for w,
        8 m + 8 p = 1,572,864 for A w and L w: 46,705,800;
      scatter: (8 + 2 zeta)(m + p) = 4,718,592 for the images and the int16 pattern,
        16 s = 6,400 for the bins: 4,724,992;
      gradient at d = 50: 8 n d = 26,214,400 for the columns of H W,
        16 n = 1,048,576 for A^T b and r: 27,262,976."""
    P = make("deblur2d", 0, "full")
    assert (P.m, P.n, P.p, P.A.nnz, P.L.nnz, P.s, P.zeta, P.dtype) == \
        (65536, 65536, 131072, 5216656, 261120, 400, 8, "f32")
    ab = bench.algorithmic_bytes(P, 50, "maintained")
    assert ab["spmv_new_column"] == 46_705_800
    assert ab["sketch_scatter"] == 4_724_992
    assert ab["gemv"] == 27_262_976


def _profile_commands():
    out = []
    d = os.path.join(ROOT, "profiles")
    for f in sorted(os.listdir(d)):
        p = os.path.join(d, f)
        if f.endswith(".json"):
            out.append((f, json.load(open(p))["command"]))
        else:
            for line in open(p):
                if line.startswith("# command:"):
                    out.append((f, line.split(":", 1)[1].strip()))
    return out


def test_profiles_name_commands_that_run_committed_files():
    cmds = _profile_commands()
    assert cmds, "no profile summaries"
    for f, cmd in cmds:
        assert "_work" not in cmd, f
        scripts = re.findall(r"python3? (?!-m)(\S+\.py)", cmd)
        modules = re.findall(r"python3? -m (\S+)", cmd)
        assert scripts or modules, (f, cmd)
        for s in scripts:
            assert os.path.isfile(os.path.join(ROOT, s)), (f, s)
        for m in modules:
            assert os.path.isfile(os.path.join(ROOT, *m.split(".")) + ".py"), (f, m)


def test_stale_profiles_are_not_used():
    """Traffic and trace figures are taken only from summaries of the current sources."""
    assert bench.load_traffic("kb_forward", "deblur2d", "0" * 16) is None
    assert bench.load_trace_avg("kb_forward", "deblur2d", "0" * 16) is None
    h = bench.source_hash()
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_kb_forward_deblur2d.json")))
    if t["source_hash"] != h:
        pytest.skip("committed profiles predate the current sources")
    assert bench.load_traffic("kb_forward", "deblur2d", h) == t["bytes_per_launch"]
    assert bench.load_trace_avg("kb_forward", "deblur2d", h) > 0
