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
      adjoint: 43,822,208 + 8 (n + 1) = 524,296 for the two transposed row-pointer
        arrays, 8 m + 8 p = 1,572,864 for (u, t), 8 n = 524,288 for the result: 46,443,656;
      scatter: 8 (m + p) = 1,572,864 for the images (the pattern is hashable: no bytes),
        16 s = 6,400 for the two bin vectors: 1,579,264;
      gradient at d = 50: 8 n d = 26,214,400 for the columns of H W,
        16 n = 1,048,576 for A^T b and r: 27,262,976."""
    P = make("deblur2d", 0, "full")
    assert (P.m, P.n, P.p, P.A.nnz, P.L.nnz, P.s, P.zeta, P.dtype) == \
        (65536, 65536, 131072, 5216656, 261120, 400, 8, "f32")
    assert bench.launch_bytes(P, "spmv_new_column") == 46_705_800
    assert bench.launch_bytes(P, "adjoint") == 46_443_656
    assert bench.launch_bytes(P, "sketch_scatter") == 1_579_264
    assert bench.launch_bytes(P, "gradient", 50) == 27_262_976


def test_expected_launches_of_one_step():
    """One expansion per k: gradient, new-column SpMV, H W adjoint (own launch unless fused
    into the append), scatter, append; with refinement the maintained form adds the new
    column of W^T H W and one launch for all the steps, the direct form a gradient, W^T r
    and the update per step; the solution adds one GEMV over ell + k columns."""
    P = make("deblur2d", 0, "small")
    ex = bench.expected_launches(P, "maintained", fused_hw=True)
    assert len(ex["gemv"]) == P.k + 1
    assert "adjoint" not in ex
    assert ex["qr_append_solve"] == [bench.launch_bytes(P, "adjoint")] * P.k
    ex = bench.expected_launches(P, "maintained", fused_hw=False)
    assert len(ex["adjoint"]) == P.k and ex["qr_append_solve"] == [0] * P.k
    Q = make("ct2d", 0, "small")
    assert Q.refine_steps == 2
    ex = bench.expected_launches(Q, "maintained", fused_hw=False)
    # maintained form: the steps run on W^T H W, whose new column is one W^T v pass
    assert len(ex["gemv"]) == Q.k + 1
    assert len(ex["gemvt_WTr"]) == Q.k and len(ex["refine_step"]) == Q.k
    d0 = Q.ell
    assert ex["gemv"][0] == bench.launch_bytes(Q, "gradient", d0)
    assert ex["gemv"][1] == bench.launch_bytes(Q, "gradient", d0 + 1)   # the next expansion
    assert ex["gemvt_WTr"][0] == bench.launch_bytes(Q, "gemvt", d0 + 1)
    assert ex["gemv"][-1] == bench.launch_bytes(Q, "gemv", Q.ell + Q.k)
    ex = bench.expected_launches(Q, "direct", fused_hw=False)
    assert len(ex["gemv"]) == Q.k * (1 + Q.refine_steps) + 1
    assert len(ex["gemvt_WTr"]) == Q.k * Q.refine_steps


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
    d = os.path.join(ROOT, "profiles")
    traffic = sorted(f for f in os.listdir(d) if f.startswith("traffic_") and f.endswith(".json"))
    assert traffic
    t = json.load(open(os.path.join(d, traffic[0])))
    assert bench.load_traffic(t["kernel"], t["workload"], "0" * 16) is None
    assert bench.load_trace_avg(t["kernel"], t["workload"], "0" * 16) is None
    h = bench.source_hash()
    if t["source_hash"] != h:
        pytest.skip("committed profiles predate the current sources")
    assert bench.load_traffic(t["kernel"], t["workload"], h) == t["bytes_per_launch"]
    assert bench.load_trace_avg(t["kernel"], t["workload"], h) > 0
