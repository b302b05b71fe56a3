#!/usr/bin/env python3
"""Benchmark of the sGKS hot path on one MI355X.

Headline: the dynamic CT workload, the largest single-GPU configuration
(30 frames of 128 x 128, n = 491,520; block-diagonal parallel-beam CT operator,
m = 327,600, 37.5 M nonzeros with FP32 values; space-time difference operator,
p = 1,474,560; sparse-sign sketch s = 800, zeta = 8; k = 200 expansions).
One step is the whole workload: sgks_create (transposes, sketch of b, initial
Krylov basis, QR factors), 200 expansions, x_k = W y written to device memory,
and the frozen-basis backward of ||x_k - x_true||^2 with respect to b and mu.
The operators and b are resident in device memory before the timed region.

The timed region runs the production path (kernel-by-kernel launches on the
caller's stream plus the library's side stream).  A second, profiled pass runs
the same steps with HIP events bound to every kernel launch (its begin and end
of execution, as a kernel trace reports them); their averages give each
kernel's time, and algorithmic bytes per launch / average time give its
achieved bandwidth.  The roofline line is that of the kernel with the largest
total time.

Secondary lines (same measurement): 2D deblurring (its operators stay inside the
256 MB Infinity Cache, so its bandwidth is not HBM evidence) and CT with two
refinement steps per projected solve.  Then the 32-problem uneven batch against
its 32 plain solves, the backward against the forward, and the FP64 CPU oracle:
its full solve of the headline workload on one thread (the reference of the
relative error), and a bounded sample of the same workload on every host core.

Printed: one JSON line on stdout (progress goes to stderr).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HEADLINE = "dynamic_ct"

# The paper's own timings, quoted as context only (another machine, another sketch,
# other test problems; not a target): Sec. 4.2.2, Exp. 3 (seismic travel-time
# tomography) and Sec. 4.3, Exp. 4 (dynamic CT), totals divided by the iteration count.
PAPER_CONTEXT = {
    "note": "context only: laptop CPU, MATLAB, FP64, SRTT sketch, other test problems",
    "hardware": "Intel Core i7-8750H @ 2.2 GHz, 128 GB RAM",
    "exp3_travel_time_n65536": {"sgks_total_s": 27, "iterations": 300, "iters_per_s": 11.1},
    "exp4_dynamic_ct_n655360": {"sgks_total_s": 33, "iterations": 400, "iters_per_s": 12.1,
                                "gks_total_s": 99},
}


def log(*a):
    """Progress on stderr (the JSON line is the only stdout output)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_18073_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ----------------------------------------------------------------------------
# algorithmic bytes
# ----------------------------------------------------------------------------

def launch_bytes(P, kind, d=0):
    """Minimal HBM bytes of one launch: CSR values and indices once, row pointers once,
    every vector read and written once, the d columns of W (or H W) for the dense
    products; the sketch pattern is hashable, so it counts zero bytes."""
    vsz = 4 if P.dtype == "f32" else 8
    nnz = P.A.nnz + P.L.nnz
    m, n, p, s = P.m, P.n, P.p, P.s
    if kind == "spmv_new_column":      # z = A w, L w: CSR, row pointers, w read; z written
        return (vsz + 4) * nnz + 4 * (m + 1) + 4 * (p + 1) + 8 * n + 8 * m + 8 * p
    if kind == "adjoint":              # A^T u + mu L^T t: transposed CSR, (u, t) read, n written
        return (vsz + 4) * nnz + 8 * (n + 1) + 8 * m + 8 * p + 8 * n
    if kind == "forward_Ax_Lx":        # direct form: u = A x - b, t = L x
        return (vsz + 4) * nnz + 4 * (m + 1) + 4 * (p + 1) + 8 * n + 8 * m + 8 * m + 8 * p
    if kind == "sketch_scatter":       # (u, t) read, the two s-vectors of bins written
        return 8 * (m + p) + 16 * s
    if kind == "gradient":             # r = (H W) y - A^T b: d columns, A^T b read, r written
        return 8 * n * d + 16 * n
    if kind == "gemv":                 # x = W y: d columns read, x written
        return 8 * n * d + 8 * n
    if kind == "gemvt":                # W^T r partials: d columns and r read
        return 8 * n * d + 8 * n
    return 0


def expected_launches(P, form="maintained", fused_hw=False, backward=False):
    """{phase: [bytes of each launch]} of one step (create excluded), in launch order."""
    ell, k, ir = P.ell, P.k, P.refine_steps
    out = {}

    def add(ph, b):
        out.setdefault(ph, []).append(b)
    for i in range(k):
        d = ell + i
        if form == "maintained":
            add("gemv", launch_bytes(P, "gradient", d))
        else:
            add("gemv", launch_bytes(P, "gemv", d))
            add("forward_Ax_Lx", launch_bytes(P, "forward_Ax_Lx"))
            add("adjoint", launch_bytes(P, "adjoint"))
        add("spmv_new_column", launch_bytes(P, "spmv_new_column"))
        if form == "maintained" and not fused_hw:
            add("adjoint", launch_bytes(P, "adjoint"))
        add("sketch_scatter", launch_bytes(P, "sketch_scatter"))
        # the append launch: with the H W adjoint inside it, that adjoint's bytes
        add("qr_append_solve", launch_bytes(P, "adjoint") if fused_hw else 0)
        if form == "maintained" and ir:
            # the new column of W^T H W (the d + 1 columns of W against the new H W
            # column), then every refinement step on the small matrix in one launch
            add("gemvt_WTr", launch_bytes(P, "gemvt", d + 1))
            add("refine_step", 0)
        for _ in range(ir if form != "maintained" else 0):
            add("gemv", launch_bytes(P, "gemv", d + 1))
            add("forward_Ax_Lx", launch_bytes(P, "forward_Ax_Lx"))
            add("adjoint", launch_bytes(P, "adjoint"))
            add("gemvt_WTr", launch_bytes(P, "gemvt", d + 1))
            add("refine_step", 0)
    add("gemv", launch_bytes(P, "gemv", ell + k))       # x_k = W y
    return out


# phase -> kernel of the maintained form
def phase_kernel(phase, tuning, fused_hw, form="maintained"):
    if phase == "gemv":
        return "kb_gradient" if form == "maintained" else "kb_gemv"
    if phase in ("spmv_new_column", "forward_Ax_Lx"):
        return "kb_forward"
    if phase == "adjoint":
        return "kb_adjoint"
    if phase == "sketch_scatter":
        return "kb_scatter"
    if phase == "gemvt_WTr":
        return "kb_mcol" if form == "maintained" else "kb_gemvt"
    if phase == "refine_step":
        return "k_mrefine" if form == "maintained" else "k_refine"
    if phase == "qr_append_solve":
        if (tuning or {}).get("append_groups", 1) == 1:
            return "k_ap1_side_hw" if fused_hw else "k_ap1_side"
        return "append_chain"
    return phase


# ----------------------------------------------------------------------------
# committed rocprofv3 summaries
# ----------------------------------------------------------------------------

def load_traffic(kernel, workload, shash):
    """HBM traffic per launch from committed rocprofv3 counter runs, if still current."""
    f = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(f):
        return None
    try:
        t = json.load(open(f))
    except Exception:
        return None
    if t.get("source_hash") != shash:
        return None
    return t.get("bytes_per_launch")


def load_trace_avg(kernel, workload, shash):
    """Average duration (us) of a kernel in the committed rocprofv3 kernel-trace summary of
    the workload, if that summary is of the current sources."""
    f = os.path.join(ROOT, "profiles", f"kernel_trace_{workload}.txt")
    if not os.path.exists(f):
        return None
    lines = open(f).read().splitlines()
    if not any(l.strip() == f"# source_hash: {shash}" for l in lines):
        return None
    for l in lines:
        parts = l.split()
        if parts and not l.startswith("#") and parts[0].split("<")[0].endswith("::" + kernel):
            try:
                return float(parts[-4])
            except (ValueError, IndexError):
                return None
    return None


# ----------------------------------------------------------------------------
# CPU oracle (worker processes; started before the GPU is touched)
# ----------------------------------------------------------------------------

def _oracle_full(name, want_x=True):
    """One full oracle solve of a workload on one thread: (x, seconds, iterations)."""
    from threadpoolctl import threadpool_limits
    from oracle import sgks_oracle as O
    from workloads import make
    P = make(name, 0, "full")
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ref = O.sgks(P.A, P.L, P.b, P.mu, P.k, P.s, P.seed, zeta=P.zeta, ell=P.ell,
                     refine_steps=P.refine_steps)
        dt = time.perf_counter() - t0
    return (ref.x if want_x else None), dt, ref.iters


def _oracle_sample(name, k):
    """Create + k iterations of the oracle on one thread: (iterations, seconds)."""
    from threadpoolctl import threadpool_limits
    from oracle import sgks_oracle as O
    from workloads import make
    P = make(name, 0, "full")
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.sgks(P.A, P.L, P.b, P.mu, k, P.s, P.seed, zeta=P.zeta, ell=P.ell,
               refine_steps=P.refine_steps)
        dt = time.perf_counter() - t0
    return k, dt


def _oracle_batch_problem(i, k):
    """Oracle x_k of problem i of the uneven batch and kappa(G_k)."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import sgks_oracle as O
    from workloads import generators as gen
    P = gen.batch_problem(i)
    with threadpool_limits(1):
        ref = O.sgks(P.A, P.L, P.b, P.mu, k, P.s, P.seed, zeta=P.zeta, ell=P.ell)
    d = P.ell + ref.iters
    kap = float(np.linalg.cond(np.vstack([ref.R_A[:d, :d], math.sqrt(P.mu) * ref.R_L[:d, :d]])))
    return ref.x, kap


def host_cores():
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    model = None
    try:
        for l in open("/proc/cpuinfo"):
            if l.startswith("model name"):
                model = l.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": share, "model": model}


# ----------------------------------------------------------------------------
# GPU measurement of one workload
# ----------------------------------------------------------------------------

def total_adjoint_cost(G, torch, np, P, order, reps=3):
    """The total-derivative adjoint (sgks_backward_total) at the workload's k, outside
    the timed steps: the forward solve with its y history recorded, then the reverse
    sweep, each timed with the stream synchronised (median of reps), and the sweep's
    rounding-error estimate d eps kappa(G)^2 (large once the basis is numerically
    rank-deficient: the gradient is then dominated by rounding)."""
    import warnings
    from workloads.generators import image_order
    dev = torch.device("cuda:0")
    A, L, b = G.upload_problem(P)
    opts = dict(ell=P.ell, max_iters=P.k, zeta=P.zeta, refine_steps=0, keep_history=True)
    io = image_order(P) if order else None
    if io is not None:
        opts["order"] = torch.as_tensor(io, dtype=torch.int32, device=dev)
    g = torch.as_tensor(2.0 * (np.zeros(P.n) - P.x_true), device=dev)
    fwd, bwd, est = [], [], None
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = G.SGKS(A, L, b, P.mu, P.s, P.seed, **opts)
        S.iterate(P.k)
        x = S.solution()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gx = 2.0 * x + g
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            _, _, est = S.backward_total(gx, with_error=True)
        t3 = time.perf_counter()
        S.close()
        if r:   # the first round warms up
            fwd.append(t1 - t0)
            bwd.append(t3 - t2)
    f, bk = 1e3 * float(np.median(fwd)), 1e3 * float(np.median(bwd))
    return {"k": P.k, "forward_with_history_ms": f, "backward_ms": bk,
            "backward_over_forward": bk / f, "err_est": est,
            "loss": "||x_k - x_true||^2", "timed": "outside the headline steps"}


def measure(G, torch, P, steps, warmup, *, backward, profile, graph=False, autotune=False,
            gradient="maintained", order=True):
    """Time `steps` complete solves of P (create + k expansions + x_k [+ backward]).
    order: work in the Morton order of the image's unknowns (the library's order option)."""
    from workloads.generators import image_order
    dev = torch.device("cuda:0")
    A, L, b = G.upload_problem(P)
    x = torch.empty(P.n, dtype=torch.float64, device=dev)
    xt = torch.as_tensor(P.x_true, device=dev)
    opts = dict(ell=P.ell, max_iters=P.k, zeta=P.zeta, refine_steps=P.refine_steps,
                graph=graph, autotune=autotune, gradient=gradient)
    io = image_order(P) if order else None
    if io is not None:
        opts["order"] = torch.as_tensor(io, dtype=torch.int32, device=dev)

    def step(acc, prof):
        t0 = time.perf_counter()
        S = G.SGKS(A, L, b, P.mu, P.s, P.seed, **opts)
        acc["tuning"] = S.tuning()
        t1 = time.perf_counter()
        if prof:
            S.profile(True)
        S.iterate(P.k)
        S.solution(out=x)
        if prof:
            ms, cnt = S.profile_read()
            for i in range(G.PHASES):
                acc["ms"][i] += ms[i]
                acc["n"][i] += cnt[i]
        if backward:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            acc["grad"] = S.backward(2.0 * (x - xt))
            acc["backward_s"] += time.perf_counter() - t2
        rc, it = S.status()
        if backward:
            acc["S_last"] = S
        else:
            S.close()
        acc["setup_s"] += t1 - t0
        assert rc == 0 and it == P.k, (rc, it)

    def fresh():
        return {"ms": [0.0] * G.PHASES, "n": [0] * G.PHASES, "setup_s": 0.0, "backward_s": 0.0}

    for _ in range(warmup):
        a = fresh()
        step(a, False)
        if "S_last" in a:
            a["S_last"].close()
    acc = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        if "S_last" in acc:
            acc.pop("S_last").close()
        step(acc, False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {
        "value": steps * P.k / wall,
        "ms_per_step": 1e3 * wall / steps,
        "setup_ms_per_step": 1e3 * acc["setup_s"] / steps,
        "iterate_only_iters_per_s": steps * P.k / (wall - acc["setup_s"] - acc["backward_s"]),
        "launch_shapes": acc.get("tuning"),
        "x": x.cpu().numpy(),
    }
    if backward:
        out["backward_ms_per_step"] = 1e3 * acc["backward_s"] / steps
        out["forward_ms_per_step"] = out["ms_per_step"] - out["backward_ms_per_step"]
        out["grad"] = acc["grad"]
        out["solver"] = acc.pop("S_last")
    if not profile:
        return out
    pacc = fresh()
    torch.cuda.synchronize()
    for _ in range(steps):
        step(pacc, True)
        if "S_last" in pacc:
            pacc.pop("S_last").close()
    names = G.PHASE_NAMES
    phase = {names[i]: {"ms_total": pacc["ms"][i], "launches": pacc["n"][i],
                        "us_avg": 1e3 * pacc["ms"][i] / pacc["n"][i]}
             for i in range(G.PHASES) if pacc["n"][i]}
    out["phases"] = phase
    tuning = acc.get("tuning") or {}
    fused = bool(tuning.get("append_groups", 1) == 1 and gradient == "maintained"
                 and phase.get("adjoint", {}).get("launches", 0) == 0)
    exp = expected_launches(P, gradient, fused)
    kern = {}
    for ph, v in phase.items():
        kname = phase_kernel(ph, tuning, fused, gradient)
        blist = exp.get(ph, [])
        nl = v["launches"]
        # every phase launches one kernel per launch listed, except the append chain
        per = blist if len(blist) * steps == nl else None
        by = (sum(per) * steps) if per is not None else 0.0
        e = kern.setdefault(kname, {"ms_total": 0.0, "launches": 0, "bytes_total": 0.0})
        e["ms_total"] += v["ms_total"]
        e["launches"] += nl
        e["bytes_total"] += by
    for kname, e in kern.items():
        e["us_avg"] = 1e3 * e["ms_total"] / e["launches"]
        e["bytes_per_launch"] = e["bytes_total"] / e["launches"]
        e["GBps"] = e["bytes_total"] / (e["ms_total"] * 1e-3) / 1e9 if e["ms_total"] > 0 else 0.0
        e["share_of_kernel_time"] = e["ms_total"] / sum(v["ms_total"] for v in kern.values())
        del e["bytes_total"]
    out["kernels"] = kern
    # the dominant kernel: the one kernel with the most time ("append_chain" is the
    # 5 + 2 (passes - 1) distinct kernels of the multi-workgroup append, each with a
    # fraction of that phase's time, so it is not a candidate)
    dom = max((k for k in kern if k != "append_chain"), key=lambda k: kern[k]["ms_total"])
    shash = source_hash()
    e = kern[dom]
    roof = {"bound": "hbm" if e["bytes_per_launch"] > 0 else "latency", "kernel": dom,
            "achieved": e["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": e["GBps"] / HBM_PEAK_GBS, "traffic": load_traffic(dom, P.name, shash),
            "algorithmic_bytes_per_launch": e["bytes_per_launch"], "avg_launch_us": e["us_avg"],
            "share_of_kernel_time": e["share_of_kernel_time"], "source_hash": shash}
    tavg = load_trace_avg(dom, P.name, shash)
    if tavg:
        roof["rocprof_avg_us"] = tavg
        roof["achieved_at_rocprof_avg"] = e["bytes_per_launch"] / (tavg * 1e-6) / 1e9
    out["roofline"] = roof
    sk = ["kb_forward", "kb_adjoint", "kb_scatter"]
    if fused:
        sk.append("k_ap1_side_hw")   # carries the H W adjoint SpMV
    tb = sum(kern[k]["bytes_per_launch"] * kern[k]["launches"] for k in sk if k in kern)
    tt = sum(kern[k]["ms_total"] for k in sk if k in kern) * 1e-3
    out["spmv_sketch_GBps"] = tb / tt / 1e9 if tt > 0 else None
    out["spmv_sketch_frac_of_hbm_peak"] = (out["spmv_sketch_GBps"] / HBM_PEAK_GBS
                                           if out["spmv_sketch_GBps"] else None)
    out["spmv_sketch_kernels"] = [k for k in sk if k in kern]
    return out


def describe(P):
    m = P.meta
    if P.name == "dynamic_ct":
        return (f"dynamic CT: {m['nt']} frames of {m['N']}x{m['N']} (n={P.n}), {m['n_angles']} "
                f"angles per frame rotating between frames x {m['n_det']} detectors "
                f"(m={P.m}), block-diagonal Siddon CSR nnz={P.A.nnz} ({P.dtype} values), "
                f"space-time L {P.p}x{P.n} nnz={P.L.nnz}, sparse-sign s={P.s} zeta={P.zeta}, "
                f"k={P.k}, mu={P.mu}, ell={P.ell}; one step = create + {P.k} expansions + x_k "
                f"+ backward of ||x_k - x_true||^2 w.r.t. b and mu")
    if P.name == "deblur2d":
        return (f"2D deblurring: {m['N']}x{m['N']} image (n={P.n}), 9x9 Gaussian PSF CSR "
                f"nnz={P.A.nnz} ({P.dtype} values), L=[Dx;Dy] {P.p}x{P.n} nnz={P.L.nnz}, "
                f"s={P.s}, k={P.k}, mu={P.mu}; one step = create + {P.k} expansions + x_k")
    if P.name == "ct2d":
        return (f"2D parallel-beam CT: {m['N']}x{m['N']} (n={P.n}), {m['n_angles']} angles x "
                f"{m['n_det']} detectors (m={P.m}), Siddon CSR nnz={P.A.nnz} ({P.dtype} values), "
                f"L=[Dx;Dy] nnz={P.L.nnz}, s={P.s}, k={P.k}, {P.refine_steps} refinement steps "
                f"per projected solve; one step = create + {P.k} expansions + x_k")
    if P.name == "ct_exp2":
        return (f"Exp. 2 shape: {m['N']}x{m['N']} parallel-beam CT (n={P.n}), {m['n_angles']} "
                f"angles x {m['n_det']} detectors (m={P.m}), nnz={P.A.nnz}, L {P.p}x{P.n}, "
                f"s={P.s}, k={P.k}, mu={P.mu}; one step = create + {P.k} expansions + x_k")
    if P.name == "traveltime_exp3":
        return (f"Exp. 3 shape: {m['N']}x{m['N']} travel-time tomography (n={P.n}), every "
                f"source-receiver pair a straight ray (m={P.m}), nnz={P.A.nnz}, L {P.p}x{P.n}, "
                f"s={P.s}, k={P.k}, mu={P.mu}; one step = create + {P.k} expansions + x_k")
    if P.name == "dynamic_ct_exp4":
        return (f"Exp. 4 shape: {m['nt']} frames of {m['N']}x{m['N']} (n={P.n}), "
                f"{m['n_angles']} angles per frame in its own sector x {m['n_det']} detectors "
                f"(m={P.m}), nnz={P.A.nnz}, space-time L {P.p}x{P.n} nnz={P.L.nnz}, s={P.s}, "
                f"k={P.k}, mu={P.mu}; one step = create + {P.k} expansions + x_k")
    return P.name


# the paper's sGKS totals for its Exp. 3 and Exp. 4 (context only, see PAPER_CONTEXT)
PAPER_TOTALS = {"traveltime_exp3": PAPER_CONTEXT["exp3_travel_time_n65536"],
                "dynamic_ct_exp4": PAPER_CONTEXT["exp4_dynamic_ct_n655360"]}


def bench_paper_scale(G, torch, make, order=True):
    """The paper's experiment shapes at full size (synthetic data): whole solves."""
    from workloads.generators import PAPER_SCALE
    out = {}
    for name in PAPER_SCALE:
        Q = make(name, 0, "full")
        try:
            r = measure(G, torch, Q, 2, 1, backward=False, profile=False, order=order)
        except Exception as e:      # reported, never fatal to the measurement
            out[name] = {"workload": describe(Q), "error": repr(e)}
            continue
        if "solver" in r:
            r["solver"].close()
        ent = {"workload": describe(Q), "value": r["value"], "unit": "iters/s",
               "ms_per_solve": r["ms_per_step"], "setup_ms": r["setup_ms_per_step"],
               "iterate_only_iters_per_s": r["iterate_only_iters_per_s"],
               "rre_gpu": float(((r["x"] - Q.x_true) ** 2).sum() ** 0.5 /
                                (Q.x_true ** 2).sum() ** 0.5)}
        if name in PAPER_TOTALS:
            ent["paper_context"] = dict(PAPER_TOTALS[name], note=PAPER_CONTEXT["note"])
        out[name] = ent
        log(f"paper scale {name}: {r['value']:.1f} iters/s")
    return out


def bench_gks(G, torch, np, P, steps=2, order=True):
    """GKS (Alg. 1) against sGKS on the same GPU and workload: whole solves and the
    expansions alone (Sec. 4.2.1 and Sec. 4.3 compare the two per iteration)."""
    from workloads.generators import image_order
    A, L, b = G.upload_problem(P)
    io = image_order(P) if order else None
    out = {}
    for method in ("gks", "sgks"):
        opts = dict(ell=P.ell, max_iters=P.k, zeta=P.zeta, method=method,
                    refine_steps=P.refine_steps if method == "sgks" else 0)
        if io is not None:
            opts["order"] = torch.as_tensor(io, dtype=torch.int32, device="cuda")
        S = G.SGKS(A, L, b, P.mu, P.s, P.seed, **opts)   # warm-up
        S.iterate(2)
        S.close()
        setup = it = 0.0
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S = G.SGKS(A, L, b, P.mu, P.s, P.seed, **opts)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            S.iterate(P.k)
            x = S.solution()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            setup += t1 - t0
            it += t2 - t1
            rc, n = S.status()
            S.close()
        out[method] = {"iters_per_s": steps * P.k / (setup + it),
                       "iterate_only_iters_per_s": steps * P.k / it,
                       "ms_per_expansion": 1e3 * it / (steps * P.k), "status": [rc, n],
                       "rre": float(np.linalg.norm(x.cpu().numpy() - P.x_true) /
                                    np.linalg.norm(P.x_true))}
    out["sgks_speedup_per_expansion"] = out["gks"]["ms_per_expansion"] / out["sgks"]["ms_per_expansion"]
    return out


def bench_batch(G, torch, np, make, oracle_refs, order=True, plain=True):
    """The 32-problem uneven batch: one batched solve against the 32 plain solves
    (plain=False: the batched solve only)."""
    from workloads.generators import image_order
    Ps = make("batch", 0, "full")
    data = G.upload_batch(Ps, orders=[image_order(P) for P in Ps] if order else None)
    k = Ps[0].k
    opts = dict(ell=Ps[0].ell, max_iters=k, zeta=Ps[0].zeta, autotune=True)
    B = G.SGKSBatch(data, **opts)      # warm-up (module load, autotuning cached per shape)
    B.iterate(2)
    B.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = G.SGKSBatch(data, **opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B.iterate(k)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    xb = [x.cpu().numpy() for x in B.solutions()]
    st_b = [B.problem(i).status() for i in range(len(Ps))]
    B.close()
    setup_p = iter_p = 0.0
    same = True
    for i, pr in enumerate(data if plain else []):
        A, L, b, mu, s, seed = pr[:6]
        torch.cuda.synchronize()
        u0 = time.perf_counter()
        S = G.SGKS(A, L, b, mu, s, seed, order=pr[6] if len(pr) > 6 else None, **opts)
        torch.cuda.synchronize()
        u1 = time.perf_counter()
        S.iterate(k)
        torch.cuda.synchronize()
        u2 = time.perf_counter()
        setup_p += u1 - u0
        iter_p += u2 - u1
        same = same and np.array_equal(S.solution().cpu().numpy(), xb[i]) and S.status() == st_b[i]
        S.close()
    total = sum(st[1] for st in st_b)
    errs = {}
    for i, fut in oracle_refs.items():
        xo, kap = fut.get()
        errs[str(i)] = {"problem": f"{Ps[i].name} N={Ps[i].meta['N']}",
                        "rel_err_vs_oracle": float(np.linalg.norm(xb[i] - xo) / np.linalg.norm(xo)),
                        "kappa_G_k": kap}
    bulk = 0.0
    for P in Ps:
        ex = expected_launches(P, "maintained", False)
        bulk += sum(sum(v) for v in ex.values())
    if not plain:
        return {"workload": f"{len(Ps)} problems, batched solve only", "problem_iterations": total,
                "batched_iters_per_s": total / (t2 - t0),
                "batched_iterate_only_iters_per_s": total / (t2 - t1),
                "batched_setup_ms": 1e3 * (t1 - t0), "sample_rel_err_vs_oracle": errs}
    return {
        "workload": (f"{len(Ps)} problems (deblurring / CT / travel time, sides 64..256 "
                     f"log-uniform, own mu), total n={sum(P.n for P in Ps)}, total nnz(A)="
                     f"{sum(P.A.nnz for P in Ps)}, s={Ps[0].s}, k={k}, FP32 operators, "
                     f"autotuned launch shapes"),
        "problem_iterations": total,
        "batched_iters_per_s": total / (t2 - t0),
        "batched_iterate_only_iters_per_s": total / (t2 - t1),
        "batched_setup_ms": 1e3 * (t1 - t0),
        "plain_iters_per_s": total / (setup_p + iter_p),
        "plain_iterate_only_iters_per_s": total / iter_p,
        "plain_setup_ms": 1e3 * setup_p,
        "speedup_whole": (setup_p + iter_p) / (t2 - t0),
        "speedup_iterate_only": iter_p / (t2 - t1),
        "batched_iteration_ms": 1e3 * (t2 - t1) / k,
        "bulk_algorithmic_GBps_batched": bulk / (t2 - t1) / 1e9,
        "bitwise_equal_to_plain": bool(same),
        "equal_rel_err": ("every problem's x_k is bit-for-bit its plain solve's, so the two rel "
                          "errs vs the oracle are equal" if same else "MISMATCH"),
        "sample_rel_err_vs_oracle": errs,
    }


def adjoint_rel_err(G, np, P, res):
    """grad_b, grad_mu of the headline step against the oracle's frozen adjoint taken on the
    GPU's own basis and factors."""
    from oracle import sgks_oracle as O
    S = res["solver"]
    gb, gmu = res["grad"]
    st = {k: S.state(k) for k in ("y", "W", "Q_A", "R_A", "Q_L", "R_L", "d_A", "G", "c_b")}
    S.close()
    x = res["x"]
    r = O.Result(x, st["y"], st["W"], st["Q_A"], st["R_A"], st["Q_L"], st["R_L"], st["d_A"],
                 st["G"], st["c_b"], P.k, 0, [], [])
    gb_ref, gmu_ref = O.frozen_adjoint_b(r, P.mu, 2 * (x - P.x_true), P.A, P.L, P.s, P.seed,
                                         P.zeta)
    gbh = gb.cpu().numpy()
    return {"grad_b_rel_err": float(np.linalg.norm(gbh - gb_ref) / np.linalg.norm(gb_ref)),
            "grad_mu_rel_err": float(abs(gmu - gmu_ref) / abs(gmu_ref)), "grad_mu": gmu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=10)
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-cores oracle sample (default: the host's CPU "
                         "share, at most 16)")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the profiled pass (no per-kernel times, no roofline)")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of captured graphs instead of kernel-by-kernel launches")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary workloads and the batched comparison")
    ap.add_argument("--gradient", choices=["maintained", "direct"], default="maintained")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time its launch shapes at create (cached per shape)")
    ap.add_argument("--no-order", action="store_true",
                    help="work in the caller's row-major order of the unknowns instead of "
                         "the Morton order of each image frame")
    ap.add_argument("--no-plain", action="store_true",
                    help="with --workload batch: time the batched solve only (no plain solves)")
    ap.add_argument("--no-total-adjoint", action="store_true",
                    help="skip the total-derivative adjoint measured beside the headline")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(see the sharding design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the oracle's worker processes start before anything touches the GPU
    pool = None
    cores = host_cores()
    nwork = args.cpu_workers or max(1, min(16, cores["affinity"]))
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(processes=max(2, nwork))
        full_ref = pool.apply_async(_oracle_full, (args.workload,))
        batch_refs = {}
        if not args.no_extras or args.workload == "batch":
            for i in (24, 10, 23):       # the smallest deblurring, CT and travel-time problems
                batch_refs[i] = pool.apply_async(_oracle_batch_problem, (i, 80))
    else:
        batch_refs = {}

    import numpy as np
    import torch

    from paper_2606_18073_amd import sgks as G
    from workloads import make

    if args.workload == "batch":
        # the uneven batch on its own (for its profiles): one batched solve, then its
        # 32 plain solves
        b = bench_batch(G, torch, np, make, batch_refs, order=not args.no_order,
                        plain=not args.no_plain)
        if pool is not None:
            pool.close()
            pool.join()
        print(json.dumps({
            "metric": "sGKS problem-iterations/s of the batched solve", "value":
            b["batched_iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": b["problem_iterations"] / b["batched_iters_per_s"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": b["workload"]}, "batched_vs_plain": b}),
            flush=True)
        return

    P = make(args.workload, 0, "full")
    backward = args.workload == HEADLINE
    log(f"{P.name}: n={P.n} m={P.m} p={P.p} nnz(A)={P.A.nnz} k={P.k}")
    order = not args.no_order
    res = measure(G, torch, P, args.steps, args.warmup, backward=backward,
                  profile=not args.no_profile, graph=args.graph, autotune=args.autotune,
                  gradient=args.gradient, order=order)
    log(f"timed: {res['value']:.1f} iters/s, {res['ms_per_step']:.2f} ms per step")
    out = {
        "metric": "sGKS iters/s + SpMV/sketch HBM GB/s; batched & adjoint vs plain at equal rel err",
        "value": res["value"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generators; operators stored FP32, vectors and accumulation FP64)",
        "config": {
            "workload": describe(P),
            "operator_storage": P.dtype, "vectors": "f64",
            "k": P.k, "n": P.n, "m": P.m, "p": P.p, "s": P.s,
            "launch": "graph replay" if args.graph else "kernel by kernel",
            "gradient_form": args.gradient,
            "unknowns_order": "Morton curve per frame" if order else "row-major",
        },
        "paper_context": PAPER_CONTEXT,
    }
    for key in ("setup_ms_per_step", "iterate_only_iters_per_s", "launch_shapes",
                "forward_ms_per_step", "backward_ms_per_step", "roofline", "kernels", "phases",
                "spmv_sketch_GBps", "spmv_sketch_frac_of_hbm_peak", "spmv_sketch_kernels"):
        if key in res:
            out[key] = res[key]
    if backward:
        fwd = res["forward_ms_per_step"]
        out["adjoint_vs_plain"] = {
            "forward_ms": fwd, "backward_ms": res["backward_ms_per_step"],
            "forward_plus_backward_over_forward": res["ms_per_step"] / fwd,
            "forward_iters_per_s": P.k / (fwd * 1e-3),
        }
        try:
            out["adjoint_vs_plain"].update(adjoint_rel_err(G, np, P, res))
        except Exception as e:      # reported, never fatal to the measurement
            out["adjoint_vs_plain"]["rel_err_error"] = repr(e)
        if not args.no_total_adjoint:
            try:
                out["total_adjoint"] = total_adjoint_cost(G, torch, np, P, order)
            except Exception as e:      # reported, never fatal to the measurement
                out["total_adjoint"] = {"error": repr(e)}
    if not args.no_extras:
        sec = {}
        for name in ("deblur2d", "ct2d"):
            if name == args.workload:
                continue
            Q = make(name, 0, "full")
            r = measure(G, torch, Q, max(5, args.steps // 2), 1, backward=False,
                        profile=not args.no_profile, order=order)
            ent = {"workload": describe(Q), "value": r["value"], "unit": "iters/s",
                   "ms_per_step": r["ms_per_step"], "setup_ms_per_step": r["setup_ms_per_step"],
                   "iterate_only_iters_per_s": r["iterate_only_iters_per_s"]}
            for key in ("roofline", "spmv_sketch_GBps", "spmv_sketch_frac_of_hbm_peak"):
                if key in r:
                    ent[key] = r[key]
            if name == "deblur2d":
                ent["note"] = ("A and A^T (about 83 MB) stay in the 256 MB Infinity Cache: its "
                               "bandwidth figures are not HBM evidence")
            sec[name] = ent
            log(f"secondary {name}: {r['value']:.1f} iters/s")
        out["secondary"] = sec
        gk = {}
        for name in ("deblur2d", HEADLINE):
            Q = P if name == args.workload else make(name, 0, "full")
            gk[name] = bench_gks(G, torch, np, Q, order=order)
            log(f"gks vs sgks {name}: {gk[name]['sgks_speedup_per_expansion']:.2f}x per expansion")
        out["gks_vs_sgks"] = gk
        out["batched_vs_plain"] = bench_batch(G, torch, np, make, batch_refs, order=order)
        log("batched comparison done")
        out["paper_scale"] = bench_paper_scale(G, torch, make, order=order)
    if pool is not None:
        log("oracle on the host ...")
        xo, dt_full, it_full = full_ref.get()
        out["rel_err_vs_oracle"] = float(np.linalg.norm(res["x"] - xo) / np.linalg.norm(xo))
        out["rre_gpu"] = float(np.linalg.norm(res["x"] - P.x_true) / np.linalg.norm(P.x_true))
        out["rre_oracle"] = float(np.linalg.norm(xo - P.x_true) / np.linalg.norm(P.x_true))
        kk = args.cpu_sample_iters
        t0 = time.perf_counter()
        samples = pool.starmap(_oracle_sample, [(args.workload, kk)] * nwork)
        wall = time.perf_counter() - t0
        agg = sum(k / dt for k, dt in samples)
        out["cpu_baseline"] = {
            "value": agg, "unit": "iters/s", "cores": nwork, "kind": "oracle",
            "sample": (f"{nwork} concurrent processes, each one create + {kk} iterations of the "
                       f"same workload (FP64 numpy/scipy, one thread each; its sparse products "
                       f"are single-threaded), rate summed over the processes; "
                       f"{wall:.1f} s wall including generation"),
            "host": cores,
            "single_thread": {"value": it_full / dt_full, "unit": "iters/s", "cores": 1,
                              "sample": f"one complete oracle solve (create + {it_full} "
                                        f"iterations), {dt_full:.1f} s"},
        }
        pool.close()
        pool.join()
    print(json.dumps(out), flush=True)


def _stop_helper_processes():
    """The spawn pools start multiprocessing's resource-tracker process, which otherwise
    exits only after it notices that this process has ended; stop it and wait for it so
    that no process of the benchmark outlives the command."""
    import gc
    gc.collect()   # the pools' semaphores are unlinked and unregistered first
    try:
        from multiprocessing import resource_tracker
        resource_tracker._resource_tracker._stop()
    except Exception:
        pass


if __name__ == "__main__":
    try:
        main()
    finally:
        _stop_helper_processes()
