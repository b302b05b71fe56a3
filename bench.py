#!/usr/bin/env python3
"""Benchmark of the sGKS hot path on one MI355X.

A step is one complete solve of the 2D deblurring workload (256x256 image,
n = 65536, 9x9 Gaussian PSF as CSR with FP32 values, L = [Dx; Dy], s = 400,
k = 100): sgks_create (transposes, sketch of b, initial Krylov basis, QR
factors), k expansions, and x_k = W y written to device memory.  The inputs
(A, L, b) are resident in device memory before the timed region starts.

The timed region runs the production path, kernel-by-kernel launches on one
stream (--graph replays captured graphs of the expansion instead, which measured
slower).  A second, profiled pass runs the same
steps kernel by kernel, every launch carrying HIP events bound to the kernel
itself (its begin and end of execution, as a kernel trace reports them); kernel
durations from it give the roofline of the dominant kernel
(algorithmic bytes per launch / average launch time) and the SpMV+sketch
bandwidth.  Then the batched solve of the 32-problem uneven batch is compared
with its 32 plain solves, and the forward solve of the dynamic CT workload with
forward + backward.  Finally the FP64 CPU oracle is timed on a bounded sample of
the main workload.

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

# The paper's own timings, quoted as context only (another machine, another sketch,
# other test problems; not a target): Sec. 4.2.2, Exp. 3 (seismic travel-time
# tomography) and Sec. 4.3, Exp. 4 (dynamic CT), totals divided by the iteration count.
PAPER_CONTEXT = {
    "note": "context only: laptop CPU, MATLAB, FP64, SRTT sketch, other test problems",
    "hardware": "Intel Core i7-8750H @ 2.2 GHz, 128 GB RAM",
    "exp3_travel_time_n65536": {"sgks_total_s": 27, "iterations": 300, "iters_per_s": 11.1},
    "exp4_dynamic_ct_n655360": {"sgks_total_s": 33, "iterations": 400, "iters_per_s": 12.1},
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


def algorithmic_bytes(P, d_avg, form="maintained"):
    """Minimal HBM bytes per launch of each bulk kernel: CSR values and indices once,
    rowptrs once, vectors read and written once, the d columns of W (or H W) for the
    dense products, the hashed pattern (2 zeta bytes per entry) for the scatter."""
    vsz = 4 if P.dtype == "f32" else 8
    nnzA, nnzL = P.A.nnz, P.L.nnz
    m, n, p, s = P.m, P.n, P.p, P.s
    csr = (vsz + 4) * (nnzA + nnzL)
    out = {
        # z = A w, L w of the new column: CSR, w read; z written
        "spmv_new_column": csr + 4 * (m + 1) + 4 * (p + 1) + 8 * n + 8 * m + 8 * p,
        # sketch bins of z: z and the pattern read, partial bins written (counted once)
        "sketch_scatter": (8 + 2 * P.zeta) * (m + p) + 16 * s,
        # adjoint products: transposed CSR, (u, t) read, one n-vector written
        "adjoint": csr + 8 * (n + 1) + 8 * m + 8 * p + 8 * n,
    }
    if form == "maintained":
        # r = (H W) y - A^T b: d columns of H W and A^T b read, r written
        out["gemv"] = 8 * n * d_avg + 16 * n
    else:
        # x = W y: the d columns of W read, x written
        out["gemv"] = 8 * n * d_avg + 8 * n
        # u = A x - b, t = L x: CSR, x, b read; u, t written
        out["forward_Ax_Lx"] = csr + 4 * (m + 1) + 4 * (p + 1) + 8 * n + 8 * m + 8 * m + 8 * p
    return out


# the kernel each phase launches
def kernel_phases(form):
    return {
        "kb_forward": ["forward_Ax_Lx", "spmv_new_column"],
        "kb_adjoint": ["adjoint"],
        "kb_scatter": ["sketch_scatter"],
        "kb_gradient" if form == "maintained" else "kb_gemv": ["gemv"],
    }


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
    f = os.path.join(ROOT, "profiles", f"kernel_trace_{workload}_k100.txt")
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


def cpu_baseline(P, reps):
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import sgks_oracle as O
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for _ in range(reps):
            ref = O.sgks(P.A, P.L, P.b, P.mu, P.k, P.s, P.seed, zeta=P.zeta, ell=P.ell,
                         refine_steps=P.refine_steps)
        dt = time.perf_counter() - t0
    return ref, {"value": reps * P.k / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
                 "sample": f"{reps} complete solves (set-up + {P.k} iterations) of the same "
                           f"workload, FP64 numpy/scipy, 1 thread, {dt:.1f} s"}


def bulk_bytes_per_iteration(P, form="maintained"):
    """Algorithmic bytes of the bulk kernels of one expansion at the mean basis size."""
    d_avg = P.ell + (P.k - 1) / 2.0
    return sum(algorithmic_bytes(P, d_avg, form).values())


def bench_batch(G, torch, np, make):
    """The 32-problem uneven batch: one batched solve against the 32 plain solves."""
    Ps = make("batch", 0, "full")
    data = G.upload_batch(Ps)
    k = Ps[0].k
    # launch shapes autotuned per operator shape (the warm-up create tunes and
    # caches them; the timed batched and plain solves reuse the same choices)
    opts = dict(ell=Ps[0].ell, max_iters=k, zeta=Ps[0].zeta, autotune=True)
    # warm-up (module load, autotuning)
    B = G.SGKSBatch(data, **opts)
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
    for i, (A, L, b, mu, s, seed) in enumerate(data):
        torch.cuda.synchronize()
        u0 = time.perf_counter()
        S = G.SGKS(A, L, b, mu, s, seed, **opts)
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
    bulk = sum(bulk_bytes_per_iteration(P) for P in Ps)
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
        "bulk_algorithmic_GBps_batched": bulk * k / (t2 - t1) / 1e9,
        "equal_rel_err": "bitwise-identical x_k to the plain solves" if same else "MISMATCH",
        "bitwise_equal_to_plain": bool(same),
    }


def bench_adjoint(G, torch, np, make):
    """Forward solve vs forward + frozen-basis backward on the dynamic CT workload."""
    P = make("dynamic_ct", 0, "full")
    A, L, b = G.upload_problem(P)
    opts = dict(ell=P.ell, max_iters=P.k, zeta=P.zeta, refine_steps=P.refine_steps)
    xt = torch.as_tensor(P.x_true, device=b.device)
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, **opts)   # warm-up
    S.iterate(2)
    S.backward(2.0 * (S.solution() - xt))
    S.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, **opts)
    S.iterate(P.k)
    x = S.solution()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gx = 2.0 * (x - xt)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gb, gmu = S.backward(gx)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    rc, it = S.status()
    S.close()
    fwd, bwd = t1 - t0, t3 - t2
    return {
        "workload": (f"{P.name}: {P.meta.get('nt')} frames of {P.meta.get('N')}^2, n={P.n}, "
                     f"m={P.m}, p={P.p}, nnz(A)={P.A.nnz}, s={P.s}, k={P.k}; loss ||x_k - "
                     f"x_true||^2, gradients w.r.t. b and mu"),
        "forward_ms": 1e3 * fwd,
        "backward_ms": 1e3 * bwd,
        "forward_iters_per_s": it / fwd,
        "forward_plus_backward_over_forward": (fwd + bwd) / fwd,
        "equal_rel_err": "the forward x_k is the one the backward differentiates (same run)",
        "grad_mu": gmu,
        "status": [rc, it],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="deblur2d")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=8)
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the profiled pass (no per-phase times, no roofline)")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of captured graphs instead of kernel-by-kernel launches")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and adjoint comparisons")
    ap.add_argument("--gradient", choices=["maintained", "direct"], default="maintained",
                    help="gradient form of the expansion")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time its launch shapes at create (cached per shape)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(see the sharding design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_18073_amd import sgks as G
    from workloads import make

    P = make(args.workload, 0, "full")
    dev = torch.device("cuda:0")
    A, L, b = G.upload_problem(P)
    x = torch.empty(P.n, dtype=torch.float64, device=dev)

    def step(acc, prof):
        t0 = time.perf_counter()
        S = G.SGKS(A, L, b, P.mu, P.s, P.seed, ell=P.ell, max_iters=P.k, zeta=P.zeta,
                   refine_steps=P.refine_steps, graph=args.graph, autotune=args.autotune,
                   gradient=args.gradient)
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
        rc, it = S.status()
        S.close()
        acc["setup_s"] += t1 - t0
        assert rc == 0 and it == P.k, (rc, it)

    def fresh():
        return {"ms": [0.0] * G.PHASES, "n": [0] * G.PHASES, "setup_s": 0.0}

    for _ in range(args.warmup):
        step(fresh(), False)
    acc = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(acc, False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed region: {args.steps} steps in {wall:.3f} s")
    ms_per_step = 1e3 * wall / args.steps
    value = args.steps * P.k / wall
    iter_s = wall - acc["setup_s"]
    xg = x.cpu().numpy()

    out = {
        "metric": "sGKS iters/s + SpMV/sketch HBM GB/s; batched & adjoint vs plain at equal rel err",
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{P.name}: {P.meta.get('N')}x{P.meta.get('N')} image, n={P.n}, "
                         f"A 9x9 Gaussian PSF CSR nnz={P.A.nnz} ({P.dtype} values), "
                         f"L=[Dx;Dy] {P.p}x{P.n} nnz={P.L.nnz}, sparse-sign s={P.s} "
                         f"zeta={P.zeta}, k={P.k}, mu={P.mu}, ell={P.ell}; one step = "
                         f"create + {P.k} iterations + x_k"),
            "operator_storage": P.dtype,
            "vectors": "f64",
            "k": P.k, "n": P.n, "s": P.s,
            "launch": "graph replay (8 expansions per graph)" if args.graph else "kernel by kernel",
            "gradient_form": args.gradient,
        },
        "paper_context": PAPER_CONTEXT,
        "setup_ms_per_step": 1e3 * acc["setup_s"] / args.steps,
        "launch_shapes": acc.get("tuning"),
        "iterate_only_iters_per_s": args.steps * P.k / iter_s if iter_s > 0 else None,
    }
    if not args.no_profile:
        # profiled pass: the same steps kernel by kernel, each launch with HIP
        # events bound to the kernel (kernel durations do not depend on how the
        # launches were issued)
        pacc = fresh()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.steps):
            step(pacc, True)
        torch.cuda.synchronize()
        out["profiled_ms_per_step"] = 1e3 * (time.perf_counter() - p0) / args.steps
        log("profiled pass done")
        names = G.PHASE_NAMES
        phase = {names[i]: {"ms_total": pacc["ms"][i], "launches": pacc["n"][i],
                            "us_avg": (1e3 * pacc["ms"][i] / pacc["n"][i]) if pacc["n"][i] else None}
                 for i in range(G.PHASES) if pacc["n"][i]}
        out["phases"] = phase
        # average d over the dense launches: iterations use d = ell .. ell + k - 1,
        # the solution uses ell + k
        ds = list(range(P.ell, P.ell + P.k)) + [P.ell + P.k]
        ab = algorithmic_bytes(P, sum(ds) / len(ds), args.gradient)
        kern = {}
        for kname, phs in kernel_phases(args.gradient).items():
            ms = sum(phase[p]["ms_total"] for p in phs if p in phase)
            nl = sum(phase[p]["launches"] for p in phs if p in phase)
            by = sum(ab.get(p, 0.0) * phase[p]["launches"] for p in phs if p in phase)
            if nl:
                kern[kname] = {"ms_total": ms, "launches": nl, "us_avg": 1e3 * ms / nl,
                               "bytes_per_launch": by / nl, "GBps": by / (ms * 1e-3) / 1e9}
        out["kernels"] = kern
        dom = max(kern, key=lambda k: kern[k]["ms_total"])
        achieved = kern[dom]["GBps"]
        shash = source_hash()
        traffic = load_traffic(dom, P.name, shash)
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": traffic,
                           "algorithmic_bytes_per_launch": kern[dom]["bytes_per_launch"],
                           "avg_launch_us": kern[dom]["us_avg"], "source_hash": shash}
        # the same kernel in the committed kernel trace of the current sources
        tavg = load_trace_avg(dom, P.name, shash)
        if tavg:
            out["roofline"]["rocprof_avg_us"] = tavg
            out["roofline"]["achieved_at_rocprof_avg"] = kern[dom]["bytes_per_launch"] / (tavg * 1e-6) / 1e9
        # the launch with the most time: the compact append (side appends with the
        # H W adjoint beside them, then the stacked step) is bound by its chain of
        # dependent one-workgroup phases, not by HBM; its time and share are shown
        # with the HBM bytes its counters measured
        ap = phase.get("qr_append_solve")
        tuning = acc.get("tuning") or {}
        if ap and tuning.get("append_groups") == 1 and ap["launches"]:
            exp_ms = sum(v["ms_total"] for v in phase.values())
            name = "k_ap1_side_hw" if args.gradient == "maintained" else "k_ap1_side"
            tr = load_traffic(name, P.name, shash)
            out["append_launch"] = {
                "kernel": name, "bound": "latency", "avg_launch_us": ap["us_avg"],
                "share_of_kernel_time": ap["ms_total"] / exp_ms if exp_ms > 0 else None,
                "hbm_bytes_per_launch": tr,
                "GBps_at_hbm_bytes": tr / (ap["us_avg"] * 1e-6) / 1e9 if tr else None}
        sk = ["kb_forward", "kb_adjoint", "kb_scatter"]
        tb = sum(kern[k]["bytes_per_launch"] * kern[k]["launches"] for k in sk if k in kern)
        tt = sum(kern[k]["ms_total"] for k in sk if k in kern) * 1e-3
        out["spmv_sketch_GBps"] = tb / tt / 1e9 if tt > 0 else None
        out["spmv_sketch_frac_of_hbm_peak"] = out["spmv_sketch_GBps"] / HBM_PEAK_GBS
    if not args.no_extras:
        out["batched_vs_plain"] = bench_batch(G, torch, np, make)
        log("batched comparison done")
        out["adjoint_vs_plain"] = bench_adjoint(G, torch, np, make)
        log("adjoint comparison done")
    if not args.no_cpu_baseline:
        log("oracle on the host ...")
        ref, cb = cpu_baseline(P, args.cpu_reps)
        out["cpu_baseline"] = cb
        out["rel_err_vs_oracle"] = float(np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x))
        out["rre_gpu"] = float(np.linalg.norm(xg - P.x_true) / np.linalg.norm(P.x_true))
        out["rre_oracle"] = float(np.linalg.norm(ref.x - P.x_true) / np.linalg.norm(P.x_true))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
