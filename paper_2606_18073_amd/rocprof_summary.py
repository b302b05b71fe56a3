"""Summaries of rocprofv3 output databases (SQLite, rocpd schema).

    python -m paper_2606_18073_amd.rocprof_summary stats DB OUT.txt --cmd "..."
        kernel-trace statistics (calls, total / average / min / max duration)
    python -m paper_2606_18073_amd.rocprof_summary traffic --fetch DB --write DB \\
        --calib-fetch DB --calib-write DB --kernel NAME --workload W --out JSON --cmd "..."
        HBM bytes per dispatch of one kernel from FETCH_SIZE / WRITE_SIZE counter runs,
        each scaled by what the same counter reads for a plain copy of known size

The summaries record the command that produced the database.
"""
import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _short(name):
    name = re.sub(r"\(.*", "", name).replace("void ", "").strip()
    return name


def kernel_stats(db):
    cur = sqlite3.connect(db).cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    ki = cols.index("name") if "name" in cols else cols.index("kernel_name")
    si, ei = cols.index("start"), cols.index("end")
    agg = {}
    for r in cur.execute("select * from kernels"):
        nm = _short(r[ki])
        dt = (r[ei] - r[si]) / 1e3
        a = agg.setdefault(nm, [0, 0.0, float("inf"), 0.0])
        a[0] += 1
        a[1] += dt
        a[2] = min(a[2], dt)
        a[3] = max(a[3], dt)
    return agg


def counter_per_dispatch(db, counter):
    """{kernel: [value per dispatch]} for one counter (summed over its instances)."""
    cur = sqlite3.connect(db).cursor()
    per = collections.defaultdict(float)
    names = {}
    for did, kn, cn, val in cur.execute(
            "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
        if cn != counter:
            continue
        per[did] += val
        names[did] = _short(kn)
    out = collections.defaultdict(list)
    for did, v in per.items():
        out[names[did]].append(v)
    return out


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_18073_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cmd_stats(args):
    agg = kernel_stats(args.db)
    tot = sum(v[1] for v in agg.values())
    lines = [f"# rocprofv3 kernel trace summary", f"# command: {args.cmd}",
             f"# source_hash: {source_hash()}",
             "%-58s %7s %12s %10s %10s %10s %6s" % ("kernel", "calls", "total_us", "avg_us",
                                                   "min_us", "max_us", "pct")]
    for nm, (c, t, mn, mx) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:args.top]:
        lines.append("%-58s %7d %12.1f %10.2f %10.2f %10.2f %6.2f" %
                     (nm[:58], c, t, t / c, mn, mx, 100 * t / tot))
    text = "\n".join(lines) + "\n"
    if args.out:
        open(args.out, "w").write(text)
    print(text)


def cmd_traffic(args):
    f = counter_per_dispatch(args.fetch, "FETCH_SIZE")
    w = counter_per_dispatch(args.write, "WRITE_SIZE")
    cf = counter_per_dispatch(args.calib_fetch, "FETCH_SIZE")
    cw = counter_per_dispatch(args.calib_write, "WRITE_SIZE")

    def pick(d, pat):
        ks = [k for k in d if pat in k]
        if not ks:
            raise SystemExit(f"no kernel matching {pat!r}: {sorted(d)[:20]}")
        return max(ks, key=lambda k: max(d[k]))

    kf, kw = pick(f, args.kernel), pick(w, args.kernel)
    copy_bytes = args.calib_bytes
    ccf, ccw = pick(cf, args.calib_kernel), pick(cw, args.calib_kernel)
    # the largest dispatches of the copy kernel are the calibration copies
    fetch_copy_kib = max(cf[ccf])
    write_copy_kib = max(cw[ccw])
    f_factor = copy_bytes / (fetch_copy_kib * 1024.0)
    w_factor = copy_bytes / (write_copy_kib * 1024.0)
    fetch_kib = sum(f[kf]) / len(f[kf])
    write_kib = sum(w[kw]) / len(w[kw])
    res = {
        "kernel": args.kernel, "workload": args.workload, "source_hash": source_hash(),
        "command": args.cmd,
        "fetch_kib_per_dispatch": fetch_kib, "write_kib_per_dispatch": write_kib,
        "dispatches": [len(f[kf]), len(w[kw])],
        "copy_calibration": {"kernel": ccf, "bytes": copy_bytes,
                             "fetch_kib": fetch_copy_kib, "write_kib": write_copy_kib,
                             "fetch_factor": f_factor, "write_factor": w_factor},
        "bytes_per_launch": fetch_kib * 1024.0 * f_factor + write_kib * 1024.0 * w_factor,
    }
    open(args.out, "w").write(json.dumps(res, indent=1) + "\n")
    print(json.dumps(res, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("db")
    a.add_argument("out", nargs="?")
    a.add_argument("--cmd", default="")
    a.add_argument("--top", type=int, default=30)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write", "kernel", "workload", "out"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--calib-kernel", default="copyBuffer")
    t.add_argument("--calib-bytes", type=float, default=512 * 2 ** 20)
    t.add_argument("--cmd", default="")
    args = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic}[args.what](args)


if __name__ == "__main__":
    main(sys.argv[1:])
