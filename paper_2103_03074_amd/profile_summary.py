"""Short text summaries of rocprofv3 databases (rocpd SQLite output).

Three runs of `profile_run` feed it: one with `--kernel-trace --stats`, one
with `--pmc FETCH_SIZE` and one with `--pmc WRITE_SIZE`.  It writes

* `<out>_kernel_trace.txt`: calls, total and average duration per kernel;
* `<out>_hbm_traffic.txt` and `.json`: FETCH_SIZE and WRITE_SIZE per
  dispatch, averaged per kernel, each turned into bytes with the factor that
  makes the same counter read the known size of the plain device copy the
  profiling driver ends with (`--copy-mib`, read once and written once).

The JSON records the SHA-256 of the kernel source the counters were taken
with (`--source-sha-file`, written next to the databases by the profiling
commands), so a reader can tell when the figures are stale.

    python -m paper_2103_03074_amd.profile_summary --trace T.db --fetch F.db --write W.db \\
        --copy-mib 1024 --out profiles/c3_5x8_m16 --command "..."
"""

import argparse
import collections
import hashlib
import json
import os
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_source_sha():
    h = hashlib.sha256()
    with open(os.path.join(HERE, "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def short_name(name):
    """Device function name without namespace, argument list or vector-type noise."""
    n = name.replace("HIP_vector_type<float, 2u>", "float2").replace("HIP_vector_type<double, 2u>", "double2")
    if n.startswith("void "):
        n = n[5:]
    if "(" in n:
        n = n[:n.index("(")]
    n = n.replace("tn::", "").replace(" ", "")
    return n


def trace_table(db):
    c = sqlite3.connect(db)
    rows = c.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                     "order by total_duration desc").fetchall()
    c.close()
    # the view reports microseconds
    return [{"kernel": short_name(r[0]), "calls": int(r[1]), "total_us": float(r[2]),
             "avg_us": float(r[3]), "pct": float(r[4])} for r in rows]


def counter_means(db, counter):
    """Mean counter value (KiB) per dispatch, per kernel."""
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, value from counters_collection where counter_name = ?",
                     (counter,)).fetchall()
    c.close()
    agg = collections.defaultdict(list)
    for name, v in rows:
        agg[short_name(name)].append(float(v))
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--out", required=True, help="output prefix")
    ap.add_argument("--command", default="", help="the profiling commands, recorded verbatim")
    ap.add_argument("--title", default="")
    ap.add_argument("--source-sha-file", default="",
                    help="sha256sum output for kernels.hip written on the profiled machine")
    args = ap.parse_args()

    tr = trace_table(args.trace)
    lines = [f"# {args.title or 'kernel trace'}", "", "Commands:", ""]
    lines += ["    " + c for c in args.command.split(" ;; ") if c]
    lines += ["", f"{'kernel':48s} {'calls':>7s} {'total us':>12s} {'avg us':>10s} {'%':>6s}"]
    for r in tr:
        if r["pct"] < 0.05 and r["kernel"] != COPY_KERNEL:
            continue
        lines.append(f"{r['kernel'][:48]:48s} {r['calls']:7d} {r['total_us']:12.1f} {r['avg_us']:10.2f} "
                     f"{r['pct']:6.2f}")
    with open(args.out + "_kernel_trace.txt", "w") as f:
        f.write("\n".join(lines) + "\n")

    fe = counter_means(args.fetch, "FETCH_SIZE")
    wr = counter_means(args.write, "WRITE_SIZE")
    copy_kib = args.copy_mib * 1024.0
    if COPY_KERNEL not in fe or COPY_KERNEL not in wr:
        raise SystemExit("the calibration copy is missing from the counter runs")
    f_fac = copy_kib / fe[COPY_KERNEL][0]
    w_fac = copy_kib / wr[COPY_KERNEL][0]
    sha = kernel_source_sha()
    if args.source_sha_file:
        with open(args.source_sha_file) as f:
            sha = f.read().split()[0]
    res = {"copy_mib": args.copy_mib, "fetch_factor": f_fac, "write_factor": w_fac,
           "kernels_source_sha256": sha, "kernels": {}}
    lines = [f"# HBM traffic per dispatch: {args.title}", "", "Commands:", ""]
    lines += ["    " + c for c in args.command.split(" ;; ") if c]
    lines += ["",
              f"Calibration: a device copy of {args.copy_mib} MiB reads FETCH_SIZE {fe[COPY_KERNEL][0]:.0f} KiB "
              f"and WRITE_SIZE {wr[COPY_KERNEL][0]:.0f} KiB: factors {f_fac:.3f} (fetch), {w_fac:.3f} (write).",
              "", f"{'kernel':48s} {'dispatches':>10s} {'fetch MiB':>10s} {'write MiB':>10s} {'HBM MiB':>10s}"]
    for k in sorted(set(fe) & set(wr), key=lambda k: -(fe[k][0] * f_fac + wr[k][0] * w_fac)):
        fb = fe[k][0] * f_fac * 1024.0
        wb = wr[k][0] * w_fac * 1024.0
        res["kernels"][k] = {"dispatches": fe[k][1], "fetch_bytes": fb, "write_bytes": wb,
                             "hbm_bytes_per_launch": fb + wb}
        lines.append(f"{k[:48]:48s} {fe[k][1]:10d} {fb / 2**20:10.2f} {wb / 2**20:10.2f} {(fb + wb) / 2**20:10.2f}")
    with open(args.out + "_hbm_traffic.txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(args.out + "_hbm_traffic.json", "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
