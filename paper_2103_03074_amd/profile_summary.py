"""Short text summaries of rocprofv3 CSV output for one bench configuration.

The profiled command is `bench.py ... --launch eager --calib-copy-mib N`: the
bench then brackets its timed steps with two plain device copies of N MiB
(read once, written once).  Only the dispatches between the two copies (the
timed steps) are summarised, so planning, autotuning, the slice-invariant
steps and every later pass are left out.

Inputs are the directories written by `rocprofv3 --output-format csv -d DIR`:

* one `--kernel-trace --stats` run: calls, total and average duration per
  kernel, written to `<out>_kernel_trace.txt`;
* one `--pmc FETCH_SIZE` run and one `--pmc WRITE_SIZE` run: the mean counter
  per dispatch of each kernel, turned into bytes by the factor that makes the
  same counter read the copies' known size (each bracketing copy is
  calibrated on its own and the two factors must agree within 5 %), written
  to `<out>_hbm_traffic.txt` and `.json`; with `--bench-json` (the bench's
  JSON line from the same configuration) each kernel's traffic is also shown
  against its algorithmic bytes per launch;
* optionally further `--pmc` runs (`--extra DIR`, repeatable), whose counters
  are averaged per dispatch of each kernel and tabulated in
  `<out>_counters.txt`.

With `--overlap` instead of the counter runs, one `--kernel-trace` run of
the bench on several lanes is summarised as concurrency: the timed window,
the summed kernel durations, the time at least one and at least two kernels
were running, and each kernel's average duration under overlap, written to
`<out>_lanes_overlap.txt`.

The JSON records the SHA-256 of the kernel source the counters were taken
with (`--source-sha-file`, written next to the CSV files by the profiling
commands), so a reader can tell when the figures are stale.

    python -m paper_2103_03074_amd.profile_summary --trace T --fetch F --write W \\
        --copy-mib 1024 --out profiles/c3_5x8_m16 --command "..."
"""

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

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
    n = n.replace("tn::", "").replace("(anonymous namespace)::", "").replace(" ", "")
    return n


def read_csv(directory, suffix):
    """Rows of the newest *suffix file under directory (one profiled process
    per directory; older files left by earlier runs are ignored)."""
    paths = glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)
    if not paths:
        raise SystemExit(f"no *{suffix} under {directory}")
    newest = max(paths, key=os.path.getmtime)
    with open(newest, newline="") as f:
        return list(csv.DictReader(f))


def col(row, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(f"none of {names} in {sorted(row)}")


def bracketed(dispatches, size_of):
    """Dispatches strictly between the two large bracketing copies.
    dispatches: list of (dispatch_id, kernel, payload) in any order;
    size_of(payload) ranks the copies (duration or counter value)."""
    dispatches = sorted(dispatches, key=lambda d: d[0])
    copies = [d for d in dispatches if d[1] == COPY_KERNEL]
    if len(copies) < 2:
        raise SystemExit("the bracketing copies are missing")
    big = max(size_of(d[2]) for d in copies)
    marks = [d for d in copies if size_of(d[2]) > 0.5 * big]
    if len(marks) != 2:
        raise SystemExit(f"expected two bracketing copies, found {len(marks)}")
    lo, hi = marks[0][0], marks[1][0]
    inner = [d for d in dispatches if lo < d[0] < hi and d[1] != COPY_KERNEL]
    return inner, marks


def trace_table(directory):
    ds = []
    for r in read_csv(directory, "kernel_trace.csv"):
        t0 = int(col(r, "Start_Timestamp"))
        t1 = int(col(r, "End_Timestamp"))
        ds.append((int(col(r, "Dispatch_Id")), short_name(col(r, "Kernel_Name")), (t1 - t0) / 1e3))
    inner, _ = bracketed(ds, lambda us: us)
    agg = collections.defaultdict(list)
    for _, k, us in inner:
        agg[k].append(us)
    total = sum(sum(v) for v in agg.values())
    rows = [{"kernel": k, "calls": len(v), "total_us": sum(v), "avg_us": sum(v) / len(v),
             "pct": 100.0 * sum(v) / total} for k, v in agg.items()]
    return sorted(rows, key=lambda r: -r["total_us"])


def overlap_summary(directory):
    """Concurrency of the bracketed dispatches: window, summed durations,
    time with >= 1 and >= 2 kernels running (us), and per-kernel averages."""
    ds = []
    for r in read_csv(directory, "kernel_trace.csv"):
        t0 = int(col(r, "Start_Timestamp"))
        t1 = int(col(r, "End_Timestamp"))
        ds.append((int(col(r, "Dispatch_Id")), short_name(col(r, "Kernel_Name")), (t0, t1)))
    inner, _ = bracketed(ds, lambda iv: iv[1] - iv[0])
    events = []
    for _, _, (t0, t1) in inner:
        events += [(t0, 1), (t1, -1)]
    events.sort()
    busy1 = busy2 = 0
    depth, last = 0, None
    for t, d in events:
        if last is not None and depth >= 1:
            busy1 += t - last
            if depth >= 2:
                busy2 += t - last
        depth += d
        last = t
    window = max(iv[1] for _, _, iv in inner) - min(iv[0] for _, _, iv in inner)
    total = sum(iv[1] - iv[0] for _, _, iv in inner)
    agg = collections.defaultdict(list)
    for _, k, (t0, t1) in inner:
        agg[k].append((t1 - t0) / 1e3)
    rows = sorted(({"kernel": k, "calls": len(v), "total_us": sum(v), "avg_us": sum(v) / len(v)}
                   for k, v in agg.items()), key=lambda r: -r["total_us"])
    return {"window_us": window / 1e3, "sum_us": total / 1e3, "busy1_us": busy1 / 1e3, "busy2_us": busy2 / 1e3,
            "dispatches": len(inner)}, rows


def counter_table(directory, copy_kib=None):
    """Per kernel: {counter: mean value per dispatch} over the bracketed
    dispatches, the dispatch count, and (when copy_kib is given) the factor of
    each counter that makes the bracketing copies read copy_kib."""
    per = collections.defaultdict(dict)   # dispatch id -> counter -> value
    name, grid = {}, {}
    for r in read_csv(directory, "counter_collection.csv"):
        d = int(col(r, "Dispatch_Id"))
        c = col(r, "Counter_Name")
        per[d][c] = per[d].get(c, 0.0) + float(col(r, "Counter_Value"))
        name[d] = short_name(col(r, "Kernel_Name"))
        grid[d] = int(col(r, "Grid_Size"))
    counters = sorted({c for v in per.values() for c in v})
    ds = [(d, name[d], (grid[d], per[d])) for d in per]
    # the bracketing copies are the copy dispatches with the largest grids
    inner, marks = bracketed(ds, lambda v: v[0])
    inner = [(d, k, v[1]) for d, k, v in inner]
    marks = [(d, k, v[1]) for d, k, v in marks]
    agg = collections.defaultdict(list)
    for _, k, v in inner:
        agg[k].append(v)
    means = {k: {c: sum(x.get(c, 0.0) for x in v) / len(v) for c in counters} for k, v in agg.items()}
    count = {k: len(v) for k, v in agg.items()}
    factors = {}
    if copy_kib:
        for c in counters:
            f = [copy_kib / m[2][c] for m in marks]
            if abs(f[0] - f[1]) > 0.05 * max(f):
                raise SystemExit(f"the two copies calibrate {c} differently: {f}")
            factors[c] = (sum(f) / 2, [m[2][c] for m in marks])
    return means, count, factors, counters


def bench_record(path):
    """Algorithmic bytes per launch of each kernel and the plan's complex
    multiply-adds per launch group, from the bench's JSON line."""
    if not path:
        return {}, None
    with open(path) as f:
        line = [ln for ln in f if ln.strip().startswith("{")][-1]
    rec = json.loads(line)
    main = rec.get("main", {})
    tab = main.get("kernels", {})
    return {k: v.get("alg_bytes_per_launch") for k, v in tab.items()}, main.get("complex_macs_per_launch_group")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--trace", default="")
    ap.add_argument("--fetch", default="")
    ap.add_argument("--write", default="")
    ap.add_argument("--overlap", default="", help="kernel-trace run of the bench on several lanes")
    ap.add_argument("--extra", action="append", default=[], help="further --pmc run directories")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--bench-json", default="")
    ap.add_argument("--out", required=True, help="output prefix")
    ap.add_argument("--command", default="", help="the profiling commands, recorded verbatim (' ;; ' separated)")
    ap.add_argument("--title", default="")
    ap.add_argument("--source-sha-file", default="",
                    help="sha256sum output for kernels.hip written on the profiled machine")
    args = ap.parse_args()
    cmd_lines = ["Commands:", ""] + ["    " + c for c in args.command.split(" ;; ") if c]
    if args.overlap:
        o, rows = overlap_summary(args.overlap)
        lines = [f"# Kernel concurrency, timed steps only: {args.title}", ""] + cmd_lines + [""]
        lines += [f"dispatches {o['dispatches']}; timed window {o['window_us']:.1f} us; summed kernel durations "
                  f"{o['sum_us']:.1f} us ({o['sum_us'] / o['window_us']:.2f}x the window); at least one kernel "
                  f"running {o['busy1_us']:.1f} us ({100 * o['busy1_us'] / o['window_us']:.1f} %); at least two "
                  f"{o['busy2_us']:.1f} us ({100 * o['busy2_us'] / o['window_us']:.1f} %).", "",
                  "Durations under overlap (two kernels share the GPU, so these are not kernel speeds):", "",
                  f"{'kernel':48s} {'calls':>7s} {'total us':>12s} {'avg us':>10s}"]
        for r in rows:
            if r["total_us"] < 1e-3 * o["sum_us"]:
                continue
            lines.append(f"{r['kernel'][:48]:48s} {r['calls']:7d} {r['total_us']:12.1f} {r['avg_us']:10.2f}")
        with open(args.out + "_lanes_overlap.txt", "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    if not (args.trace and args.fetch and args.write):
        raise SystemExit("--trace, --fetch and --write are required (or --overlap)")

    tr = trace_table(args.trace)
    lines = [f"# Kernel trace, timed steps only: {args.title}", ""] + cmd_lines
    lines += ["", f"{'kernel':48s} {'calls':>7s} {'total us':>12s} {'avg us':>10s} {'%':>6s}"]
    for r in tr:
        if r["pct"] < 0.05:
            continue
        lines.append(f"{r['kernel'][:48]:48s} {r['calls']:7d} {r['total_us']:12.1f} {r['avg_us']:10.2f} "
                     f"{r['pct']:6.2f}")
    with open(args.out + "_kernel_trace.txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))

    copy_kib = args.copy_mib * 1024.0
    fe, fe_n, fe_f, _ = counter_table(args.fetch, copy_kib)
    wr, _, wr_f, _ = counter_table(args.write, copy_kib)
    f_fac, f_raw = fe_f["FETCH_SIZE"]
    w_fac, w_raw = wr_f["WRITE_SIZE"]
    alg, plan_cmacs = bench_record(args.bench_json)
    sha = kernel_source_sha()
    if args.source_sha_file:
        with open(args.source_sha_file) as f:
            sha = f.read().split()[0]
    res = {"copy_mib": args.copy_mib, "fetch_factor": f_fac, "write_factor": w_fac,
           "kernels_source_sha256": sha, "plan_cmacs_per_launch_group": plan_cmacs, "kernels": {}}
    lines = [f"# HBM traffic per dispatch, timed steps only: {args.title}", ""] + cmd_lines
    lines += ["",
              f"Calibration: each of the two bracketing device copies of {args.copy_mib} MiB reads FETCH_SIZE "
              f"{f_raw[0]:.0f} / {f_raw[1]:.0f} KiB and WRITE_SIZE {w_raw[0]:.0f} / {w_raw[1]:.0f} KiB: "
              f"factors {f_fac:.3f} (fetch), {w_fac:.3f} (write).",
              "", f"{'kernel':48s} {'dispatches':>10s} {'fetch MiB':>10s} {'write MiB':>10s} {'HBM MiB':>10s}"
              f" {'alg MiB':>10s} {'ratio':>6s}"]
    for k in sorted(set(fe) & set(wr), key=lambda k: -(fe[k]["FETCH_SIZE"] + wr[k]["WRITE_SIZE"])):
        fb = fe[k]["FETCH_SIZE"] * f_fac * 1024.0
        wb = wr[k]["WRITE_SIZE"] * w_fac * 1024.0
        a = alg.get(k)
        res["kernels"][k] = {"dispatches": fe_n[k], "fetch_bytes": fb, "write_bytes": wb,
                             "hbm_bytes_per_launch": fb + wb, "algorithmic_bytes_per_launch": a}
        a_txt = f"{a / 2**20:10.2f} {(fb + wb) / a:6.2f}" if a else f"{'-':>10s} {'-':>6s}"
        lines.append(f"{k[:48]:48s} {fe_n[k]:10d} {fb / 2**20:10.2f} {wb / 2**20:10.2f} {(fb + wb) / 2**20:10.2f} "
                     + a_txt)
    with open(args.out + "_hbm_traffic.txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(args.out + "_hbm_traffic.json", "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    print("\n".join(lines))

    if args.extra:
        tabs = [counter_table(d) for d in args.extra]
        names = [c for t in tabs for c in t[3]]
        kernels = sorted({k for t in tabs for k in t[0]},
                         key=lambda k: -max(r["total_us"] for r in tr if r["kernel"] == k) if any(
                             r["kernel"] == k for r in tr) else 0)
        lines = [f"# Counters per dispatch (means), timed steps only: {args.title}", ""] + cmd_lines + [""]
        lines.append(f"{'kernel':40s} " + " ".join(f"{c[:22]:>22s}" for c in names))
        for k in kernels:
            vals = []
            for t in tabs:
                for c in t[3]:
                    v = t[0].get(k, {}).get(c)
                    vals.append(f"{v:22.4g}" if v is not None else f"{'-':>22s}")
            lines.append(f"{k[:40]:40s} " + " ".join(vals))
        with open(args.out + "_counters.txt", "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))


if __name__ == "__main__":
    main()
