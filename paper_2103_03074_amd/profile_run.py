"""Short run of the benchmark's launch sequence for profilers.

Plans the 40-qubit workload exactly as bench.py does (same seed, restarts,
slicing, autotuning), then contracts `--groups` launch groups (2^b slices
each) with the same kernels, plus one plain device-to-device copy of
`--copy-mib` MiB through torch.  Under `rocprofv3 --pmc FETCH_SIZE` (or
WRITE_SIZE) the copy's counter reading against its known size gives the
factor that turns the counter into HBM bytes.

    rocprofv3 --kernel-trace --stats -d DIR -- python3 -m paper_2103_03074_amd.profile_run
    rocprofv3 --pmc FETCH_SIZE -d DIR -- python3 -m paper_2103_03074_amd.profile_run --groups 2
"""

import argparse
import sys

SLICE_EDGES = {"c3_5x8_m16": 16, "c2_5x5_m16": 8}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="c3_5x8_m16")
    ap.add_argument("--prec", default="c64")
    ap.add_argument("--groups", type=int, default=8)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--restarts", type=int, default=16)
    ap.add_argument("--branch-merge", type=int, default=1)
    ap.add_argument("--tune-cache", default="", help="autotuner cache (read, and extended)")
    ap.add_argument("--events", action="store_true",
                    help="also time every step with the library's HIP events (as bench.py does) and print "
                         "the mean per launch of each device function")
    args = ap.parse_args()
    import torch
    import rqc
    from . import tn, runtime
    torch.cuda.set_device(0)
    w = rqc.workload(args.workload)
    p = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], prec=args.prec, restarts=args.restarts,
                n_slice_edges=SLICE_EDGES.get(args.workload, -1), seed=0, branch_merge=args.branch_merge)
    s = p.stats()
    ws = runtime.workspace(p)
    acc = runtime.accumulator(p)
    p.autotune(ws, acc, args.tune_cache or None, reps=5)
    acc.zero_()
    per = 2 ** s["batch_log2"]
    if args.events:
        p.set_profiling(True)
    p.contract_slices(ws, acc, 0, per * args.groups)
    if args.events:
        torch.cuda.synchronize()
        agg = {}
        for st in p.step_profile():
            a = agg.setdefault(st["kernel_name"], [0.0, 0])
            a[0] += st["total_ms"]
            a[1] += st["launches"]
        p.set_profiling(False)
        for name, (ms, n) in sorted(agg.items(), key=lambda kv: -kv[1][0]):
            if n:
                print(f"profile_run events: {name} launches {n} mean_us {1e3 * ms / n:.2f}", file=sys.stderr,
                      flush=True)
    n = args.copy_mib << 18                      # float32 elements
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"profile_run: {args.workload} {args.prec}, {args.groups} launch groups of {per} slices, "
          f"copy of {args.copy_mib} MiB", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
