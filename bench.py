#!/usr/bin/env python3
"""Throughput of the sliced big-head contraction on one MI355X.

Workload (default): the 40-qubit 5x8-grid random circuit, 16 cycles, 16 open
and 24 fixed qubits, sliced into 2^16 subtasks.  One step is the whole job:
contract every slice (several slices per launch sequence), sum them in
float64, form the 2^16 amplitudes and compute XEB.  Inputs are synthetic and
seeded (circuit seed 0, fixed-bit seed 1) and resident on the GPU before the
timed region.

Prints one JSON line with TFLOP/s of the executed contraction tree (8 real
flops per complex multiply-add, Eq. (3) of the paper), its fraction of the
FP32 MFMA peak, amplitudes/s, the roofline record of the dominant kernel
(measured with HIP events inside the library over the timed steps) and the
CPU oracle timed on a bounded sample of the same workload.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6, "split_fp16": 2500.0, "bf16": 2500.0}   # dense MFMA, MI355X
PEAK_HBM_GBS = 8000.0
METRIC = "sliced-contraction TFLOP/s (% MFMA peak) & amplitudes/s, mixed vs c64 plain"

WORKLOAD_TEXT = {
    "c3_5x8_m16": "40-qubit 5x8 grid random circuit, 16 cycles (ABCDCDAB), 16 open / 24 fixed qubits, "
                  "2^16 slices, all contracted",
    "c2_5x5_m16": "25-qubit 5x5 grid random circuit, 16 cycles, 10 open / 15 fixed qubits, 2^8 slices",
}
SLICE_EDGES = {"c3_5x8_m16": 16, "c2_5x5_m16": 8, "c1_tiny_3x4_m8": 2}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def dominant_kernel(profile, prec):
    """Aggregate the per-step event timings by device function; return the
    roofline record of the function with the largest GPU time."""
    agg = {}
    for st in profile:
        name = st["kernel_name"] or "?"
        a = agg.setdefault(name, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
        a["ms"] += st["total_ms"]
        a["launches"] += st["launches"]
        a["flops"] += 8.0 * st["cmacs"] * st["launches"]
        a["bytes"] += st["bytes"] * st["launches"]
    name, a = max(agg.items(), key=lambda kv: kv[1]["ms"])
    sec = a["ms"] / 1e3
    peak_f = PEAK_TFLOPS[prec]
    ridge = peak_f * 1e12 / (PEAK_HBM_GBS * 1e9)
    ai = a["flops"] / max(a["bytes"], 1.0)
    if ai >= ridge:
        ach = a["flops"] / sec / 1e12
        rec = {"bound": "mfma", "achieved": ach, "peak": peak_f, "unit": "TFLOP/s", "frac": ach / peak_f}
    else:
        ach = a["bytes"] / sec / 1e9
        rec = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS}
    rec.update({"kernel": name, "launches": a["launches"], "avg_launch_us": a["ms"] * 1e3 / max(1, a["launches"]),
                "bytes_per_launch": a["bytes"] / max(1, a["launches"]),
                "share_of_gpu_time": a["ms"] / max(1e-12, sum(v["ms"] for v in agg.values())),
                "traffic": None})
    table = {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                 "TFLOP/s": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                 "GB/s": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in agg.items()}
    return rec, table


def tree_roofline_fraction(profile, prec):
    """Sum over the timed steps of t_min = max(flops / MFMA peak, bytes / HBM
    peak), over their summed measured time: the roofline fraction of the whole
    tree, skinny steps included.  Low-precision GEMM kernels count against the
    FP16/BF16 peak, everything else against the peak of the storage form."""
    t_min = t_meas = 0.0
    for st in profile:
        if not st["launches"]:
            continue
        name = st["kernel_name"] or ""
        peak = PEAK_TFLOPS["split_fp16"] if "_lp" in name else PEAK_TFLOPS["c128" if prec == "c128" else "c64"]
        per = max(8.0 * st["cmacs"] / (peak * 1e12), st["bytes"] / (PEAK_HBM_GBS * 1e9))
        t_min += per * st["launches"]
        t_meas += st["total_ms"] / 1e3
    return t_min / t_meas if t_meas > 0 else None


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE + WRITE_SIZE, calibrated against a
    plain copy), or None when there is none or the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_2103_03074_amd", "csrc", "kernels.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("kernels_source_sha256") != sha or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]["hbm_bytes_per_launch"]


def cpu_baseline(w, plan, budget_s=30.0):
    """The oracle (complex128 numpy contraction) on one slice of the same
    workload, with the plan's tree as its schedule; projected to the whole
    job.  Sample: slice 0 (and more slices while under the time budget)."""
    import numpy as np
    from oracle import network as nw
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    ex = plan.export()
    sliced = [tuple(e) for e in ex["sliced"]]
    tree = list(zip(ex["lhs"], ex["rhs"]))
    net = nw.build_network(w["circuit"], w["open_q"], w["fixed_q"], w["bits"])
    done, t_all, macs_all = 0, 0.0, 0.0
    while True:
        sub = nw.slice_network(net, sliced, nw.slice_values(sliced, done))
        _, macs = nw.log2_sizes(sub.labels, tree)
        t0 = time.perf_counter()
        nw.contract(sub, tree)
        t_all += time.perf_counter() - t0
        macs_all += macs
        done += 1
        if t_all > budget_s / 3 or done >= 4:
            break
    n_slices = 2 ** len(sliced)
    t_slice = t_all / done
    amps = 2 ** len(w["open_q"])
    return {"value": 8.0 * macs_all / t_all / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{done} slice(s) of {n_slices}, complex128 numpy tensordot, plan tree as schedule",
            "seconds_per_slice": t_slice,
            "amplitudes_per_s": amps / (t_slice * n_slices)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_5x8_m16")
    ap.add_argument("--prec", default="c64")
    ap.add_argument("--compare", default="split_fp16",
                    help="second precision timed on the same workload (\"\" for none)")
    ap.add_argument("--restarts", type=int, default=16)
    ap.add_argument("--batch-log2", type=int, default=-1)
    ap.add_argument("--branch-merge", type=int, default=1,
                    help="re-tune the tree for estimated time (merges small branches first)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported: slices are independent, "
              "so N GPUs would each take 1/N of the slice range and one float64 reduction would "
              "combine the accumulators (not built here).", file=sys.stderr)
        sys.exit(2)

    import torch
    import rqc
    from paper_2103_03074_amd import tn, runtime

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = rqc.workload(args.workload)

    def make(prec):
        t0 = time.perf_counter()
        p = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], prec=prec, restarts=args.restarts,
                    n_slice_edges=SLICE_EDGES.get(args.workload, -1), batch_log2=args.batch_log2, seed=0,
                    branch_merge=args.branch_merge)
        return p, time.perf_counter() - t0

    def run(prec, steps, warmup, profile):
        plan, t_plan = make(prec)
        s = plan.stats()
        ws = runtime.workspace(plan)
        acc = runtime.accumulator(plan)
        amps = torch.empty(2 << s["n_open"], dtype=torch.float64, device="cuda")
        n_tuned = 0
        if not args.no_autotune:
            t0 = time.perf_counter()
            n_tuned = plan.autotune(ws, acc, None, reps=5)
            log(f"{prec}: autotuned {n_tuned} step shapes in {time.perf_counter() - t0:.1f}s")
            s = plan.stats()
        n = s["n_slices"]
        xres = None

        def step():
            nonlocal xres
            acc.zero_()
            plan.contract_slices(ws, acc, 0, n)
            plan.amplitudes(acc, amps, ws)
            xres = tn.xeb(amps, s["n_open"], w["circuit"].n_qubits, 1.0, ks=[1, 2 ** (s["n_open"] - 4)])

        t0 = time.perf_counter()
        for i in range(warmup):
            step()
            log(f"{prec} warmup step {i} done")
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t0
        if profile:
            plan.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step()
            log(f"{prec} timed step {i} done")
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        prof = plan.step_profile() if profile else None
        if profile:
            plan.set_profiling(False)
        cmacs = s["cmacs_per_batch"] * (n >> s["batch_log2"])
        unmerged = s["cmacs_per_slice_unmerged"] * n + s["cmacs_invariant"]
        return {"plan": plan, "stats": s, "sec": dt, "cmacs": cmacs, "unmerged": unmerged, "prof": prof, "xeb": xres,
                "t_plan": t_plan, "t_warm": t_warm, "n_tuned": n_tuned, "amps": amps.clone()}

    log(f"workload {args.workload}, precision {args.prec}")
    main_run = run(args.prec, args.steps, args.warmup, True)
    s = main_run["stats"]
    sec = main_run["sec"]
    tflops = 8.0 * main_run["cmacs"] / sec / 1e12
    amps_per_s = 2 ** s["n_open"] / sec
    roof, table = dominant_kernel(main_run["prof"], args.prec)
    roof["traffic"] = measured_traffic(args.workload, roof["kernel"])
    roof["algorithmic_bytes_per_launch"] = roof.pop("bytes_per_launch")
    out = {
        "metric": METRIC, "value": tflops, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOAD_TEXT.get(args.workload, args.workload),
                   "n_slices": s["n_slices"], "slices_per_launch_sequence": 2 ** s["batch_log2"],
                   "largest_intermediate_log2": s["max_log2_size"], "restarts": args.restarts,
                   "autotuned_shapes": main_run["n_tuned"], "branch_merge": args.branch_merge, "launch": "eager with per-step HIP events"},
        "pct_mfma_peak": 100.0 * tflops / PEAK_TFLOPS[args.prec],
        "amplitudes_per_s": amps_per_s,
        "complex_macs_per_step": main_run["cmacs"],
        "complex_macs_per_step_unmerged_tree": main_run["unmerged"],
        "roofline_fraction_tree": tree_roofline_fraction(main_run["prof"], args.prec),
        "xeb": {k: main_run["xeb"][k] for k in ("F_unif", "F_self", "P_s1", "cond_xeb")},
        "roofline": roof,
        "kernels": table,
        "plan_seconds": main_run["t_plan"],
    }
    if args.compare:
        cmp_run = run(args.compare, args.steps, args.warmup, True)
        out["compare"] = {"dtype": args.compare, "ms_per_step": cmp_run["sec"] * 1e3,
                          "TFLOP/s": 8.0 * cmp_run["cmacs"] / cmp_run["sec"] / 1e12,
                          "amplitudes_per_s": 2 ** s["n_open"] / cmp_run["sec"],
                          "speedup_vs_main": sec / cmp_run["sec"],
                          "roofline_fraction_tree": tree_roofline_fraction(cmp_run["prof"], args.compare),
                          "dominant_kernel": dominant_kernel(cmp_run["prof"], args.compare)[0],
                          "xeb": {k: cmp_run["xeb"][k] for k in ("F_unif", "F_self")},
                          "xeb_delta_vs_main": {k: cmp_run["xeb"][k] - main_run["xeb"][k] for k in ("F_unif", "F_self")},
                          "amplitudes_norm_rel_diff_vs_main": float(torch.linalg.vector_norm(cmp_run["amps"] - main_run["amps"]) /
                                                                    torch.linalg.vector_norm(main_run["amps"]))}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(w, main_run["plan"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
