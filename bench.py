#!/usr/bin/env python3
"""Throughput of the sliced big-head contraction on one MI355X.

Workload (default): the 40-qubit 5x8-grid random circuit, 16 cycles, 16 open
and 24 fixed qubits, sliced into 2^16 subtasks that run in launch groups of
2^8 slices.  Inputs are synthetic and seeded (circuit seed 0, fixed-bit seed
1) and resident on the GPU before any timed region.

One step is a fixed chunk of full launch groups (default 16 groups = 4096
slices) contracted through tn_contract_slices, which replays the captured
graph of a launch group; consecutive steps walk through the job's groups.
The groups of a step run on two concurrent lanes (tn_plan_set_lanes: two
HIP streams, each with its own workspace, graphs and float64 accumulator,
the lanes' sums added in lane order at the end of the call).
The value is TFLOP/s of the executed contraction tree over the timed steps
(8 real flops per complex multiply-add, Eq. (3) of the paper).  Whole-job
seconds and amplitudes/s are projected from the step time (all groups plus
the amplitudes call) and also measured on one full job outside the timed
loop, which supplies the amplitudes and the XEB figures.  The per-kernel
roofline record comes from a separate, untimed pass that launches a few
groups kernel by kernel with HIP events on the library's stream.

The complex64 form is the main line; the split-FP16 form is timed the same
way on the same workload (--compare) and reported beside it with its
speedup, its amplitude difference and its XEB difference.  The CPU oracle
(complex128) is timed on a bounded sample of slices of the same workload.
Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6, "split_fp16": 2500.0, "bf16": 2500.0}   # dense MFMA, MI355X
PEAK_HBM_GBS = 8000.0
METRIC = "sliced-contraction TFLOP/s (% MFMA peak) & amplitudes/s, mixed vs c64 plain"
# real MFMA products issued per complex multiply-add: 4 real products, times
# 3 hi/lo terms in the split-FP16 form
ISSUED_PER_CMAC = {"c64": 8.0, "c128": 8.0, "split_fp16": 24.0, "bf16": 8.0}

WORKLOAD_TEXT = {
    "c3_5x8_m16": "40-qubit 5x8 grid random circuit, 16 cycles (ABCDCDAB), 16 open / 24 fixed qubits, "
                  "2^16 slices",
    "c2_5x5_m16": "25-qubit 5x5 grid random circuit, 16 cycles, 10 open / 15 fixed qubits, 2^8 slices",
    "c1_tiny_3x4_m8": "12-qubit 3x4 grid random circuit, 8 cycles, 6 open / 6 fixed qubits, 2^2 slices",
}
SLICE_EDGES = {"c3_5x8_m16": 16, "c2_5x5_m16": 8, "c1_tiny_3x4_m8": 2}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_table(profile):
    """Per-step event timings aggregated by device function."""
    agg = {}
    for st in profile:
        name = st["kernel_name"] or "?"
        a = agg.setdefault(name, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
        a["ms"] += st["total_ms"]
        a["launches"] += st["launches"]
        a["flops"] += 8.0 * st["cmacs"] * st["launches"]
        a["bytes"] += st["bytes"] * st["launches"]
    return agg


def roofline_record(profile, prec, workload, cmacs_per_group):
    """Roofline record of the device function with the largest GPU time in
    the events pass: algorithmic flops (or bytes) per launch over its average
    launch duration, against the MFMA peak of the form (or HBM)."""
    agg = kernel_table(profile)
    name, a = max(agg.items(), key=lambda kv: kv[1]["ms"])
    n = max(1, a["launches"])
    avg_s = a["ms"] / 1e3 / n
    lowp = "_lp" in name
    peak_f = PEAK_TFLOPS[prec if lowp or prec in ("c64", "c128") else "c64"]
    ridge = peak_f * 1e12 / (PEAK_HBM_GBS * 1e9)
    ai = a["flops"] / max(a["bytes"], 1.0)
    if ai >= ridge:
        ach = a["flops"] / n / avg_s / 1e12
        rec = {"bound": "mfma", "achieved": ach, "peak": peak_f, "unit": "TFLOP/s", "frac": ach / peak_f}
    else:
        ach = a["bytes"] / n / avg_s / 1e9
        rec = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS}
    rec["traffic"] = measured_traffic(workload, prec, name, cmacs_per_group)
    rec.update({"kernel": name, "launches": a["launches"], "avg_launch_us": avg_s * 1e6,
                "algorithmic_flops_per_launch": a["flops"] / n, "algorithmic_bytes_per_launch": a["bytes"] / n,
                "arithmetic_intensity": ai,
                "share_of_gpu_time": a["ms"] / max(1e-12, sum(v["ms"] for v in agg.values()))})
    if lowp:
        issued = a["flops"] / 8.0 * ISSUED_PER_CMAC[prec] / n / avg_s / 1e12
        rec["issued_mfma_TFLOP/s"] = issued
        rec["issued_frac_of_peak"] = issued / peak_f
    table = {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                 "avg_us": round(v["ms"] * 1e3 / max(1, v["launches"]), 1),
                 "alg_bytes_per_launch": v["bytes"] / max(1, v["launches"]),
                 "alg_flops_per_launch": v["flops"] / max(1, v["launches"]),
                 "TFLOP/s": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                 "GB/s": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in agg.items()}
    return rec, table


def tree_roofline_fraction(profile, prec):
    """Sum over the profiled steps of t_min = max(flops / MFMA peak, bytes /
    HBM peak), over their summed measured time: the roofline fraction of the
    whole tree, skinny steps included.  Low-precision GEMM kernels count
    against the FP16/BF16 peak, everything else against the FP32 (FP64) peak."""
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


def measured_traffic(workload, prec, kernel, cmacs_per_group):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload and form (FETCH_SIZE + WRITE_SIZE, calibrated
    against a plain copy), or None when there is none, the kernel source has
    changed since the counters were taken, or the plan differs (its complex
    multiply-adds per launch group are recorded with the counters)."""
    import hashlib
    suffix = "" if prec == "c64" else f"_{prec}"
    path = os.path.join(ROOT, "profiles", f"{workload}{suffix}_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_2103_03074_amd", "csrc", "kernels.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("kernels_source_sha256") != sha or kernel not in rec.get("kernels", {}):
        return None
    if rec.get("plan_cmacs_per_launch_group") != cmacs_per_group:
        return None
    return rec["kernels"][kernel]["hbm_bytes_per_launch"]


def cpu_baseline(w, plan, budget_s=20.0):
    """The oracle (complex128 numpy contraction) on slices of the same
    workload, with the plan's tree as its schedule, projected to the whole
    job.  Sample: slice 0, then further slices while under the budget."""
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
    n_slices = 2 ** len(sliced)
    while True:
        sub = nw.slice_network(net, sliced, nw.slice_values(sliced, done))
        _, macs = nw.log2_sizes(sub.labels, tree)
        t0 = time.perf_counter()
        nw.contract(sub, tree)
        t_all += time.perf_counter() - t0
        macs_all += macs
        done += 1
        if t_all > budget_s or done >= min(n_slices, 1024):
            break
    t_slice = t_all / done
    amps = 2 ** len(w["open_q"])
    return {"value": 8.0 * macs_all / t_all / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"slices 0..{done - 1} of {n_slices}, complex128 numpy tensordot, plan tree as schedule, "
                      f"{t_all:.1f} s",
            "seconds_per_slice": t_slice,
            "projected_seconds_per_job": t_slice * n_slices,
            "amplitudes_per_s": amps / (t_slice * n_slices)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3_5x8_m16")
    ap.add_argument("--prec", default="c64")
    ap.add_argument("--compare", default="split_fp16",
                    help="second form timed on the same workload (\"\" for none)")
    ap.add_argument("--groups-per-step", type=int, default=16,
                    help="launch groups (2^batch_log2 slices each) per step")
    ap.add_argument("--events-groups", type=int, default=4,
                    help="launch groups of the untimed per-kernel events pass")
    ap.add_argument("--launch", choices=("graph", "eager"), default="graph",
                    help="eager: the timed steps launch kernel by kernel (for profilers)")
    ap.add_argument("--lanes", type=int, default=2,
                    help="concurrent lanes of launch groups (HIP streams) in each contraction call")
    ap.add_argument("--restarts", type=int, default=16)
    ap.add_argument("--batch-log2", type=int, default=-1)
    ap.add_argument("--branch-merge", type=int, default=1,
                    help="re-tune the tree for estimated time (merges small branches first)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2103_03074_amd", "tune", "gfx950.txt"),
                    help="autotune cache file (read, and extended with new decisions); the default is the "
                         "committed cache written by this bench on MI355X, so runs and profiles use the same "
                         "kernel per step shape (\"\" to re-tune every shape)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-full-job", action="store_true", help="skip the measured full job")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="bracket the timed steps of the main form with two plain device copies of this many "
                         "MiB, outside the timed region (markers and calibration for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported: slices are independent, "
              "so N GPUs would each take 1/N of the launch groups and one float64 reduction would "
              "combine the accumulators (not built here).", file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()
    if args.launch == "eager":
        os.environ["TN_NO_GRAPH"] = "1"   # read by the library at its first contraction call

    import torch
    import rqc
    from paper_2103_03074_amd import tn, runtime

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = rqc.workload(args.workload)
    n_qubits = w["circuit"].n_qubits

    def calib_copies(prec):
        if not args.calib_copy_mib or prec != args.prec:
            return lambda: None
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)

        def copy():
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
        return copy

    def run(prec):
        t0 = time.perf_counter()
        plan = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], prec=prec, restarts=args.restarts,
                       n_slice_edges=SLICE_EDGES.get(args.workload, -1), batch_log2=args.batch_log2, seed=0,
                       branch_merge=args.branch_merge)
        t_plan = time.perf_counter() - t0
        plan.set_lanes(args.lanes)
        s = plan.stats()
        log(f"{prec}: planned in {t_plan:.1f}s: {s['n_slices']} slices, 2^{s['batch_log2']} per launch group, "
            f"largest tensor 2^{s['max_log2_size']}, {args.lanes} lanes")
        ws = runtime.workspace(plan)
        acc = runtime.accumulator(plan)
        amps = torch.empty(2 << s["n_open"], dtype=torch.float64, device="cuda")
        n_tuned, t_tune = 0, 0.0
        if not args.no_autotune:
            t0 = time.perf_counter()
            n_tuned = plan.autotune(ws, acc, args.tune_cache or None, reps=5)
            t_tune = time.perf_counter() - t0
            log(f"{prec}: autotuned {n_tuned} step shapes in {t_tune:.1f}s")
            s = plan.stats()
        B = 1 << s["batch_log2"]
        n_groups = s["n_slices"] // B
        G = max(1, min(args.groups_per_step, n_groups))
        while n_groups % G:
            G -= 1
        acc.zero_()
        plan.contract_slices(ws, acc, 0, B)   # first call: leaves and slice-invariant subtrees
        torch.cuda.synchronize()

        cursor = [0]

        def step():
            g0 = cursor[0]
            plan.contract_slices(ws, acc, g0 * B, (g0 + G) * B)
            cursor[0] = (g0 + G) % n_groups

        for i in range(args.warmup):
            step()
        torch.cuda.synchronize()
        log(f"{prec}: {args.warmup} warm-up steps of {G} launch groups done")
        copy = calib_copies(prec)
        copy()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step()
            if (i + 1) % 5 == 0 or i + 1 == args.steps:
                torch.cuda.synchronize()
                log(f"{prec}: timed step {i + 1}/{args.steps}")
        torch.cuda.synchronize()
        sec_step = (time.perf_counter() - t0) / args.steps
        copy()

        # untimed events pass: kernel-by-kernel launches with per-step HIP
        # events on the library's stream
        E = max(1, min(args.events_groups, n_groups))
        plan.set_profiling(True)
        plan.contract_slices(ws, acc, 0, E * B)
        torch.cuda.synchronize()
        prof = plan.step_profile()
        plan.set_profiling(False)

        # one measured full job: all slices, amplitudes, XEB
        job = None
        if not args.no_full_job:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            acc.zero_()
            plan.contract_slices(ws, acc, 0, s["n_slices"])
            plan.amplitudes(acc, amps, ws)
            torch.cuda.synchronize()
            t_job = time.perf_counter() - t0
            t1 = time.perf_counter()
            xres = tn.xeb(amps, s["n_open"], n_qubits, 1.0, ks=[1, 2 ** max(0, s["n_open"] - 4)])
            t_xeb = time.perf_counter() - t1
            log(f"{prec}: full job {t_job:.2f}s")
            job = {"seconds": t_job, "xeb_seconds": t_xeb, "xeb": xres, "amps": amps.clone()}
        # amplitudes call alone (the tail with the big-head split; a copy otherwise)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.amplitudes(acc, amps, ws)
        torch.cuda.synchronize()
        t_amp = time.perf_counter() - t0
        cmacs_step = s["cmacs_per_batch"] * G
        out = {"plan": plan, "stats": s, "sec_step": sec_step, "groups_per_step": G, "n_groups": n_groups,
               "cmacs_step": cmacs_step, "prof": prof, "events_groups": E, "job": job, "t_amp": t_amp,
               "t_plan": t_plan, "t_tune": t_tune, "n_tuned": n_tuned}
        del ws, acc
        torch.cuda.empty_cache()
        return out

    def summarize(r, prec):
        s = r["stats"]
        tflops = 8.0 * r["cmacs_step"] / r["sec_step"] / 1e12
        proj_job = r["sec_step"] / r["groups_per_step"] * r["n_groups"] + r["t_amp"]
        roof, table = roofline_record(r["prof"], prec, args.workload, s["cmacs_per_batch"])
        d = {"ms_per_step": r["sec_step"] * 1e3, "TFLOP/s": tflops,
             "pct_of_form_mfma_peak": 100.0 * tflops / PEAK_TFLOPS[prec],
             "projected_seconds_per_job": proj_job,
             "projected_amplitudes_per_s": 2 ** s["n_open"] / proj_job,
             "roofline": roof, "roofline_fraction_tree": tree_roofline_fraction(r["prof"], prec),
             "kernels": table, "plan_seconds": r["t_plan"], "autotune_seconds": r["t_tune"],
             "autotuned_shapes": r["n_tuned"],
             "complex_macs_per_step": r["cmacs_step"],
             "complex_macs_per_launch_group": s["cmacs_per_batch"],
             "complex_macs_per_slice_unmerged_tree": s["cmacs_per_slice_unmerged"],
             "complex_macs_slice_invariant_once": s["cmacs_invariant"]}
        if prec in ("split_fp16", "bf16"):
            d["pct_fp16_mfma_peak_issued"] = 100.0 * tflops / 8.0 * ISSUED_PER_CMAC[prec] / PEAK_TFLOPS[prec]
        if r["job"]:
            d["measured_job_seconds"] = r["job"]["seconds"]
            d["measured_amplitudes_per_s"] = 2 ** s["n_open"] / r["job"]["seconds"]
            d["xeb"] = {k: r["job"]["xeb"][k] for k in ("F_unif", "F_self", "P_s1", "cond_xeb")}
            d["xeb"]["top_k"] = r["job"]["xeb"]["topk"]
        return d

    log(f"workload {args.workload}, main form {args.prec}, compare {args.compare or 'none'}, "
        f"launch {args.launch}")
    main_run = run(args.prec)
    s = main_run["stats"]
    m = summarize(main_run, args.prec)
    out = {
        "metric": METRIC, "value": m["TFLOP/s"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOAD_TEXT.get(args.workload, args.workload),
                   "n_slices": s["n_slices"], "slices_per_launch_group": 2 ** s["batch_log2"],
                   "launch_groups_per_step": main_run["groups_per_step"],
                   "slices_per_step": main_run["groups_per_step"] << s["batch_log2"],
                   "largest_intermediate_log2": s["max_log2_size"], "restarts": args.restarts,
                   "branch_merge": args.branch_merge,
                   "tune_cache": os.path.relpath(args.tune_cache, ROOT) if args.tune_cache else None,
                   "launch": "graph replay per launch group" if args.launch == "graph" else "eager",
                   "lanes": args.lanes,
                   "events_pass_groups": main_run["events_groups"]},
        "pct_mfma_peak": m["pct_of_form_mfma_peak"],
        "amplitudes_per_s": m.get("measured_amplitudes_per_s", m["projected_amplitudes_per_s"]),
        "amplitudes_per_s_kind": "measured full job" if main_run["job"] else "projected",
        "roofline": m.pop("roofline"),
        "main": m,
    }
    if args.compare:
        main_amps = main_run["job"].pop("amps") if main_run["job"] else None
        main_xeb = main_run["job"]["xeb"] if main_run["job"] else None
        cmp_run = run(args.compare)
        c = summarize(cmp_run, args.compare)
        c["dtype"] = args.compare
        c["speedup_vs_main_step"] = main_run["sec_step"] / cmp_run["sec_step"]
        if cmp_run["job"] and main_amps is not None:
            c["speedup_vs_main_job"] = main_run["job"]["seconds"] / cmp_run["job"]["seconds"]
            c["xeb_delta_vs_main"] = {k: cmp_run["job"]["xeb"][k] - main_xeb[k] for k in ("F_unif", "F_self")}
            diff = cmp_run["job"]["amps"] - main_amps
            c["amplitudes_norm_rel_diff_vs_main"] = float(torch.linalg.vector_norm(diff) /
                                                          torch.linalg.vector_norm(main_amps))
            ref_rms = float(torch.sqrt(torch.mean(main_amps.view(-1, 2).pow(2).sum(1))))
            c["amplitudes_max_abs_diff_over_rms_vs_main"] = float(diff.view(-1, 2).pow(2).sum(1).sqrt().max()) / ref_rms
        out["compare"] = c
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(w, main_run["plan"])
    out["bench_wall_seconds"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
