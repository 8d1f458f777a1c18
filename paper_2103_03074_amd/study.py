"""Precision study on the 53-qubit, 20-cycle workload.

16 slice ids (--samples) are sampled (seed 2) out of the 2^k slices of the plan for the
54-site diagonal grid with 53 active qubits, 20 open and 33 fixed.  The same
tree and slicing are contracted in complex128 (the float64 recontraction),
complex64, split-FP16 and BF16.  For each form the study reports the
norm-relative error of the summed partial amplitudes against complex128, the
time per slice, and XEB of the partial sums with every probability scaled by
2^k / n_samples (partial sums over a sample are not amplitudes; the scaled
estimator is computed the same way for every form, so the XEB differences
measure precision only).

    python -m paper_2103_03074_amd.study --out result.json

With `--bighead` it instead times whole jobs (all slices, then the
amplitudes call) on the 40-qubit 5x8 / 16-cycle workload, complex64: the
single tree whose root carries the open legs through every slice, with the
2^16 slices of the benchmark and with the planner's own slicing, against the
big-head split (head slices summed into v_head over the cut legs, the tail
contracted once by the amplitudes call) with the planner's slicing, and the
big-head split of open qubits read off a contraction order of the closed
network (tn_choose_open_qubits).

    python -m paper_2103_03074_amd.study --bighead --out bighead.json
"""

import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print("[study]", *a, file=sys.stderr, flush=True)


def precision_study(n_samples=16, precs=("c128", "c64", "split_fp16", "bf16"), restarts=16):
    import torch
    import rqc
    from . import tn, runtime
    w = rqc.workload("c4_diag53_m20")
    # sampled slices are scattered over the 2^k ids: one slice per launch
    # group, so no sampled slice pays for the rest of a group
    base = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], restarts=restarts, seed=0, branch_merge=1,
                   batch_log2=0)
    ex = base.export()
    tree = list(zip(ex["lhs"], ex["rhs"]))
    sliced = [tuple(e) for e in ex["sliced"]]
    k = len(sliced)
    ids = [int(i) for i in rqc.sample_slice_ids(k, n_samples, seed=2)]
    weight = float(2.0 ** k / len(ids))
    out = {"n_qubits": w["circuit"].n_qubits, "n_open": len(w["open_q"]), "n_sliced": k,
           "n_samples": len(ids), "weight": weight, "forms": {}}
    amps = {}
    for prec in precs:
        p = tn.Plan(w["circuit"], w["open_q"], w["fixed_q"], w["bits"], tree=tree, sliced=sliced, prec=prec,
                    batch_log2=0)
        s = p.stats()
        ws = runtime.workspace(p)
        acc = runtime.accumulator(p)
        p.contract_slice_list(ws, acc, ids[:1])       # prepares the plan on the device
        torch.cuda.synchronize()
        acc.zero_()
        t0 = time.perf_counter()
        p.contract_slice_list(ws, acc, ids)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        a = torch.empty(2 << s["n_open"], dtype=torch.float64, device="cuda")
        p.amplitudes(acc, a, ws)
        x = tn.xeb(a, s["n_open"], w["circuit"].n_qubits, weight, ks=[1, 2 ** (s["n_open"] - 4)])
        amps[prec] = a.cpu().numpy().view(np.complex128)
        out["forms"][prec] = {"seconds_per_slice": dt / len(ids), "cmacs_per_slice": s["cmacs_per_slice"],
                              "TFLOP/s": 8.0 * s["cmacs_per_slice"] * len(ids) / dt / 1e12,
                              "F_unif_scaled": x["F_unif"], "F_self_scaled": x["F_self"],
                              "topk_xeb": x["topk"]}
        log(prec, out["forms"][prec])
        p.close()
    ref = amps.get("c128")
    if ref is not None:
        for prec in precs:
            d = amps[prec] - ref
            out["forms"][prec]["norm_rel_err_vs_c128"] = float(np.linalg.norm(d) / np.linalg.norm(ref))
            out["forms"][prec]["F_unif_delta_vs_c128"] = (out["forms"][prec]["F_unif_scaled"] -
                                                          out["forms"]["c128"]["F_unif_scaled"])
    return out


def bighead_study(restarts=16):
    import torch
    import rqc
    from . import tn, runtime
    w = rqc.workload("c3_5x8_m16")
    res = {}
    # the last mode opens the qubits read off a contraction order of the
    # closed network instead of the workload's region (another subspace of
    # the same circuit, same fixed-bit seed)
    oq, _ = tn.choose_open_qubits(w["circuit"], len(w["open_q"]), restarts=restarts, seed=0)
    fq = [q for q in range(w["circuit"].n_qubits) if q not in set(oq)]
    spaces = {"region": (w["open_q"], w["fixed_q"], w["bits"]), "order": (oq, fq, rqc.fixed_bits(len(fq), seed=1))}
    modes = (("single_tree_2^16_slices", "region", dict(n_slice_edges=16)),
             ("single_tree_planner_slicing", "region", dict()),
             ("bighead_planner_slicing", "region", dict(bighead=1)),
             ("bighead_open_qubits_from_order", "order", dict(bighead=1)))
    for mode, space, extra in modes:
        o_q, f_q, bits = spaces[space]
        t0 = time.perf_counter()
        p = tn.Plan(w["circuit"], o_q, f_q, bits, restarts=restarts, seed=0, branch_merge=1, **extra)
        t_plan = time.perf_counter() - t0
        ws = runtime.workspace(p)
        acc = runtime.accumulator(p)
        p.autotune(ws, acc, None, reps=5)          # also sets up the plan on the device
        s = p.stats()
        n = s["n_slices"]
        amps = torch.empty(2 << s["n_open"], dtype=torch.float64, device="cuda")
        p.amplitudes(acc, amps, ws)                # first tail call prepares the tail
        torch.cuda.synchronize()
        acc.zero_()
        t0 = time.perf_counter()
        p.contract_slices(ws, acc, 0, n)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p.amplitudes(acc, amps, ws)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x = tn.xeb(amps, s["n_open"], w["circuit"].n_qubits, 1.0, ks=[1])
        total = s["cmacs_invariant"] + n * s["cmacs_per_slice"] + s["cmacs_tail"]
        res[mode] = {"n_slices": n, "batch_log2": s["batch_log2"], "n_c": s["n_c"], "n_open": s["n_open"],
                     "largest_intermediate_log2": s["max_log2_size"], "plan_seconds": t_plan,
                     "cmacs_total": total, "cmacs_per_slice": s["cmacs_per_slice"], "cmacs_tail": s["cmacs_tail"],
                     "contract_seconds": t1 - t0, "amplitudes_call_ms": 1e3 * (t2 - t1),
                     "job_seconds": t2 - t0, "amplitudes_per_s": 2 ** s["n_open"] / (t2 - t0),
                     "TFLOP/s": 8.0 * n * s["cmacs_per_slice"] / (t1 - t0) / 1e12,
                     "F_self": x["F_self"], "F_unif": x["F_unif"]}
        log(mode, res[mode])
        p.close()
    res["bighead_open_qubits_from_order"]["open_qubits"] = [int(q) for q in oq]
    ref = res["single_tree_2^16_slices"]
    for mode, _, _ in modes:
        res[mode]["job_time_vs_single_tree_2^16"] = res[mode]["job_seconds"] / ref["job_seconds"]
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--samples", type=int, default=16)
    ap.add_argument("--bighead", action="store_true")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    res = bighead_study() if args.bighead else precision_study(args.samples)
    text = json.dumps(res)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")


if __name__ == "__main__":
    main()
